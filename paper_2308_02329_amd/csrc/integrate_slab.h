// Streamed-J CHYM integrator for large N (gfx950).
//
// One block of W wavefronts (eight: two per SIMD; sixteen, four per SIMD
// with half the registers, for few row tiles) owns a column slab -- 16
// replicas x D components of one problem -- for the whole run.  Row tiles (16 rows) are dealt to the
// wavefronts round-robin: wavefront w owns tiles w, w+W, ...,
// whose float32 state lives in its registers in the 16x16 MFMA accumulator
// layout (lane j + 16 g holds rows 16 I + 4 g + v of replica j).
//
// The contraction G = J X (paper: C = J_N (x) 1_D, Eq. (1)-(2)) runs on
// v_mfma_f32_16x16x32_bf16.  The state's bf16 operand (one term, or the
// three exact terms of the float32 form) lives in LDS in B-fragment order;
// each tile's owner writes it after every step and every wavefront reads all
// of it.  K-chunk c is made of row tiles 2c and 2c+1 in the order the
// accumulator layout already uses (slot s of lane (j, g) is row
// 16 (2c + s/4) + 4 g + s%4), the same permutation as the register-resident
// kernel, so the two kernels accumulate every G in the same order and give
// identical results.  J is staged once per problem into the caller's
// workspace as A fragments in that order and is streamed from L2 every step
// (at this size it does not fit in LDS).  In batches, J is staged narrower
// where that is exact, and widened to bf16 in registers: couplings in
// {-1, 0, +1} (in any storage) as four-bit E2M1 codes
// (v_cvt_scalef32_pk_bf16_fp4), otherwise, when every row of J is a set of
// E4M3 values times one power of two (FP8 storage always), as one E4M3 byte
// per coupling (v_cvt_scalef32_pk_bf16_fp8).  This cuts the L2 footprint
// and the HBM traffic of the many distinct couplings a batch streams at once
// (a quarter, or half, of the bf16 bytes).  A single problem's J stays bf16
// (k_integrate_slab).
//
// Per step: for each group of owned tiles (one to eight, by block size and
// D), accumulate G over all chunks (the J fragments of the next chunk are
// fetched while the current chunk's matrix-core work runs), then apply the
// fused Euler update to those tiles in registers; after a barrier every
// wavefront writes its tiles' new operand terms to LDS, and a second barrier
// publishes them.
//
// Component passes (the float32 form at large N, whose three-term operand of
// all D components exceeds LDS): LDS holds one component's operand, and a
// step makes D passes over the J stream, one per component.  The update of a
// hyperspin needs only its own component's G and the norm of its old state,
// so the norm-dependent coefficient is formed from the old state at the start
// of the step, each pass updates its component as soon as its G is complete,
// and the later passes still write operands of their components' old values.
// Every accumulator takes the same products in the same order and the update
// is the same arithmetic, so the results equal those of the one-pass form.
#pragma once

#include "integrate_kernel.h"

namespace chym {

// Staged couplings of one problem (caller workspace, 256-byte aligned):
//   [0, 256)           header: int32 format, kStageBf16, kStageE4M3 or kStageE2M1
//   [256, 256 + S)     float row scales 2^e_p [tiles * 16] (E4M3 fragments)
//   [256 + S, ...)     fragments: bf16 [tile][chunk][JS][64 lanes] x 16 B,
//                      E4M3 [tile][chunk][64 lanes] x 8 B, or
//                      E2M1 [tile][chunk][64 lanes] x 4 B
constexpr size_t kStageHeader = 256;
constexpr int kStageBf16 = 0;
constexpr int kStageE4M3 = 1;
constexpr int kStageE2M1 = 2;  // couplings in {-1, 0, +1}
// the most chunks of J fragments the streamed-J kernel keeps in flight (its
// prefetch ring); the staging carries that many chunks of padding after the
// last tile
constexpr int kSlabRingChunks = 4;
__host__ __device__ inline size_t stage_scale_bytes(int tiles) { return ((size_t)tiles * 64 + 255) / 256 * 256; }
__host__ __device__ inline size_t stage_frag_offset(int tiles) { return kStageHeader + stage_scale_bytes(tiles); }

// Buffer resource over n bytes at p (raw, 32-bit data format): loads through
// it take a per-lane offset and a wave-uniform offset, and return 0 past n.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_over(const void *p, uint32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, 0x00020000);
}

__device__ __forceinline__ bf16x8 load_frag16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef __attribute__((ext_vector_type(4))) int i4;
    const i4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ uint2 load_frag8(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef __attribute__((ext_vector_type(2))) int i2;
    const i2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return uint2{(uint32_t)v.x, (uint32_t)v.y};
}

__device__ __forceinline__ uint32_t load_frag4(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

// Eight E2M1 codes (slot s in nibble s: byte s / 2, low nibble first) as
// bf16; the instruction widens byte b into slots 2b (low nibble), 2b + 1.
__device__ __forceinline__ bf16x8 fp4_fragment(uint32_t w) {
    const bf16x2 a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 0);
    const bf16x2 b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 1);
    const bf16x2 c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 2);
    const bf16x2 d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 3);
    const auto ab = __builtin_shufflevector(a, b, 0, 1, 2, 3);
    const auto cd = __builtin_shufflevector(c, d, 0, 1, 2, 3);
    return __builtin_shufflevector(ab, cd, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Eight E4M3 codes (slots 0..7 in byte order) times a power of two, as bf16.
__device__ __forceinline__ bf16x8 fp8_fragment(uint2 w, float scale) {
    const bf16x2 a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.x, scale, false);
    const bf16x2 b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.x, scale, true);
    const bf16x2 c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.y, scale, false);
    const bf16x2 d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.y, scale, true);
    const auto ab = __builtin_shufflevector(a, b, 0, 1, 2, 3);
    const auto cd = __builtin_shufflevector(c, d, 0, 1, 2, 3);
    return __builtin_shufflevector(ab, cd, 0, 1, 2, 3, 4, 5, 6, 7);
}

// LDS operand layout: [chunk][component][term][64 lanes] of bf16x8 (1 KB
// each); D components, or one in the component-pass form.
__device__ __forceinline__ int slab_b_index(int c, int mu, int t, int lane, int D, int XS) {
    return ((c * D + mu) * XS + t) * 64 + lane;
}

// Writes the operand terms of one component of tile I (its four rows of this
// lane, v) into the half (I & 1) of the fragments lb[f0 + 64 q], q < XS.
template <int XS>
__device__ __forceinline__ void slab_write_comp(const float (&v)[4], int I, int f0, bf16x8 *lb) {
    typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
    bf16x2 t[XS][2];
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
        const float a = v[2 * pr], b = v[2 * pr + 1];
        const bf16x2 h = pack_rne(a, b);
        t[0][pr] = h;
        if constexpr (XS == 3) {
            const float ra = resid_lo(h, a), rb = resid_hi(h, b);
            const bf16x2 m = pack_rne(ra, rb);
            const float sa = resid_lo(m, ra), sb = resid_hi(m, rb);
            t[1][pr] = m;
            t[2][pr] = pack_rne(sa, sb);
        }
    }
#pragma unroll
    for (int q = 0; q < XS; ++q) {
        bf16x4 *dst = reinterpret_cast<bf16x4 *>(lb + f0 + 64 * q) + (I & 1);
        *dst = __builtin_shufflevector(t[q][0], t[q][1], 0, 1, 2, 3);
    }
}

// Writes the operand terms of every component of tile I into chunk I >> 1.
template <int D, int XS>
__device__ __forceinline__ void slab_write_tile(const float (&xt)[D][4], int I, int lane, bf16x8 *lb) {
#pragma unroll
    for (int mu = 0; mu < D; ++mu) slab_write_comp<XS>(xt[mu], I, slab_b_index(I >> 1, mu, 0, lane, D, XS), lb);
}

// Integrates the column slab rep0 .. rep0+15 of problem a.  stage: the
// staged couplings (layout above); FMT: the fragments' format (kStage*); ncp:
// chunk count of the staging; lb: LDS operand area of ncp * D * XS
// fragments.  Called by all W wavefronts of the block; contains block
// barriers.
//
// The J fragments a wavefront needs form one fixed sequence per step: its
// tile groups in order, each group's chunks in order.  They are read as one
// continuous stream, RD chunks ahead through a ring of registers: the slot
// of chunk c is c % RD (every group starts at slot 0), and the load that
// refills a slot after its chunk is taken fetches the next chunk of the same
// slot, which is chunk c + RD of the group or, past the group's end, chunk
// c % RD of the next group (the first group of the next step after the last
// one: J does not change between steps).  Every refill is a load, so a slot's
// next value is always the register its load writes, and the prefetch crosses
// group and step boundaries.
template <int D, int XS, int JS, int TPW, int FMT, int W, int RDB = 2, bool CP = false>
__device__ __forceinline__ void integrate_slab(const IntegArgs &a, int rep0, const unsigned char *__restrict__ stage,
                                               int ncp, bf16x8 *lb) {
    // tiles accumulated together (register budget per lane: 128 at four
    // wavefronts per SIMD, 256 at two, 512 at one)
    constexpr int GS0 = W == 16 ? (D >= 3 ? 1 : 2) : (W == 8 ? (D >= 3 ? 2 : 4) : (D >= 3 ? 4 : 8));
    constexpr int GS = GS0 < TPW ? GS0 : TPW;
    constexpr int NG = TPW / GS;        // groups of owned tiles
    // chunks of J fragments in flight: E4M3 fragments take two registers
    // per tile, bf16 ones four per term (RDB chunks)
    constexpr bool F8 = FMT == kStageE4M3;
    constexpr bool F4 = FMT == kStageE2M1;
    constexpr int RD = FMT != kStageBf16 ? 4 : RDB;
    static_assert(RD <= kSlabRingChunks, "the staging pads kSlabRingChunks chunks past the last tile");
    // PF: the state operand of the next chunk is read from LDS while the
    // current chunk's products run, where its registers fit
    constexpr bool PF = XS == 1 ? D >= 3 : D == 2;
    // CP: component passes; DP components in the LDS operand and the
    // accumulators of one pass, NPH passes per step
    constexpr int DP = CP ? 1 : D;
    constexpr int NPH = CP ? D : 1;
    const int n = a.n;
    const int r = a.r;
    const int nt = (n + 15) / 16;
    const int lane = threadIdx.x & 63;
    // wave-uniform: tile and chunk offsets stay in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jcol = lane & 15;
    const int g = lane >> 4;
    const int rep = rep0 + jcol;
    const bool valid = rep < r;
    // J fragments through a buffer resource: per-lane offset lane * bytes,
    // wave-uniform offset of (tile, chunk, term) in scalar registers
    constexpr int FB = F8 ? 8 : (F4 ? 4 : 16);                    // bytes per lane per fragment
    constexpr int CHB = (FMT != kStageBf16 ? 1 : JS) * 64 * FB;   // bytes per (tile, chunk)
    const __amdgpu_buffer_rsrc_t jres = buffer_over(stage + stage_frag_offset(nt), (uint32_t)(nt * ncp * CHB));
    const int jvoff = lane * FB;
    // row scales 2^e_p of the E4M3 fragments (per-lane offset jcol, tile offset uniform)
    const __amdgpu_buffer_rsrc_t sres = buffer_over(stage + kStageHeader, (uint32_t)(nt * 64));

    // groups holding at least one tile (their first tiles are w + GS W grp)
    int ngw = 0;
#pragma unroll
    for (int grp = 0; grp < NG; ++grp)
        if (w + GS * W * grp < nt) ngw = grp + 1;
    // byte offset of the first chunk of tile i of group grp (past the last
    // tile: the group's first tile, whose products are never used)
    auto tile_off = [&](int grp, int i) __attribute__((always_inline)) {
        const int I0 = w + GS * W * grp;
        const int I = I0 + W * i < nt ? I0 + W * i : I0;
        return I * ncp * CHB;
    };
    auto scale_of = [&](int grp, int i) __attribute__((always_inline)) {
        const int I0 = w + GS * W * grp;
        const int I = I0 + W * i < nt ? I0 + W * i : I0;
        // the lane's A row is 16 I + (lane & 15)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sres, jcol * 4, I * 64, 0));
    };

    // zero the operand area (chunks past the last tile read as zero)
    for (int i = threadIdx.x; i < ncp * DP * XS * 64; i += blockDim.x) lb[i] = bf16x8{};
    __syncthreads();

    float x[TPW][D][4];
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int I = w + W * k;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            const bool ok = valid && p < n;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) x[k][mu][v] = ok ? a.x[((size_t)p * r + rep) * D + mu] : 0.0f;
        }
        if (!CP && I < nt) slab_write_tile<D, XS>(x[k], I, lane, lb);
    }

    // the ring holds the first RD chunks of group 0; the scales of group 0
    bf16x8 ring[FMT != kStageBf16 ? 1 : RD][GS][JS];
    uint2 ring8[F8 ? RD : 1][GS];
    uint32_t ring4[F4 ? RD : 1][GS];
    float sc[GS];
#pragma unroll
    for (int i = 0; i < GS; ++i) sc[i] = F8 ? scale_of(0, i) : 1.0f;
#pragma unroll
    for (int sl = 0; sl < RD; ++sl)
#pragma unroll
        for (int i = 0; i < GS; ++i) {
            // chunks past the tile's last (ncp < RD) are the next tile's or the
            // staging's padding, loaded and never used
            if constexpr (F8) {
                ring8[sl][i] = load_frag8(jres, jvoff, tile_off(0, i) + sl * CHB);
            } else if constexpr (F4) {
                ring4[sl][i] = load_frag4(jres, jvoff, tile_off(0, i) + sl * CHB);
            } else {
#pragma unroll
                for (int t = 0; t < JS; ++t) ring[sl][i][t] = load_frag16(jres, jvoff, tile_off(0, i) + sl * CHB + t * 1024);
            }
        }
    __syncthreads();

    const float base = valid ? fmaf(a.dt, a.pump[rep] - 1.0f, 1.0f) : 0.0f;
    const float nbd = -(a.dt * a.btil);
    const float ned = -(a.dt * a.eta);
    const float dte = a.dt * a.eps;
    constexpr int NP = JS == 1 ? XS : 6;
    constexpr int pj[6] = {JS == 1 ? 0 : 2, JS == 1 ? 0 : 1, 0, JS == 1 ? 0 : 1, 0, 0};
    constexpr int px[6] = {JS == 1 ? XS - 1 : 0, JS == 1 ? (XS > 1 ? XS - 2 : 0) : 1, JS == 1 ? 0 : 2, 0, 1, 0};

    bf16x8 bxr[PF ? DP : 1][PF ? XS : 1];  // PF: the state operand of the next chunk
    for (int k = 0; k < a.steps; ++k) {
        const float *al = a.alpha + (size_t)(a.start_step + k) * D;
        float ga[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) ga[mu] = dte * al[mu];
        // CP: the norm-dependent coefficient of every owned hyperspin, from
        // the old state
        float ccp[CP ? TPW : 1][4];
        if constexpr (CP) {
#pragma unroll
            for (int kk = 0; kk < TPW; ++kk)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float S = x[kk][0][v] * x[kk][0][v];
#pragma unroll
                    for (int mu = 1; mu < D; ++mu) S = S + x[kk][mu][v] * x[kk][mu][v];
                    ccp[kk][v] = fmaf(nbd, S, base);
                }
        }

#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
        if constexpr (CP) {
            __syncthreads();  // every wavefront is done reading the previous operand
#pragma unroll
            for (int kk = 0; kk < TPW; ++kk) {
                const int I = w + W * kk;
                if (I < nt) slab_write_comp<XS>(x[kk][ph], I, slab_b_index(I >> 1, 0, 0, lane, 1, XS), lb);
            }
            __syncthreads();
        }
#pragma unroll
        for (int grp = 0; grp < NG; ++grp) {
            if (grp >= ngw) break;  // wave-uniform
            // the group whose chunks follow this group's in the stream
            const bool more = grp + 1 < ngw;
            int so[GS], son[GS];
            float scn[GS];
#pragma unroll
            for (int i = 0; i < GS; ++i) {
                so[i] = tile_off(grp, i);
                son[i] = more ? tile_off(grp + 1 < NG ? grp + 1 : 0, i) : tile_off(0, i);
                if constexpr (F8) scn[i] = more ? scale_of(grp + 1 < NG ? grp + 1 : 0, i) : scale_of(0, i);
            }
            f32x4 acc[GS][DP];
#pragma unroll
            for (int i = 0; i < GS; ++i)
#pragma unroll
                for (int mu = 0; mu < DP; ++mu) acc[i][mu] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (PF) {
                if (grp == 0) {
                    // later groups find chunk 0 in bxr, read during the previous
                    // group's last chunk
#pragma unroll
                    for (int mu = 0; mu < DP; ++mu)
#pragma unroll
                        for (int t = 0; t < XS; ++t) bxr[mu][t] = lb[slab_b_index(0, mu, t, lane, DP, XS)];
                }
            }
            // chunk c (c % RD == sl): take its J fragments from ring slot sl and
            // refill the slot, take its state operand, accumulate
            auto chunk = [&](int sl, int c) __attribute__((always_inline)) {
                bf16x8 af[GS][JS];
                const int cn = c + RD;
#pragma unroll
                for (int i = 0; i < GS; ++i) {
                    const int nxt = cn < ncp ? so[i] + cn * CHB : son[i] + sl * CHB;
                    if constexpr (F8) {
                        af[i][0] = fp8_fragment(ring8[sl][i], sc[i]);
                        ring8[sl][i] = load_frag8(jres, jvoff, nxt);
                    } else if constexpr (F4) {
                        af[i][0] = fp4_fragment(ring4[sl][i]);
                        ring4[sl][i] = load_frag4(jres, jvoff, nxt);
                    } else {
#pragma unroll
                        for (int t = 0; t < JS; ++t) {
                            af[i][t] = ring[sl][i][t];
                            ring[sl][i][t] = load_frag16(jres, jvoff, nxt + t * 1024);
                        }
                    }
                }
                bf16x8 bx[DP][XS];
                if constexpr (PF) {
                    // past the last chunk: chunk 0 of the next group
                    const int cb = c + 1 < ncp ? c + 1 : 0;
#pragma unroll
                    for (int mu = 0; mu < DP; ++mu)
#pragma unroll
                        for (int t = 0; t < XS; ++t) {
                            bx[mu][t] = bxr[PF ? mu : 0][PF ? t : 0];
                            bxr[PF ? mu : 0][PF ? t : 0] = lb[slab_b_index(cb, mu, t, lane, DP, XS)];
                        }
                } else {
#pragma unroll
                    for (int mu = 0; mu < DP; ++mu)
#pragma unroll
                        for (int t = 0; t < XS; ++t) bx[mu][t] = lb[slab_b_index(c, mu, t, lane, DP, XS)];
                }
#pragma unroll
                for (int q = 0; q < NP; ++q)
#pragma unroll
                    for (int i = 0; i < GS; ++i)
#pragma unroll
                        for (int mu = 0; mu < DP; ++mu)
                            acc[i][mu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i][pj[q]], bx[mu][px[q]],
                                                                                acc[i][mu], 0, 0, 0);
            };
            int c = 0;
            for (; c + RD <= ncp; c += RD) {
#pragma unroll
                for (int sl = 0; sl < RD; ++sl) chunk(sl, c + sl);
            }
#pragma unroll
            for (int sl = 0; sl + 1 < RD; ++sl)
                if (c + sl < ncp) chunk(sl, c + sl);
            // fused Euler update of the group's tiles
#pragma unroll
            for (int i = 0; i < GS; ++i) {
                const int kk = GS * grp + i;
                if (w + W * kk >= nt) continue;
                if constexpr (CP) {
                    // component ph only; x^2 formed again rather than kept
                    // live from the coefficient's sum
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        float xv = x[kk][ph][v];
                        asm volatile("" : "+v"(xv));
                        const float y = xv * fmaf(ned, xv * xv, ccp[kk][v]);
                        x[kk][ph][v] = fmaf(ga[ph], acc[i][0][v], y);
                    }
                    continue;
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float x2[D];
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) x2[mu] = x[kk][mu][v] * x[kk][mu][v];
                    float S = x2[0];
#pragma unroll
                    for (int mu = 1; mu < D; ++mu) S = S + x2[mu];
                    const float cc = fmaf(nbd, S, base);
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) {
                        const float y = x[kk][mu][v] * fmaf(ned, x2[mu], cc);
                        x[kk][mu][v] = fmaf(ga[mu], acc[i][CP ? 0 : mu][v], y);
                    }
                }
            }
            if constexpr (F8) {
#pragma unroll
                for (int i = 0; i < GS; ++i) sc[i] = scn[i];
            }
        }
        }
        if constexpr (!CP) {
            __syncthreads();  // every wavefront is done reading the old operand
#pragma unroll
            for (int kk = 0; kk < TPW; ++kk) {
                const int I = w + W * kk;
                if (I < nt) slab_write_tile<D, XS>(x[kk], I, lane, lb);
            }
            __syncthreads();
        }
    }

    // addresses of the final store are formed here, not kept live through the run
    int lane_s = lane;
    asm volatile("" : "+v"(lane_s));
    const int g_s = lane_s >> 4;
    const int rep_s = rep0 + (lane_s & 15);
#pragma unroll
    for (int kk = 0; kk < TPW; ++kk) {
        const int I = w + W * kk;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g_s + v;
            if (rep_s < r && p < n) {
#pragma unroll
                for (int mu = 0; mu < D; ++mu) a.x[((size_t)p * r + rep_s) * D + mu] = x[kk][mu][v];
            }
        }
    }
}

// Stages J of one problem as A fragments: bf16 [tile][chunk][JS][64 lanes],
// or (JS = 1 and the header flag set) E4M3 [tile][chunk][64 lanes] in the
// same slot order.  Threads first, first + stride, ... of the launch share
// the fragment slots.
template <int JS>
__device__ __forceinline__ void stage_jfrag_part(const IntegArgs &a, int ncp, unsigned char *__restrict__ stage,
                                                 int first, int stride) {
    const int nt = (a.n + 15) / 16;
    const int total = nt * ncp * 64;
    const int fmt = JS == 1 ? *reinterpret_cast<const int *>(stage) : kStageBf16;
    const float *scale = reinterpret_cast<const float *>(stage + kStageHeader);
    bf16x8 *out = reinterpret_cast<bf16x8 *>(stage + stage_frag_offset(nt));
    uint2 *out8 = reinterpret_cast<uint2 *>(stage + stage_frag_offset(nt));
    uint32_t *out4 = reinterpret_cast<uint32_t *>(stage + stage_frag_offset(nt));
    for (int idx = first; idx < total; idx += stride) {
        const int lane = idx & 63;
        const int c = (idx >> 6) % ncp;
        const int I = (idx >> 6) / ncp;
        if (fmt == kStageE2M1) {
            // every coupling is -1, 0 or +1: E2M1 codes 0xA, 0x0, 0x2
            const int i = lane & 15, g = lane >> 4;
            const int p = 16 * I + i;
            uint32_t wd = 0u;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int q = 32 * c + 16 * (s >> 2) + 4 * g + (s & 3);
                const float v = (p < a.n && q < a.n) ? coupling(a.j, a.j_dtype, a.n, p, q) : 0.0f;
                const uint32_t code = v > 0.0f ? 0x2u : (v < 0.0f ? 0xAu : 0x0u);
                wd |= code << (4 * s);
            }
            out4[(size_t)(I * ncp + c) * 64 + lane] = wd;
        } else if (fmt == kStageE4M3) {
            const int i = lane & 15, g = lane >> 4;
            const int p = 16 * I + i;
            const int e = p < a.n ? ilogbf(scale[p]) : 0;
            uint32_t wd[2] = {0u, 0u};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int q = 32 * c + 16 * (s >> 2) + 4 * g + (s & 3);
                uint32_t code = 0u;
                if (p < a.n && q < a.n) {
                    code = (a.j_dtype == CHYM_J_FP8) ? reinterpret_cast<const uint8_t *>(a.j)[(size_t)p * a.n + q]
                                                      : e4m3_code(ldexpf(coupling(a.j, a.j_dtype, a.n, p, q), -e));
                }
                wd[s >> 2] |= code << (8 * (s & 3));
            }
            out8[(size_t)(I * ncp + c) * 64 + lane] = uint2{wd[0], wd[1]};
        } else {
            bf16x8 f[JS];
            j_fragment<JS>(a, I, c, lane, f);
#pragma unroll
            for (int t = 0; t < JS; ++t) out[((size_t)(I * ncp + c) * JS + t) * 64 + lane] = f[t];
        }
    }
}

template <int JS>
__global__ __launch_bounds__(256) void k_stage_jfrag(IntegArgs a, int ncp, unsigned char *__restrict__ stage) {
    stage_jfrag_part<JS>(a, ncp, stage, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// The same for the tasks list[0 .. n) of a batch, bpt blocks per task:
// task list[b / bpt] is staged into stages[task] with ncps[task] chunks.
template <int JS>
__global__ __launch_bounds__(256) void k_stage_jfrag_batched(const IntegArgs *__restrict__ tasks,
                                                             const int *__restrict__ list, int bpt,
                                                             const int *__restrict__ ncps,
                                                             unsigned char *const *__restrict__ stages) {
    const int t = list[blockIdx.x / bpt];
    const IntegArgs a = tasks[t];
    stage_jfrag_part<JS>(a, ncps[t], stages[t], (blockIdx.x % bpt) * blockDim.x + threadIdx.x, bpt * blockDim.x);
}

// The narrow formats exist for single-term couplings; the header is uniform.
template <int D, int XS, int JS, int TPW, int W, bool CP>
__device__ __forceinline__ void slab_run(const IntegArgs &a, int rep0, const unsigned char *stage, int ncp,
                                         bf16x8 *lb) {
    if constexpr (JS == 1) {
        const int fmt = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const int *>(stage));
        if (fmt == kStageE2M1) {
            integrate_slab<D, XS, JS, TPW, kStageE2M1, W, 2, CP>(a, rep0, stage, ncp, lb);
            return;
        }
        if (fmt == kStageE4M3) {
            integrate_slab<D, XS, JS, TPW, kStageE4M3, W, 2, CP>(a, rep0, stage, ncp, lb);
            return;
        }
    }
    integrate_slab<D, XS, JS, TPW, kStageBf16, W, 2, CP>(a, rep0, stage, ncp, lb);
}

// Column slabs of one problem: block b integrates replicas 16 b .. 16 b + 15.
// A single problem's J is read by every CU from the same L2 lines, so it is
// staged as bf16 fragments (no E4M3 path: the conversion per value and
// product on the vector ALU costs more than the halved L2 bytes save there,
// measured 3-10% at N = 200 - 1000); with the registers that frees, blocks of
// eight wavefronts keep four chunks of the bf16 stream in flight (measured
// 1-5% faster at N = 800 - 1000).  Batches, whose tasks stream many distinct
// couplings through L2 at once, take the E4M3 path where it applies
// (k_integrate_slab_persistent).
template <int D, int XS, int JS, int TPW, int W, bool CP = false>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(W / 4)))
void k_integrate_slab(IntegArgs a, const unsigned char *__restrict__ stage, int ncp) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RDB = (W == 8 && XS == 1 && JS == 1) ? 4 : 2;
    integrate_slab<D, XS, JS, TPW, kStageBf16, W, RDB, CP>(a, blockIdx.x * 16, stage, ncp,
                                                      reinterpret_cast<bf16x8 *>(smem));
}

// Persistent form: blocks pop (task, column slab) items; jfs[task] is the
// task's staged J and ncps[task] its chunk count.
template <int D, int XS, int JS, int TPW, int W, bool CP = false>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(W / 4)))
void k_integrate_slab_persistent(const IntegArgs *__restrict__ tasks, const int2 *__restrict__ items, int n_items,
                                 int *__restrict__ counter, const unsigned char *const *__restrict__ jfs,
                                 const int *__restrict__ ncps) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int2 wi = items[it];
        const IntegArgs a = tasks[wi.x];
        slab_run<D, XS, JS, TPW, W, CP>(a, wi.y * 16, jfs[wi.x], ncps[wi.x], reinterpret_cast<bf16x8 *>(smem));
    }
}

struct SlabKernels {
    void (*single)(IntegArgs, const unsigned char *, int);
    void (*persistent)(const IntegArgs *, const int2 *, int, int *, const unsigned char *const *, const int *);
    int waves;
};

// Slab shapes: eight wavefronts with 4 or 8 tiles each, and in the bf16
// form sixteen wavefronts with 1 or 2 tiles each, or 4 at D <= 2 (measured faster up to
// about 32 row tiles: more wavefronts cover the latency of the operand reads
// and of the J stream when each owns few tiles).  One wavefront per SIMD with
// 16 tiles measured slower at N = 1000, D = 4 (a lone wavefront cannot cover
// the L2 latency of the J stream), and at N = 200 - 800 too.  cp: the
// component-pass form, built for the float32 form at d >= 2 in blocks of
// eight wavefronts.
template <int D, int XS, int JS>
SlabKernels slab_lookup_tpw(int tpw, int waves, bool cp) {
    if (cp) {
        // the shapes whose float32 operand exceeds LDS: up to 32 tiles only at d = 4
        if constexpr (XS == 3 && D >= 2) {
            if constexpr (D == 4) {
                if (waves == 8 && tpw == 4)
                    return SlabKernels{k_integrate_slab<D, XS, JS, 4, 8, true>,
                                       k_integrate_slab_persistent<D, XS, JS, 4, 8, true>, 8};
            }
            if (waves == 8 && tpw == 8)
                return SlabKernels{k_integrate_slab<D, XS, JS, 8, 8, true>,
                                   k_integrate_slab_persistent<D, XS, JS, 8, 8, true>, 8};
        }
        return SlabKernels{nullptr, nullptr, 0};
    }
    if (waves == 8 && tpw == 4)
        return SlabKernels{k_integrate_slab<D, XS, JS, 4, 8>, k_integrate_slab_persistent<D, XS, JS, 4, 8>, 8};
    if (waves == 8 && tpw == 8)
        return SlabKernels{k_integrate_slab<D, XS, JS, 8, 8>, k_integrate_slab_persistent<D, XS, JS, 8, 8>, 8};
    if constexpr (XS == 1) {
        if (waves == 16 && tpw == 1)
            return SlabKernels{k_integrate_slab<D, XS, JS, 1, 16>, k_integrate_slab_persistent<D, XS, JS, 1, 16>, 16};
        if (waves == 16 && tpw == 2)
            return SlabKernels{k_integrate_slab<D, XS, JS, 2, 16>, k_integrate_slab_persistent<D, XS, JS, 2, 16>, 16};
        if constexpr (D <= 2) {  // four tiles of three or four components spill at 128 registers
            if (waves == 16 && tpw == 4)
                return SlabKernels{k_integrate_slab<D, XS, JS, 4, 16>, k_integrate_slab_persistent<D, XS, JS, 4, 16>,
                                   16};
        }
    }
    return SlabKernels{nullptr, nullptr, 0};
}

#define CHYM_DECLARE_SLAB(D, XS, JS) SlabKernels lookup_slab_##D##_##XS##_##JS(int tpw, int waves, bool cp);
CHYM_DECLARE_SLAB(1, 3, 1) CHYM_DECLARE_SLAB(1, 1, 1) CHYM_DECLARE_SLAB(1, 3, 3)
CHYM_DECLARE_SLAB(2, 3, 1) CHYM_DECLARE_SLAB(2, 1, 1) CHYM_DECLARE_SLAB(2, 3, 3)
CHYM_DECLARE_SLAB(3, 3, 1) CHYM_DECLARE_SLAB(3, 1, 1) CHYM_DECLARE_SLAB(3, 3, 3)
CHYM_DECLARE_SLAB(4, 3, 1) CHYM_DECLARE_SLAB(4, 1, 1) CHYM_DECLARE_SLAB(4, 3, 3)
#undef CHYM_DECLARE_SLAB

}  // namespace chym

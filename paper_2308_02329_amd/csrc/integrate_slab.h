// Streamed-J CHYM integrator for large N (gfx950).
//
// One block of eight wavefronts (two per SIMD) owns a column slab -- 16
// replicas x D components of one problem -- for the whole run.  Row tiles (16
// rows) are dealt to the wavefronts round-robin: wavefront w owns tiles w,
// w+8, ...,
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
// (at this size it does not fit in LDS).
//
// Per step: for each group of four owned tiles, accumulate G over all
// chunks (the J fragments of the next chunk are fetched while the current
// chunk's matrix-core work runs), then apply the fused Euler update to those
// tiles in registers; after a barrier every wavefront writes its tiles' new
// operand terms to LDS, and a second barrier publishes them.
constexpr int kSlabWaves = 8;
#pragma once

#include "integrate_kernel.h"

namespace chym {

// LDS operand layout: [chunk][component][term][64 lanes] of bf16x8 (1 KB each).
__device__ __forceinline__ int slab_b_index(int c, int mu, int t, int lane, int D, int XS) {
    return ((c * D + mu) * XS + t) * 64 + lane;
}

// Writes the operand terms of tile I (its four rows of this lane) into the
// half (I & 1) of chunk I >> 1.
template <int D, int XS>
__device__ __forceinline__ void slab_write_tile(const float (&xt)[D][4], int I, int lane, bf16x8 *lb,
                                                const NegPair &k) {
    typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        bf16x2 t[XS][2];
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            const float a = xt[mu][2 * pr], b = xt[mu][2 * pr + 1];
            const bf16x2 h = pack_rne(a, b);
            t[0][pr] = h;
            if constexpr (XS == 3) {
                const float ra = resid_lo(h, a, k), rb = resid_hi(h, b, k);
                const bf16x2 m = pack_rne(ra, rb);
                const float sa = resid_lo(m, ra, k), sb = resid_hi(m, rb, k);
                t[1][pr] = m;
                t[2][pr] = pack_rne(sa, sb);
            }
        }
#pragma unroll
        for (int q = 0; q < XS; ++q) {
            bf16x4 *dst = reinterpret_cast<bf16x4 *>(lb + slab_b_index(I >> 1, mu, q, lane, D, XS)) + (I & 1);
            *dst = __builtin_shufflevector(t[q][0], t[q][1], 0, 1, 2, 3);
        }
    }
}

// Integrates the column slab rep0 .. rep0+15 of problem a.  jf: staged A
// fragments [tile][chunk][JS][64]; ncp: chunk count of the staging; lb: LDS
// operand area of ncp * D * XS fragments.  Called by all kSlabWaves
// wavefronts of the block; contains block barriers.
template <int D, int XS, int JS, int TPW>
__device__ __forceinline__ void integrate_slab(const IntegArgs &a, int rep0, const bf16x8 *__restrict__ jf, int ncp,
                                               bf16x8 *lb) {
    constexpr int GS = D >= 3 ? 2 : 4;  // tiles accumulated together (register budget)
    constexpr int NG = TPW / GS;        // groups of owned tiles
    const int n = a.n;
    const int r = a.r;
    const int nt = (n + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int jcol = lane & 15;
    const int g = lane >> 4;
    const int rep = rep0 + jcol;
    const bool valid = rep < r;
    const NegPair negk = neg_pair();

    // zero the operand area (chunks past the last tile read as zero)
    for (int i = threadIdx.x; i < ncp * D * XS * 64; i += blockDim.x) lb[i] = bf16x8{};
    __syncthreads();

    float x[TPW][D][4];
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int I = w + kSlabWaves * k;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            const bool ok = valid && p < n;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) x[k][mu][v] = ok ? a.x[((size_t)p * r + rep) * D + mu] : 0.0f;
        }
        if (I < nt) slab_write_tile<D, XS>(x[k], I, lane, lb, negk);
    }
    __syncthreads();

    const float base = valid ? fmaf(a.dt, a.pump[rep] - 1.0f, 1.0f) : 0.0f;
    const float nbd = -(a.dt * a.btil);
    const float ned = -(a.dt * a.eta);
    const float dte = a.dt * a.eps;
    constexpr int NP = JS == 1 ? XS : 6;
    constexpr int pj[6] = {JS == 1 ? 0 : 2, JS == 1 ? 0 : 1, 0, JS == 1 ? 0 : 1, 0, 0};
    constexpr int px[6] = {JS == 1 ? XS - 1 : 0, JS == 1 ? (XS > 1 ? XS - 2 : 0) : 1, JS == 1 ? 0 : 2, 0, 1, 0};

    for (int k = 0; k < a.steps; ++k) {
        const float *al = a.alpha + (size_t)(a.start_step + k) * D;
        float ga[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) ga[mu] = dte * al[mu];

#pragma unroll
        for (int grp = 0; grp < NG; ++grp) {
            // tiles I0 + 8 i, i < GS
            const int I0 = w + GS * kSlabWaves * grp;
            if (I0 >= nt) break;  // wave-uniform
            f32x4 acc[GS][D];
#pragma unroll
            for (int i = 0; i < GS; ++i)
#pragma unroll
                for (int mu = 0; mu < D; ++mu) acc[i][mu] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const bf16x8 *jrow[GS];
#pragma unroll
            for (int i = 0; i < GS; ++i) {
                const int I = I0 + kSlabWaves * i < nt ? I0 + kSlabWaves * i : I0;  // past the end: a valid tile
                jrow[i] = jf + (size_t)I * ncp * JS * 64 + lane;
            }
            // J fragments two chunks ahead: ring slots 0 (even chunks), 1 (odd)
            bf16x8 ring[2][GS][JS];
#pragma unroll
            for (int sl = 0; sl < 2; ++sl)
#pragma unroll
                for (int i = 0; i < GS; ++i)
#pragma unroll
                    for (int t = 0; t < JS; ++t)
                        ring[sl][i][t] = sl < ncp ? jrow[i][(size_t)(sl * JS + t) * 64] : bf16x8{};
            auto chunk = [&](int c, bf16x8 (&af)[GS][JS]) __attribute__((always_inline)) {
                bf16x8 bx[D][XS];
#pragma unroll
                for (int mu = 0; mu < D; ++mu)
#pragma unroll
                    for (int t = 0; t < XS; ++t) bx[mu][t] = lb[slab_b_index(c, mu, t, lane, D, XS)];
#pragma unroll
                for (int q = 0; q < NP; ++q)
#pragma unroll
                    for (int i = 0; i < GS; ++i)
#pragma unroll
                        for (int mu = 0; mu < D; ++mu)
                            acc[i][mu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i][pj[q]], bx[mu][px[q]],
                                                                                acc[i][mu], 0, 0, 0);
            };
            for (int c = 0; c < ncp; c += 2) {
#pragma unroll
                for (int sl = 0; sl < 2; ++sl) {
                    const int cc = c + sl;
                    if (cc < ncp) {
                        bf16x8 af[GS][JS];
#pragma unroll
                        for (int i = 0; i < GS; ++i)
#pragma unroll
                            for (int t = 0; t < JS; ++t) af[i][t] = ring[sl][i][t];
                        if (cc + 2 < ncp) {
#pragma unroll
                            for (int i = 0; i < GS; ++i)
#pragma unroll
                                for (int t = 0; t < JS; ++t)
                                    ring[sl][i][t] = jrow[i][(size_t)((cc + 2) * JS + t) * 64];
                        }
                        chunk(cc, af);
                    }
                }
            }
            // fused Euler update of the group's tiles
#pragma unroll
            for (int i = 0; i < GS; ++i) {
                const int kk = GS * grp + i;
                if (w + kSlabWaves * kk >= nt) continue;
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
                        x[kk][mu][v] = fmaf(ga[mu], acc[i][mu][v], y);
                    }
                }
            }
        }
        __syncthreads();  // every wavefront is done reading the old operand
#pragma unroll
        for (int kk = 0; kk < TPW; ++kk) {
            const int I = w + kSlabWaves * kk;
            if (I < nt) slab_write_tile<D, XS>(x[kk], I, lane, lb, negk);
        }
        __syncthreads();
    }

#pragma unroll
    for (int kk = 0; kk < TPW; ++kk) {
        const int I = w + kSlabWaves * kk;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            if (valid && p < n) {
#pragma unroll
                for (int mu = 0; mu < D; ++mu) a.x[((size_t)p * r + rep) * D + mu] = x[kk][mu][v];
            }
        }
    }
}

// Stages J of one problem as A fragments [tile][chunk][JS][64 lanes].
template <int JS>
__global__ __launch_bounds__(256) void k_stage_jfrag(IntegArgs a, int ncp, bf16x8 *__restrict__ out) {
    const int nt = (a.n + 15) / 16;
    const int total = nt * ncp * 64;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int lane = idx & 63;
        const int c = (idx >> 6) % ncp;
        const int I = (idx >> 6) / ncp;
        bf16x8 f[JS];
        j_fragment<JS>(a, I, c, lane, f);
#pragma unroll
        for (int t = 0; t < JS; ++t) out[((size_t)(I * ncp + c) * JS + t) * 64 + lane] = f[t];
    }
}

// Column slabs of one problem: block b integrates replicas 16 b .. 16 b + 15.
template <int D, int XS, int JS, int TPW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void k_integrate_slab(IntegArgs a, const bf16x8 *__restrict__ jf, int ncp) {
    extern __shared__ __align__(16) unsigned char smem[];
    integrate_slab<D, XS, JS, TPW>(a, blockIdx.x * 16, jf, ncp, reinterpret_cast<bf16x8 *>(smem));
}

// One work item of the persistent form.
template <int D, int XS, int JS, int TPW>
__device__ __forceinline__ void slab_item(const IntegArgs *__restrict__ tasks, int2 wi,
                                                    const bf16x8 *const *__restrict__ jfs, const int *__restrict__ ncps,
                                                    bf16x8 *lb) {
    const IntegArgs a = tasks[wi.x];
    integrate_slab<D, XS, JS, TPW>(a, wi.y * 16, jfs[wi.x], ncps[wi.x], lb);
}

// Persistent form: blocks pop (task, column slab) items; jfs[task] is the
// task's staged J and ncps[task] its chunk count.
template <int D, int XS, int JS, int TPW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void k_integrate_slab_persistent(const IntegArgs *__restrict__ tasks, const int2 *__restrict__ items, int n_items,
                                 int *__restrict__ counter, const bf16x8 *const *__restrict__ jfs,
                                 const int *__restrict__ ncps) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        slab_item<D, XS, JS, TPW>(tasks, items[it], jfs, ncps, reinterpret_cast<bf16x8 *>(smem));
    }
}

struct SlabKernels {
    void (*single)(IntegArgs, const bf16x8 *, int);
    void (*persistent)(const IntegArgs *, const int2 *, int, int *, const bf16x8 *const *, const int *);
};

template <int D, int XS, int JS>
SlabKernels slab_lookup_tpw(int tpw) {
    switch (tpw) {
        case 4: return SlabKernels{k_integrate_slab<D, XS, JS, 4>, k_integrate_slab_persistent<D, XS, JS, 4>};
        case 8: return SlabKernels{k_integrate_slab<D, XS, JS, 8>, k_integrate_slab_persistent<D, XS, JS, 8>};
        default: return SlabKernels{nullptr, nullptr};
    }
}

#define CHYM_DECLARE_SLAB(D, XS, JS) SlabKernels lookup_slab_##D##_##XS##_##JS(int tpw);
CHYM_DECLARE_SLAB(1, 3, 1) CHYM_DECLARE_SLAB(1, 1, 1) CHYM_DECLARE_SLAB(1, 3, 3)
CHYM_DECLARE_SLAB(2, 3, 1) CHYM_DECLARE_SLAB(2, 1, 1) CHYM_DECLARE_SLAB(2, 3, 3)
CHYM_DECLARE_SLAB(3, 3, 1) CHYM_DECLARE_SLAB(3, 1, 1) CHYM_DECLARE_SLAB(3, 3, 3)
CHYM_DECLARE_SLAB(4, 3, 1) CHYM_DECLARE_SLAB(4, 1, 1) CHYM_DECLARE_SLAB(4, 3, 3)
#undef CHYM_DECLARE_SLAB

}  // namespace chym

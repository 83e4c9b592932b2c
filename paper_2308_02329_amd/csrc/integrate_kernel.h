// Register-resident CHYM integrator for gfx950 (CDNA4).
//
// One wavefront owns 16 replicas of one problem for the whole run.  Their
// state, all N rows x D components, lives in VGPRs in the layout of the
// 16x16 MFMA accumulator: lane l = j + 16 g holds, for row tile I and
// component mu, the four rows 16 I + 4 g + v (v = 0..3) of replica j.
// Component mu of every replica forms its own 16-column plane, so the D
// components of one hyperspin sit in one lane and the nonlocal loss
// S_p = sum_nu x_{p,nu}^2 needs no cross-lane traffic.
//
// The contraction G = J X (paper: C = J_N (x) 1_D acting on the amplified
// fields, Eq. (1)-(2)) runs on v_mfma_f32_16x16x32_bf16 with J as the A
// operand and the state as the B operand.  The order in which the 32 values
// of a K-chunk are summed is free, so chunk c is defined as the rows a lane
// already holds in row tiles 2c and 2c+1: the B operand is built from the
// lane's own registers with no LDS round trip and no shuffle, and J is laid
// out in the matching (permuted) order as A fragments, either gathered once
// per work item into registers (one wavefront per work item) or staged once
// per work item into LDS and shared by the wavefronts of a block (which
// frees the registers for a second wavefront per SIMD, so that one wave's
// matrix-core work overlaps the other's vector work).
//
// Float32 form: x is fed as the exact sum x = hi + mid + lo of three bf16
// terms (each residual of a round-to-nearest bf16 has at most 16, then 8,
// significant bits), so every product J_pq x_q is formed exactly and summed
// in float32.  An integer J is exact in bf16; a float J is split the same
// way and the six leading cross terms are kept (error ~2^-24 relative).
// BF16 form: one bf16 term each.  The split works on pairs of values: one
// packed conversion rounds two values, and each residual x - hi is a plain
// float subtraction of the widened bf16 half, exact because the residual is
// representable.
//
// The Euler update (pump gain, coupling with the annealing weight, nonlocal
// loss, local saturation) is fused after the contraction and works on the
// accumulator registers in place; the whole step loop runs inside the
// kernel, with no barrier and no global-memory traffic per step except the
// D annealing weights alpha[k][mu] (scalar loads).
#pragma once

#include "chym_internal.h"

namespace chym {

typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

template <int XS>
struct XSplit {
    bf16x8 t[XS];
};

__device__ __forceinline__ float bf_to_f(__bf16 h) { return (float)h; }

__device__ __forceinline__ bf16x2 pack_rne(float a, float b) { return __builtin_convertvector((f32x2){a, b}, bf16x2); }

// a - (float)h.x and b - (float)h.y, exact when representable.  The halves
// are widened by a shift or a mask and subtracted on the vector ALU: a bf16
// dot product against (-1, 0) gives the same value, but on gfx950 the dot
// instruction does not execute alongside matrix-core products (measured: each
// one costs several times a plain vector instruction when interleaved with
// them).
__device__ __forceinline__ float resid_lo(bf16x2 h, float a) {
    return a - __uint_as_float(__builtin_bit_cast(uint32_t, h) << 16);
}
__device__ __forceinline__ float resid_hi(bf16x2 h, float b) {
    return b - __uint_as_float(__builtin_bit_cast(uint32_t, h) & 0xffff0000u);
}

__device__ __forceinline__ bf16x8 join4(bf16x2 p0, bf16x2 p1, bf16x2 p2, bf16x2 p3) {
    typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
    const bf16x4 lo = __builtin_shufflevector(p0, p1, 0, 1, 2, 3);
    const bf16x4 hi = __builtin_shufflevector(p2, p3, 0, 1, 2, 3);
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Splits 8 floats (4 pairs) into XS bf16 terms whose sum is exact.
template <int XS>
__device__ __forceinline__ void split8(const float (&v)[8], XSplit<XS> &out) {
    bf16x2 t[XS][4];
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
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
    for (int k = 0; k < XS; ++k) out.t[k] = join4(t[k][0], t[k][1], t[k][2], t[k][3]);
}

// Loads one coupling value as float (0 outside the n x n matrix).
__device__ __forceinline__ float j_at(const IntegArgs &a, int p, int q) {
    if (p >= a.n || q >= a.n) return 0.0f;
    return coupling(a.j, a.j_dtype, a.n, p, q);
}

// A fragment (I, c) for lane (i, g): slot s holds
// J[16 I + i][32 c + 16 (s >> 2) + 4 g + (s & 3)], split into JS bf16 terms.
template <int JS>
__device__ __forceinline__ void j_fragment(const IntegArgs &a, int I, int c, int lane, bf16x8 (&f)[JS]) {
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const float v = j_at(a, 16 * I + i, 32 * c + 16 * (s >> 2) + 4 * g + (s & 3));
        if constexpr (JS == 1) {
            f[0][s] = (__bf16)v;
        } else {
            const __bf16 h = (__bf16)v;
            const float r1 = v - bf_to_f(h);
            const __bf16 m = (__bf16)r1;
            const float r2 = r1 - bf_to_f(m);
            f[0][s] = h;
            f[1][s] = m;
            f[2][s] = (__bf16)r2;
        }
    }
}

// Stages all A fragments of J into LDS, layout [JS][NT][NC][64 lanes].
template <int NT, int JS>
__device__ __forceinline__ void stage_j(const IntegArgs &a, bf16x8 *jl) {
    constexpr int NC = (NT + 1) / 2;
    for (int idx = threadIdx.x; idx < NT * NC * 64; idx += blockDim.x) {
        const int lane = idx & 63;
        const int c = (idx >> 6) % NC;
        const int I = (idx >> 6) / NC;
        bf16x8 f[JS];
        j_fragment<JS>(a, I, c, lane, f);
#pragma unroll
        for (int t = 0; t < JS; ++t) jl[t * NT * NC * 64 + idx] = f[t];
    }
}

// Gain of the nonlinear medium for a field of amplitude A under pump h:
// K = P / (P cosh(kl P) - h sinh(kl P)), P = sqrt(h^2 + A^2), written as
// 2 P e / ((P + h) + (P - h) e^2) with e = exp(kl P); with P - h = A^2 / (P + h)
// and both terms multiplied by s = P + h this is 2 P e s / (s^2 + A^2 e^2),
// which has no cancellation for h >= 0 and needs one reciprocal.  The square
// root, reciprocal and exponential are the hardware's (each within about
// 1 ulp); kl2 = kl log2(e).
__device__ __forceinline__ float nlm_gain(float A, float h, float kl2) {
    const float A2 = A * A;
    const float P = __builtin_amdgcn_sqrtf(fmaf(h, h, A2));
    const float s = P + h;
    if (!(s > 0.0f)) return 1.0f;  // A = h = 0: the medium is transparent
    const float e = __builtin_amdgcn_exp2f(kl2 * P);
    const float den = fmaf(A2, e * e, s * s);
    return (2.0f * P * e * s) * __builtin_amdgcn_rcpf(den);
}

// Integrates the 16 replicas rep0 .. rep0+15 of problem a for a.steps steps.
// Called by one whole wavefront.  JLDS: J fragments are read from the
// block's LDS copy every step; otherwise they are gathered into registers.
// MAP: the round-trip map of Eq. (2) instead of its continuous limit: every
// amplitude first passes the medium (A <- K(A) A, pump h = pump[replica]),
// then the same update runs with the map's coefficients, which the host puts
// in eps, btil, eta and c0 (dt = 1).
template <int NT, int D, int XS, int JS, bool JLDS, bool MAP = false>
__device__ __forceinline__ void integrate_group(const IntegArgs &a, int rep0, const bf16x8 *jl) {
    constexpr int NC = (NT + 1) / 2;
    const int n = a.n;
    const int r = a.r;
    const int lane = threadIdx.x & 63;
    const int jcol = lane & 15;
    const int g = lane >> 4;
    const int rep = rep0 + jcol;
    const bool valid = rep < r;

    bf16x8 jr[JLDS ? 1 : JS][JLDS ? 1 : NT][JLDS ? 1 : NC];
    if constexpr (!JLDS) {
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bf16x8 f[JS];
                j_fragment<JS>(a, I, c, lane, f);
#pragma unroll
                for (int t = 0; t < JS; ++t) jr[t][I][c] = f[t];
            }
    }

    // ---- load the state (zero for padded rows and replicas) ----
    float x[NT][D][4];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            const bool ok = valid && p < n;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) x[I][mu][v] = ok ? a.x[((size_t)p * r + rep) * D + mu] : 0.0f;
        }

    // 1 + dt (r_i - 1); for the map the constant (1 - loss)(1 - b), and its pump h
    const float base = valid ? (MAP ? a.c0 : fmaf(a.dt, a.pump[rep] - 1.0f, 1.0f)) : 0.0f;
    const float hmap = (MAP && valid) ? a.pump[rep] : 0.0f;
    const float kl2 = a.kl * 1.44269504088896340736f;  // kl log2(e)
    const float nbd = -(a.dt * a.btil);
    const float ned = -(a.dt * a.eta);
    const float dte = a.dt * a.eps;

    // D = 2, 3 with J in LDS: at D = 3 the state (NT * 12 registers), the
    // accumulators (as many) and the three split terms of every component
    // (36) leave no room at two wavefronts per SIMD, and the compiler spills.
    // There the local part is formed after the contraction from x, which
    // stays whole (no separate y while x is live), one component is split at
    // a time, and a scheduling barrier closes every chunk, so that nothing is
    // hoisted into an earlier chunk.  The arithmetic and every summation
    // order are unchanged, so the result is bit-identical.  At D = 2 the same
    // order measured 4% faster; at D = 4 slower.
    constexpr bool CO = JLDS && (D == 2 || D == 3) && !MAP;

    for (int k = 0; k < a.steps; ++k) {
            if constexpr (JLDS) {
                // keep the J fragments in LDS: reload them every step instead of
                // letting them be hoisted into registers
                asm volatile("" ::: "memory");
            }
            const float *al = a.alpha + (size_t)(a.start_step + k) * D;
            float ga[D];
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                // wave-uniform: kept in scalar registers
                const float w = dte * al[mu];
                ga[mu] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(w)));
            }

            // The update is x <- y + dt eps alpha_mu G with the local part
            // y = x (1 + dt (r-1) - dt btil S - dt eta x^2).  y is formed tile by
            // tile just before the tile's state is split into matrix-core
            // operands; the split then consumes x in place, and y becomes the new
            // state with one multiply-add once G is complete.
            float y[NT][D][4];
            f32x4 acc[NT][D];
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int mu = 0; mu < D; ++mu) acc[I][mu] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int I = 2 * c + h;
                    if (I < NT && !CO) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            if constexpr (MAP) {
#pragma unroll
                                for (int mu = 0; mu < D; ++mu)
                                    x[I][mu][v] = nlm_gain(x[I][mu][v], hmap, kl2) * x[I][mu][v];
                            }
                            float x2[D];
#pragma unroll
                            for (int mu = 0; mu < D; ++mu) x2[mu] = x[I][mu][v] * x[I][mu][v];
                            float S = x2[0];
#pragma unroll
                            for (int mu = 1; mu < D; ++mu) S = S + x2[mu];
                            const float cc = fmaf(nbd, S, base);
#pragma unroll
                            for (int mu = 0; mu < D; ++mu) y[I][mu][v] = x[I][mu][v] * fmaf(ned, x2[mu], cc);
                        }
                    }
                }
                if constexpr (CO) {
                    // one component at a time: split, and its products for every
                    // row tile (the J fragment reads of the D components are the
                    // same loads, which the compiler merges)
                    constexpr int NP = JS == 1 ? XS : 6;
                    constexpr int pj[6] = {JS == 1 ? 0 : 2, JS == 1 ? 0 : 1, 0, JS == 1 ? 0 : 1, 0, 0};
                    constexpr int px[6] = {JS == 1 ? XS - 1 : 0, JS == 1 ? (XS > 1 ? XS - 2 : 0) : 1,
                                           JS == 1 ? 0 : 2, 0, 1, 0};
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) {
                        XSplit<XS> bm;
                        {
                            float v8[8];
#pragma unroll
                            for (int s = 0; s < 8; ++s) {
                                const int tile = 2 * c + (s >> 2);
                                v8[s] = (tile < NT) ? x[tile < NT ? tile : 0][mu][s & 3] : 0.0f;
                            }
                            split8<XS>(v8, bm);
                        }
                        bf16x8 af[NT][JS];
#pragma unroll
                        for (int I = 0; I < NT; ++I)
#pragma unroll
                            for (int t = 0; t < JS; ++t) af[I][t] = jl[((t * NT + I) * NC + c) * 64 + lane];
#pragma unroll
                        for (int q = 0; q < NP; ++q)
#pragma unroll
                            for (int I = 0; I < NT; ++I)
                                acc[I][mu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[I][pj[q]], bm.t[px[q]],
                                                                                     acc[I][mu], 0, 0, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                } else {
                    // term pairs (J term, state term), smallest first
                    constexpr int NP = JS == 1 ? XS : 6;
                    constexpr int pj[6] = {JS == 1 ? 0 : 2, JS == 1 ? 0 : 1, 0, JS == 1 ? 0 : 1, 0, 0};
                    constexpr int px[6] = {JS == 1 ? XS - 1 : 0, JS == 1 ? (XS > 1 ? XS - 2 : 0) : 1,
                                           JS == 1 ? 0 : 2, 0, 1, 0};
                    // B operands of chunk c straight from the lane's own registers
                    XSplit<XS> bx[D];
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) {
                        float v8[8];
#pragma unroll
                        for (int s = 0; s < 8; ++s) {
                            const int tile = 2 * c + (s >> 2);
                            v8[s] = (tile < NT) ? x[tile < NT ? tile : 0][mu][s & 3] : 0.0f;
                        }
                        split8<XS>(v8, bx[mu]);
                    }
                    // row tiles in groups of TG, each accumulator taking its term
                    // pairs in the order above whatever TG is: with D >= 3 one tile
                    // at a time (its J fragments are the only ones live, and its D
                    // accumulators separate two products into one accumulator);
                    // with D <= 2 all tiles at once (measured faster: 2 D
                    // accumulators between dependent products are too few)
                    constexpr int TG = D >= 3 ? 1 : NT;
#pragma unroll
                    for (int I0 = 0; I0 < NT; I0 += TG) {
                        bf16x8 af[TG][JS];
#pragma unroll
                        for (int i = 0; i < TG; ++i) {
                            const int I = I0 + i < NT ? I0 + i : I0;  // past the end: unused
#pragma unroll
                            for (int t = 0; t < JS; ++t) {
                                if constexpr (JLDS)
                                    af[i][t] = jl[((t * NT + I) * NC + c) * 64 + lane];
                                else
                                    af[i][t] = jr[JLDS ? 0 : t][JLDS ? 0 : I][JLDS ? 0 : c];
                            }
                        }
#pragma unroll
                        for (int q = 0; q < NP; ++q)
#pragma unroll
                            for (int i = 0; i < TG; ++i)
#pragma unroll
                                for (int mu = 0; mu < D; ++mu)
                                    if (I0 + i < NT)
                                        acc[I0 + i][mu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                            af[i][pj[q]], bx[mu].t[px[q]], acc[I0 + i][mu], 0, 0, 0);
                    }
                }
            }

#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int mu = 0; mu < D; ++mu)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (CO && mu == 0) {
                            // the local part, as in the chunks of the other variants
                            float x2[D];
#pragma unroll
                            for (int m = 0; m < D; ++m) x2[m] = x[I][m][v] * x[I][m][v];
                            float S = x2[0];
#pragma unroll
                            for (int m = 1; m < D; ++m) S = S + x2[m];
                            const float cc = fmaf(nbd, S, base);
#pragma unroll
                            for (int m = 0; m < D; ++m) y[I][m][v] = x[I][m][v] * fmaf(ned, x2[m], cc);
                        }
                        x[I][mu][v] = fmaf(ga[mu], acc[I][mu][v], y[I][mu][v]);
                    }
    }

    // ---- store ----
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            if (valid && p < n) {
#pragma unroll
                for (int mu = 0; mu < D; ++mu) a.x[((size_t)p * r + rep) * D + mu] = x[I][mu][v];
            }
        }
}

// One problem: wavefront w of the grid integrates replicas 16 w .. 16 w + 15.
template <int NT, int D, int XS, int JS, bool MAP = false>
__global__ __launch_bounds__(256) void k_integrate_resident(IntegArgs a) {
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int rep0 = wave * 16;
    if (rep0 >= a.r) return;
    integrate_group<NT, D, XS, JS, false, MAP>(a, rep0, nullptr);
}

// Many problems of one variant: a persistent grid whose wavefronts pop work
// items (problem, 16-replica group) from a counter until the list is empty.
// Items are listed longest first by the host.  The counter must be zero at
// launch; the host zeroes it with k_zero_counters in the same stream.  MAP
// selects the round-trip map of Eq. (2) instead of its continuous limit.
template <int NT, int D, int XS, int JS, bool MAP = false>
__global__ __launch_bounds__(256) void k_integrate_persistent(const IntegArgs *__restrict__ tasks,
                                                              const int2 *__restrict__ items, int n_items,
                                                              int *__restrict__ counter) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(counter, 1);
        // wave-uniform from here on: the item and its task live in SGPRs
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (it >= n_items) break;
        const int2 w = items[it];
        const IntegArgs a = tasks[w.x];
        integrate_group<NT, D, XS, JS, false, MAP>(a, w.y * 16, nullptr);
    }
}

// Same, with J shared through LDS: a block of W wavefronts pops work items
// (problem, slab of 16 W replicas), stages the problem's J fragments once,
// and each wavefront integrates its 16 replicas reading J from LDS.  WPE
// wavefronts per SIMD: 2 caps each at 256 registers so that one wave's
// matrix-core work can overlap the other's vector work; 3 caps each at 168,
// for the variants whose step loop still fits (lds3_max_tiles); 1 leaves the
// full register file to a single wave.
template <int NT, int D, int XS, int JS, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_integrate_persistent_lds(const IntegArgs *__restrict__ tasks, const int2 *__restrict__ items, int n_items,
                                int *__restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem[];
    bf16x8 *jl = reinterpret_cast<bf16x8 *>(smem);
    __shared__ int s_item;
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    for (;;) {
        __syncthreads();  // the previous item's LDS reads are done
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int2 w = items[it];
        const IntegArgs a = tasks[w.x];
        stage_j<NT, JS>(a, jl);
        __syncthreads();
        const int rep0 = (w.y * waves + wave) * 16;
        if (rep0 < a.r) integrate_group<NT, D, XS, JS, true>(a, rep0, jl);
    }
}

// ---------------------------------------------------------------------------
// Software-pipelined variant: one wavefront per SIMD, J in the block's LDS.
//
// With the products of a step issued back to back and the vector work of
// the update and the operand split done between steps, a wavefront keeps
// the matrix cores idle during its vector work; two wavefronts per SIMD
// only cover for each other when their phases happen to alternate.  Here a
// single wavefront interleaves the two itself: while chunk c of step k runs
// on the matrix cores it finishes the update of step k-1 for row tiles
// 2c+2 and 2c+3 (whose products completed in step k-1) and splits them into
// the operands of chunk c+1 of step k; in the last chunk, whose products are
// issued tile by tile, it updates tiles 0 and 1 of step k as soon as their
// products are complete and splits the next step's chunk 0.  Step k-1's
// products (being consumed) and step k's (being formed) live in two
// accumulator sets, and two operand sets alternate; the step loop is
// unrolled by two so that every choice of set is static.  Each accumulator
// takes its products in the same order as in every other variant (chunk by
// chunk, state terms smallest first), and the update is the same arithmetic,
// so results are bit-identical.

// The Euler update of one row tile (4 rows x D components of the lane's
// replica) from its products: x <- x (1 + dt (r-1) - dt btil S - dt eta x^2)
// + dt eps alpha_mu G, written as in integrate_group.
template <int D>
__device__ __forceinline__ void pipe_update_tile(float (&xt)[D][4], const f32x4 (&acc)[D], const float (&ga)[D],
                                                 float base, float nbd, float ned) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        float x2[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) x2[mu] = xt[mu][v] * xt[mu][v];
        float S = x2[0];
#pragma unroll
        for (int mu = 1; mu < D; ++mu) S = S + x2[mu];
        const float cc = fmaf(nbd, S, base);
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            const float y = xt[mu][v] * fmaf(ned, x2[mu], cc);
            xt[mu][v] = fmaf(ga[mu], acc[mu][v], y);
        }
    }
}

// Operands of chunk c (row tiles 2c and 2c+1 of the lane's own state).
template <int NT, int D, int XS>
__device__ __forceinline__ void pipe_split_chunk(const float (&x)[NT][D][4], int c, XSplit<XS> (&b)[D]) {
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        float v8[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int tile = 2 * c + (s >> 2);
            v8[s] = (tile < NT) ? x[tile < NT ? tile : 0][mu][s & 3] : 0.0f;
        }
        split8<XS>(v8, b[mu]);
    }
}

// The products of chunk c for every row tile, tile by tile; the chunk-0
// products start from zero.
template <int NT, int D, int XS, int JS>
__device__ __forceinline__ void pipe_products(f32x4 (&acc)[NT][D], const XSplit<XS> (&b)[D], const bf16x8 *jl,
                                              int c, int lane) {
    constexpr int NC = (NT + 1) / 2;
    constexpr int NP = JS == 1 ? XS : 6;
    constexpr int pj[6] = {JS == 1 ? 0 : 2, JS == 1 ? 0 : 1, 0, JS == 1 ? 0 : 1, 0, 0};
    constexpr int px[6] = {JS == 1 ? XS - 1 : 0, JS == 1 ? (XS > 1 ? XS - 2 : 0) : 1, JS == 1 ? 0 : 2, 0, 1, 0};
#pragma unroll
    for (int I = 0; I < NT; ++I) {
        bf16x8 af[JS];
#pragma unroll
        for (int t = 0; t < JS; ++t) af[t] = jl[((t * NT + I) * NC + c) * 64 + lane];
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int mu = 0; mu < D; ++mu)
                acc[I][mu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    af[pj[q]], b[mu].t[px[q]], (c == 0 && q == 0) ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : acc[I][mu], 0, 0,
                    0);
    }
}

// One step of the pipelined loop.  cur receives this step's products; prev
// holds the previous step's (PREV), whose update is finished here for row
// tiles 2 .. NT-1; bx[P] holds this step's chunk-0 operands on entry.  NEXT:
// the last chunk also finishes this step's update of tiles 0 and 1 and
// splits the next step's chunk 0 into bx[(P + NC) & 1].
template <int NT, int D, int XS, int JS, int P, bool PREV, bool NEXT>
__device__ __forceinline__ void pipe_step(float (&x)[NT][D][4], f32x4 (&cur)[NT][D], const f32x4 (&prev)[NT][D],
                                          XSplit<XS> (&bx)[2][D], const float (&ga_cur)[D], const float (&ga_prev)[D],
                                          const bf16x8 *jl, int lane, float base, float nbd, float ned) {
    constexpr int NC = (NT + 1) / 2;
    constexpr int NP = JS == 1 ? XS : 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int bi = (P + c) & 1;
        pipe_products<NT, D, XS, JS>(cur, bx[bi], jl, c, lane);
        if (c + 1 < NC) {
            if constexpr (PREV) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int I = 2 * c + 2 + h;
                    if (I < NT) pipe_update_tile<D>(x[I < NT ? I : 0], prev[I < NT ? I : 0], ga_prev, base, nbd, ned);
                }
            }
            pipe_split_chunk<NT, D, XS>(x, c + 1, bx[bi ^ 1]);
        } else if constexpr (NEXT) {
            pipe_update_tile<D>(x[0], cur[0], ga_cur, base, nbd, ned);
            if (NT > 1) pipe_update_tile<D>(x[NT > 1 ? 1 : 0], cur[NT > 1 ? 1 : 0], ga_cur, base, nbd, ned);
            pipe_split_chunk<NT, D, XS>(x, 0, bx[bi ^ 1]);
        }
        // chunks stay in their order (no code moves across this point); an
        // explicit interleave pattern of products and vector instructions
        // (1:2, 1:4, 1:6) measured slower than the scheduler's own order
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Integrates the 16 replicas rep0 .. rep0+15 of problem a with the pipelined
// step loop; J fragments are read from the block's LDS copy.
template <int NT, int D, int XS, int JS>
__device__ __forceinline__ void integrate_group_pipe(const IntegArgs &a, int rep0, const bf16x8 *jl) {
    const int n = a.n;
    const int r = a.r;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int rep = rep0 + (lane & 15);
    const bool valid = rep < r;

    float x[NT][D][4];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            const bool ok = valid && p < n;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) x[I][mu][v] = ok ? a.x[((size_t)p * r + rep) * D + mu] : 0.0f;
        }
    const float base = valid ? fmaf(a.dt, a.pump[rep] - 1.0f, 1.0f) : 0.0f;
    const float nbd = -(a.dt * a.btil);
    const float ned = -(a.dt * a.eta);
    const float dte = a.dt * a.eps;
    auto weights = [&](int k, float (&ga)[D]) __attribute__((always_inline)) {
        const float *al = a.alpha + (size_t)(a.start_step + k) * D;
#pragma unroll
        for (int mu = 0; mu < D; ++mu)
            ga[mu] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(dte * al[mu])));
    };

    constexpr int NC = (NT + 1) / 2;
    constexpr int P1 = NC & 1;  // chunk-0 operand set of odd steps
    const int steps = a.steps;
    if (steps > 0) {
        f32x4 accA[NT][D], accB[NT][D];
        XSplit<XS> bx[2][D];
        float ga0[D], ga1[D];
        pipe_split_chunk<NT, D, XS>(x, 0, bx[0]);
        weights(0, ga0);
        if (steps == 1) {
            pipe_step<NT, D, XS, JS, 0, false, false>(x, accA, accB, bx, ga0, ga0, jl, lane, base, nbd, ned);
#pragma unroll
            for (int I = 0; I < NT; ++I) pipe_update_tile<D>(x[I], accA[I], ga0, base, nbd, ned);
        } else {
            pipe_step<NT, D, XS, JS, 0, false, true>(x, accA, accB, bx, ga0, ga0, jl, lane, base, nbd, ned);
            int k = 1;
            // pairs of steps (k odd into accB, k + 1 even into accA), each with a successor
            for (; k + 2 < steps; k += 2) {
                asm volatile("" ::: "memory");  // J fragments stay in LDS, read again every step
                weights(k, ga1);
                pipe_step<NT, D, XS, JS, P1, true, true>(x, accB, accA, bx, ga1, ga0, jl, lane, base, nbd, ned);
                asm volatile("" ::: "memory");
                weights(k + 1, ga0);
                pipe_step<NT, D, XS, JS, 0, true, true>(x, accA, accB, bx, ga0, ga1, jl, lane, base, nbd, ned);
            }
            asm volatile("" ::: "memory");
            weights(k, ga1);
            if (k + 1 < steps) {  // two steps left: k into accB, k + 1 (the last) into accA
                pipe_step<NT, D, XS, JS, P1, true, true>(x, accB, accA, bx, ga1, ga0, jl, lane, base, nbd, ned);
                weights(k + 1, ga0);
                pipe_step<NT, D, XS, JS, 0, true, false>(x, accA, accB, bx, ga0, ga1, jl, lane, base, nbd, ned);
#pragma unroll
                for (int I = 0; I < NT; ++I) pipe_update_tile<D>(x[I], accA[I], ga0, base, nbd, ned);
            } else {  // one step left: k (the last) into accB
                pipe_step<NT, D, XS, JS, P1, true, false>(x, accB, accA, bx, ga1, ga0, jl, lane, base, nbd, ned);
#pragma unroll
                for (int I = 0; I < NT; ++I) pipe_update_tile<D>(x[I], accB[I], ga1, base, nbd, ned);
            }
        }
    }

    // the store's addresses are formed here from an opaque base, so that
    // the load's are not kept live through the step loop
    float *xout = a.x;
    int rr = r;
    asm volatile("" : "+s"(xout), "+s"(rr));
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * I + 4 * g + v;
            if (valid && p < n) {
#pragma unroll
                for (int mu = 0; mu < D; ++mu) xout[((size_t)p * rr + rep) * D + mu] = x[I][mu][v];
            }
        }
}

// Many problems of one variant with the pipelined step loop: a block of W
// wavefronts, one per SIMD, pops work items (problem, slab of 16 W
// replicas), stages the problem's J fragments in LDS once, and each
// wavefront integrates its 16 replicas.
template <int NT, int D, int XS, int JS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
void k_integrate_persistent_pipe(const IntegArgs *__restrict__ tasks, const int2 *__restrict__ items, int n_items,
                                 int *__restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem[];
    bf16x8 *jl = reinterpret_cast<bf16x8 *>(smem);
    __shared__ int s_item;
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    for (;;) {
        __syncthreads();  // the previous item's LDS reads are done
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int2 w = items[it];
        const IntegArgs a = tasks[w.x];
        stage_j<NT, JS>(a, jl);
        __syncthreads();
        const int rep0 = (w.y * waves + wave) * 16;
        if (rep0 < a.r) integrate_group_pipe<NT, D, XS, JS>(a, rep0, jl);
    }
}

// Shapes the pipelined variant is built for: two accumulator sets, two
// operand sets and the state within one wavefront's 512 registers.
constexpr bool pipe_supported(int nt, int d, int xs, int js) {
    return js == 1 && (d == 2 || d == 3) && nt >= 2 && nt <= 7 && xs >= 1;
}

template <int NT, int JS>
constexpr size_t lds_j_bytes() {
    return (size_t)JS * NT * ((NT + 1) / 2) * 64 * sizeof(bf16x8);
}

// Largest row-tile count per (d, xs, js) whose three-wavefronts-per-SIMD
// LDS kernel keeps its step loop free of scratch spills (168 registers;
// spills in the set-up before the loop are allowed).
constexpr int lds3_max_tiles(int d, int xs, int js) {
    if (d == 1) return js == 3 ? 8 : 10;
    if (d == 2) return js == 3 ? 5 : 7;
    if (d == 3) return js == 3 ? 3 : 4;
    return 3;
}

template <int NT, int D, int XS, int JS>
constexpr void (*lds3_fn())(const IntegArgs *, const int2 *, int, int *) {
    if constexpr (NT <= lds3_max_tiles(D, XS, JS)) return k_integrate_persistent_lds<NT, D, XS, JS, 3>;
    else return nullptr;
}

struct KernelSet {
    void (*single)(IntegArgs);
    void (*persistent)(const IntegArgs *, const int2 *, int, int *);
    void (*persistent_lds)(const IntegArgs *, const int2 *, int, int *);   // two wavefronts per SIMD
    void (*persistent_lds1)(const IntegArgs *, const int2 *, int, int *);  // one wavefront per SIMD
    size_t lds_bytes;
    void (*single_map)(IntegArgs);  // round-trip map form (single coupling term only)
    void (*persistent_map)(const IntegArgs *, const int2 *, int, int *);  // same, many problems
    void (*persistent_pipe)(const IntegArgs *, const int2 *, int, int *);  // pipelined, one wavefront per SIMD
    void (*persistent_lds3)(const IntegArgs *, const int2 *, int, int *);  // three wavefronts per SIMD
};

// Largest row-tile count per (d, xs, js) that compiles without scratch
// spills (state, accumulators and J fragments within 512 registers).
constexpr int resident_max_tiles(int d, int xs, int js) {
    if (js == 3) return d == 1 ? 8 : (d <= 3 ? 6 : 5);
    if (d == 1) return 12;
    if (d == 2) return xs == 3 ? 9 : 10;
    if (d == 3) return 8;
    return 7;
}

template <int NT, int D, int XS, int JS>
constexpr void (*pipe_fn())(const IntegArgs *, const int2 *, int, int *) {
    if constexpr (pipe_supported(NT, D, XS, JS)) return k_integrate_persistent_pipe<NT, D, XS, JS>;
    else return nullptr;
}

template <int NT, int D, int XS, int JS>
KernelSet variant_or_null() {
    if constexpr (NT <= resident_max_tiles(D, XS, JS))
        return KernelSet{k_integrate_resident<NT, D, XS, JS>, k_integrate_persistent<NT, D, XS, JS>,
                         k_integrate_persistent_lds<NT, D, XS, JS, 2>, k_integrate_persistent_lds<NT, D, XS, JS, 1>,
                         lds_j_bytes<NT, JS>(),
                         (JS == 1 && NT <= kMapMaxTiles) ? k_integrate_resident<NT, D, XS, JS, true> : nullptr,
                         (JS == 1 && NT <= kMapMaxTiles) ? k_integrate_persistent<NT, D, XS, JS, true> : nullptr,
                         pipe_fn<NT, D, XS, JS>(), lds3_fn<NT, D, XS, JS>()};
    else
        return KernelSet{nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
}

// One translation unit per (D, XS, JS) instantiates all tile counts.
template <int D, int XS, int JS>
KernelSet lookup_tiles(int tiles) {
    switch (tiles) {
        case 1: return variant_or_null<1, D, XS, JS>();
        case 2: return variant_or_null<2, D, XS, JS>();
        case 3: return variant_or_null<3, D, XS, JS>();
        case 4: return variant_or_null<4, D, XS, JS>();
        case 5: return variant_or_null<5, D, XS, JS>();
        case 6: return variant_or_null<6, D, XS, JS>();
        case 7: return variant_or_null<7, D, XS, JS>();
        case 8: return variant_or_null<8, D, XS, JS>();
        case 9: return variant_or_null<9, D, XS, JS>();
        case 10: return variant_or_null<10, D, XS, JS>();
        case 11: return variant_or_null<11, D, XS, JS>();
        case 12: return variant_or_null<12, D, XS, JS>();
        default: return KernelSet{nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
    }
}

#define CHYM_DECLARE_LOOKUP(D, XS, JS) KernelSet lookup_resident_##D##_##XS##_##JS(int tiles);
CHYM_DECLARE_LOOKUP(1, 3, 1) CHYM_DECLARE_LOOKUP(1, 1, 1) CHYM_DECLARE_LOOKUP(1, 3, 3)
CHYM_DECLARE_LOOKUP(2, 3, 1) CHYM_DECLARE_LOOKUP(2, 1, 1) CHYM_DECLARE_LOOKUP(2, 3, 3)
CHYM_DECLARE_LOOKUP(3, 3, 1) CHYM_DECLARE_LOOKUP(3, 1, 1) CHYM_DECLARE_LOOKUP(3, 3, 3)
CHYM_DECLARE_LOOKUP(4, 3, 1) CHYM_DECLARE_LOOKUP(4, 1, 1) CHYM_DECLARE_LOOKUP(4, 3, 3)
#undef CHYM_DECLARE_LOOKUP

}  // namespace chym

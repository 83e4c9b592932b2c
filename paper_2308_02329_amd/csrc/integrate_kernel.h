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
// lane's own registers with no LDS round trip and no shuffle, and J is
// gathered once per work item into registers in the matching (permuted)
// order as A fragments.
//
// Float32 form: x is fed as the exact sum x = hi + mid + lo of three bf16
// terms (each residual of a round-to-nearest bf16 has at most 16, then 8,
// significant bits), so every product J_pq x_q is formed exactly and summed
// in float32.  An integer J is exact in bf16; a float J is split the same
// way and the six leading cross terms are kept (error ~2^-24 relative).
// BF16 form: one bf16 term each.
//
// The Euler update (pump gain, coupling with the annealing weight, nonlocal
// loss, local saturation) is fused after the contraction and works on the
// accumulator registers in place; the whole step loop runs inside the
// kernel, with no LDS, no barrier and no global-memory traffic per step
// except the D annealing weights alpha[k][mu] (scalar loads).  Wavefronts
// never wait on each other, so work is handed out per 16-replica group.
#pragma once

#include "chym_internal.h"

namespace chym {


template <int XS>
struct XSplit {
    bf16x8 t[XS];
};

__device__ __forceinline__ float bf_to_f(__bf16 h) { return (float)h; }

// Loads one coupling value as float (0 outside the n x n matrix).
__device__ __forceinline__ float j_at(const IntegArgs &a, int p, int q) {
    if (p >= a.n || q >= a.n) return 0.0f;
    return (a.j_dtype == CHYM_J_I8) ? (float)reinterpret_cast<const int8_t *>(a.j)[(size_t)p * a.n + q]
                                    : reinterpret_cast<const float *>(a.j)[(size_t)p * a.n + q];
}

// Integrates the 16 replicas rep0 .. rep0+15 of problem a for a.steps steps.
// Called by one whole wavefront; uses no LDS and no barrier.
template <int NT, int D, int XS, int JS>
__device__ __forceinline__ void integrate_group(const IntegArgs &a, int rep0) {
    constexpr int NC = (NT + 1) / 2;
    const int n = a.n;
    const int r = a.r;
    const int lane = threadIdx.x & 63;
    const int jcol = lane & 15;
    const int g = lane >> 4;
    const int rep = rep0 + jcol;
    const bool valid = rep < r;

    // ---- J as MFMA A fragments, held in registers for the whole run ----
    // fragment (I, c), lane (i, g), slot s: J[16 I + i][32 c + 16 (s >> 2) + 4 g + (s & 3)]
    bf16x8 jf[JS][NT][NC];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const float v = j_at(a, 16 * I + jcol, 32 * c + 16 * (s >> 2) + 4 * g + (s & 3));
                if constexpr (JS == 1) {
                    jf[0][I][c][s] = (__bf16)v;
                } else {
                    const __bf16 h = (__bf16)v;
                    const float r1 = v - bf_to_f(h);
                    const __bf16 m = (__bf16)r1;
                    const float r2 = r1 - bf_to_f(m);
                    jf[0][I][c][s] = h;
                    jf[1][I][c][s] = m;
                    jf[2][I][c][s] = (__bf16)r2;
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

    const float base = valid ? fmaf(a.dt, a.pump[rep] - 1.0f, 1.0f) : 0.0f;  // 1 + dt (r_i - 1)
    const float nbd = -(a.dt * a.btil);
    const float ned = -(a.dt * a.eta);
    const float dte = a.dt * a.eps;

    for (int k = 0; k < a.steps; ++k) {
        const float *al = a.alpha + (size_t)(a.start_step + k) * D;
        float ga[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) ga[mu] = dte * al[mu];

        f32x4 acc[NT][D];
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int mu = 0; mu < D; ++mu) acc[I][mu] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // B operands of chunk c straight from the lane's own registers
            XSplit<XS> bx[D];
#pragma unroll
            for (int mu = 0; mu < D; ++mu)
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int tile = 2 * c + (s >> 2);
                    const float v = (tile < NT) ? x[tile < NT ? tile : 0][mu][s & 3] : 0.0f;
                    if constexpr (XS == 1) {
                        bx[mu].t[0][s] = (__bf16)v;
                    } else {
                        const __bf16 h = (__bf16)v;
                        const float r1 = v - bf_to_f(h);
                        const __bf16 m = (__bf16)r1;
                        const float r2 = r1 - bf_to_f(m);
                        bx[mu].t[0][s] = h;
                        bx[mu].t[1][s] = m;
                        bx[mu].t[2][s] = (__bf16)r2;
                    }
                }
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int mu = 0; mu < D; ++mu) {
                    f32x4 cacc = acc[I][mu];
                    if constexpr (JS == 1) {
                        // smallest terms first
#pragma unroll
                        for (int t = XS - 1; t >= 0; --t)
                            cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[0][I][c], bx[mu].t[t], cacc, 0, 0, 0);
                    } else {
                        cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[2][I][c], bx[mu].t[0], cacc, 0, 0, 0);
                        cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[1][I][c], bx[mu].t[1], cacc, 0, 0, 0);
                        cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[0][I][c], bx[mu].t[2], cacc, 0, 0, 0);
                        cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[1][I][c], bx[mu].t[0], cacc, 0, 0, 0);
                        cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[0][I][c], bx[mu].t[1], cacc, 0, 0, 0);
                        cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(jf[0][I][c], bx[mu].t[0], cacc, 0, 0, 0);
                    }
                    acc[I][mu] = cacc;
                }
        }

        // ---- fused Euler update on the accumulator tiles ----
        // x <- x (1 + dt (r-1) - dt btil S - dt eta x^2) + dt eps alpha_mu G
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float x2[D];
#pragma unroll
                for (int mu = 0; mu < D; ++mu) x2[mu] = x[I][mu][v] * x[I][mu][v];
                float S = x2[0];
#pragma unroll
                for (int mu = 1; mu < D; ++mu) S = S + x2[mu];
                const float cc = fmaf(nbd, S, base);
#pragma unroll
                for (int mu = 0; mu < D; ++mu) {
                    const float t = fmaf(ned, x2[mu], cc);
                    const float y = x[I][mu][v] * t;
                    x[I][mu][v] = fmaf(ga[mu], acc[I][mu][v], y);
                }
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
template <int NT, int D, int XS, int JS>
__global__ __launch_bounds__(256) void k_integrate_resident(IntegArgs a) {
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int rep0 = wave * 16;
    if (rep0 >= a.r) return;
    integrate_group<NT, D, XS, JS>(a, rep0);
}

// Many problems of one variant: a persistent grid whose wavefronts pop work
// items (problem, 16-replica group) from a counter until the list is empty.
// Items are listed longest first by the host.  The counter must be zero at
// launch; the host zeroes it with k_zero_counters in the same stream.
template <int NT, int D, int XS, int JS>
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
        integrate_group<NT, D, XS, JS>(a, w.y * 16);
    }
}


struct KernelPair {
    void (*single)(IntegArgs);
    void (*persistent)(const IntegArgs *, const int2 *, int, int *);
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
KernelPair variant_or_null() {
    if constexpr (NT <= resident_max_tiles(D, XS, JS))
        return KernelPair{k_integrate_resident<NT, D, XS, JS>, k_integrate_persistent<NT, D, XS, JS>};
    else
        return KernelPair{nullptr, nullptr};
}

// One translation unit per (D, XS, JS) instantiates all tile counts.
template <int D, int XS, int JS>
KernelPair lookup_tiles(int tiles) {
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
        default: return KernelPair{nullptr, nullptr};
    }
}

#define CHYM_DECLARE_LOOKUP(D, XS, JS) KernelPair lookup_resident_##D##_##XS##_##JS(int tiles);
CHYM_DECLARE_LOOKUP(1, 3, 1) CHYM_DECLARE_LOOKUP(1, 1, 1) CHYM_DECLARE_LOOKUP(1, 3, 3)
CHYM_DECLARE_LOOKUP(2, 3, 1) CHYM_DECLARE_LOOKUP(2, 1, 1) CHYM_DECLARE_LOOKUP(2, 3, 3)
CHYM_DECLARE_LOOKUP(3, 3, 1) CHYM_DECLARE_LOOKUP(3, 1, 1) CHYM_DECLARE_LOOKUP(3, 3, 3)
CHYM_DECLARE_LOOKUP(4, 3, 1) CHYM_DECLARE_LOOKUP(4, 1, 1) CHYM_DECLARE_LOOKUP(4, 3, 3)
#undef CHYM_DECLARE_LOOKUP

}  // namespace chym

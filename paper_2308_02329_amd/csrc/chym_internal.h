// Internal declarations of libchym (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/chym.h"

namespace chym {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// Value of an OCP E4M3 (e4m3fn) byte: sign, 4 exponent bits (bias 7), 3
// mantissa bits; exponent field 0 holds the subnormals m * 2^-9; 0x7f and
// 0xff are NaN (the format has no infinities).
__device__ __forceinline__ float e4m3_value(uint32_t b) {
    const uint32_t mag = b & 0x7fu;
    float v;
    if (mag == 0x7fu)
        v = __builtin_nanf("");
    else if (mag < 8u)
        v = (float)mag * 0x1p-9f;
    else
        v = __uint_as_float((((mag >> 3) + 120u) << 23) | ((mag & 7u) << 20));
    return (b & 0x80u) ? -v : v;
}

// Nearest E4M3 code of a (|a| <= 448 assumed), ties to even; sign from the
// float's sign bit.
__device__ __forceinline__ uint32_t e4m3_code(float v) {
    const uint32_t bits = __float_as_uint(v);
    const uint32_t sign = (bits >> 24) & 0x80u;
    const float a = fabsf(v);
    uint32_t code;
    if (a < 0x1p-6f) {
        // subnormal spacing 2^-9; a * 512 is exact, rintf rounds to even
        code = (uint32_t)rintf(a * 512.0f);  // 8 is the smallest normal, 0x08
    } else {
        const uint32_t ab = __float_as_uint(a);
        int e = (int)(ab >> 23) - 127;
        const uint32_t mant = ab & 0x7fffffu;
        uint32_t m3 = mant >> 20;
        const uint32_t rest = mant & 0xfffffu;
        if (rest > 0x80000u || (rest == 0x80000u && (m3 & 1u))) ++m3;
        if (m3 == 8u) {
            m3 = 0u;
            ++e;
        }
        code = ((uint32_t)(e + 7) << 3) | m3;
    }
    return sign | code;
}

// Least e with amax <= 448 * 2^e (0 for amax = 0): the power-of-two row
// scale that puts a row's largest magnitude at the top E4M3 binade.
__device__ __forceinline__ int e4m3_row_exponent(float amax) {
    if (!(amax > 0.0f)) return 0;
    int k;
    frexpf(amax, &k);  // amax = f 2^k, f in [0.5, 1)
    int e = k - 9;     // 448 * 2^(k - 9) = 0.875 * 2^k: the answer is e or e + 1
    if (amax > ldexpf(448.0f, e)) ++e;
    if (amax <= ldexpf(448.0f, e - 1)) --e;
    return e;
}

// Sparse (ELL) couplings, int32 [n + 1][2 w]: row 0 = {n, w, ...}; row p + 1
// = w columns, then w float32 couplings (bit patterns).
struct EllView {
    const int *rows;
    int w;
    __device__ __forceinline__ const int *row(int p) const { return rows + (size_t)(p + 1) * 2 * w; }
};
// A header that does not describe an n-row matrix reads as no couplings.
__device__ __forceinline__ EllView ell_view(const void *j, int n) {
    const int *h = reinterpret_cast<const int *>(j);
    return EllView{h, (h[0] == n && h[1] > 0) ? h[1] : 0};
}

// Coupling J_pq of an n x n matrix stored as j_dtype, as float (exact for
// every storage type but float32 input, where it is the stored value).
__device__ __forceinline__ float coupling(const void *j, int j_dtype, int n, int p, int q) {
    const size_t i = (size_t)p * n + q;
    switch (j_dtype) {
        case CHYM_J_I8: return (float)reinterpret_cast<const int8_t *>(j)[i];
        case CHYM_J_F32: return reinterpret_cast<const float *>(j)[i];
        case CHYM_J_BF16: return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(j)[i] << 16);
        default: {
            const uint8_t *b = reinterpret_cast<const uint8_t *>(j);
            const uint32_t e = b[(size_t)n * n + p];
            if (e == 0xffu) return __builtin_nanf("");
            return ldexpf(e4m3_value(b[i]), (int)e - 127);
        }
    }
}

// Largest row-tile count (16 rows per tile) of the register-resident
// integrator for d components, xs state terms and js J terms (0 if none).
int resident_tile_limit(int d, int xs, int js);

// Arguments of one integration launch (one problem, one replica block).
struct IntegArgs {
    const void *j;
    const float *pump;
    float *x;
    const float *alpha;
    int32_t n, d, r, steps, start_step, j_dtype;
    float eps, btil, eta, dt;
    // round-trip map form only: kappa L of the medium, and the constant part
    // (1 - loss)(1 - b) of the per-round-trip factor
    float kl, c0;
};

// Host-side launcher of the resident integrator for one (tiles, d, xs, js)
// variant; returns hipSuccess or the launch error.
hipError_t launch_integrate(int tiles, int d, int xs, int js, int waves_per_block,
                            const IntegArgs &a, hipStream_t stream, bool *supported);
// The round-trip map form (single coupling term only), up to this many row
// tiles (the medium's gain per amplitude needs registers the largest
// register-resident shapes do not have).
constexpr int kMapMaxTiles = 7;
hipError_t launch_integrate_map(int tiles, int d, int xs, int waves_per_block, const IntegArgs &a,
                                hipStream_t stream, bool *supported);
// Many map problems of one variant: a persistent grid of 256-thread blocks
// whose wavefronts pop items (task, 16-replica group) from *counter (zero at
// launch) until n_items are taken.
bool map_variant_exists(int tiles, int d, int xs);
hipError_t map_persistent_occupancy(int tiles, int d, int xs, int *blocks_per_cu);
hipError_t launch_integrate_map_persistent(int tiles, int d, int xs, int blocks, const IntegArgs *tasks,
                                           const int2 *items, int n_items, int *counter, hipStream_t stream);
bool integrate_variant_exists(int tiles, int d, int xs, int js);
// Persistent kernel kinds: J gathered into each wavefront's registers, work
// items of 16 replicas; or J staged in LDS per block, work items of
// 16 * waves_per_block replicas.
constexpr int kKernelRegJ = 0;
constexpr int kKernelLdsJ = 1;   // two wavefronts per SIMD
constexpr int kKernelLdsJ1 = 2;  // one wavefront per SIMD
constexpr int kKernelPipe = 3;   // one wavefront per SIMD, update and split interleaved with the products
constexpr int kKernelLdsJ3 = 4;  // three wavefronts per SIMD
// Whether a persistent kernel of this kind is built for the shape (the
// pipelined kind exists for some shapes only).
bool persistent_kind_exists(int tiles, int d, int xs, int js, int kind);
hipError_t persistent_occupancy(int tiles, int d, int xs, int js, int kind, int waves_per_block, int *blocks_per_cu);
hipError_t launch_zero_counters(int *counters, int n, hipStream_t stream);
// FP8 (E4M3 + per-row power-of-two) packing of a float32 coupling matrix.
hipError_t launch_quantize_fp8(int n, const float *j, uint8_t *out, hipStream_t stream);
// Sparse (ELL) couplings: replicas per block for n, d (0 if n is too large),
// and the gather integrator.
int ell_replicas_per_block(int n, int d);
hipError_t launch_integrate_ell(const IntegArgs &a, hipStream_t stream);
// LDS bytes of one block of the gather integrator for n, d; the persistent
// form over many problems of one d (items: task, replica block of
// ell_replicas_per_block(n, d) replicas), launched with the largest LDS
// size of its tasks.
size_t ell_lds_bytes(int n, int d);
hipError_t ell_persistent_occupancy(int d, size_t lds, int *blocks_per_cu);
hipError_t launch_integrate_ell_persistent(int d, int blocks, size_t lds, const IntegArgs *tasks, const int2 *items,
                                           int n_items, int *counter, hipStream_t stream);
// Synthetic timing problem for the autotuner.
hipError_t launch_fill_probe(void *j, int j_dtype, int n, float *pump, int r, float *alpha, int na,
                             hipStream_t stream);
hipError_t launch_fill_state(float *x, size_t nx, hipStream_t stream);
hipError_t launch_split3(const float *x, int64_t n, uint16_t *hi, uint16_t *mid, uint16_t *lo, hipStream_t stream);
// Persistent launch over a work list: items[i] = (task index, replica slab).
hipError_t launch_integrate_persistent(int tiles, int d, int xs, int js, int kind, int waves_per_block, int blocks,
                                       const IntegArgs *tasks, const int2 *items, int n_items, int *counter,
                                       hipStream_t stream);

// Per-task arguments of the batched scoring kernels.
struct ScoreArgs {
    const float *x;
    const void *j;
    uint64_t *spins;
    int32_t *e_i32;
    double *e_f64;
    double *e_hs;
    double *extra;
    uint8_t *diverged;
    int32_t n, d, r, j_dtype;
};

// Readout, Ising energy and hyperspin energy of every replica of every task
// (first = replica prefix table, first[n_tasks] = total_replicas).
hipError_t launch_score_batched(const ScoreArgs *tasks, const int64_t *first, int n_tasks, int64_t total_replicas,
                                int max_nd, bool any_readout, bool any_ising, bool any_hs, int cus,
                                hipStream_t stream);

// Streamed-J slab integrator (large n).  Tiles of 16 rows; kSlabMaxLds
// bounds the LDS operand area of one column slab (beyond it the float32 form
// holds one component at a time and makes d passes over J per step).
constexpr size_t kSlabMaxLds = 159 * 1024;  // 160 KiB per CU, less room for static LDS
// Blocks of eight or sixteen wavefronts (kSlabWaves8, kSlabWaves16); the
// sixteen-wavefront shapes are built for the bf16 form, up to 32 tiles (64
// at d <= 2).
constexpr int kSlabWaves8 = 8;
constexpr int kSlabWaves16 = 16;
int slab_tpw_for(int tiles, int waves);
size_t slab_lds_bytes(int tiles, int d, int xs);
size_t slab_jfrag_bytes(int tiles, int js);
bool slab_variant_exists(int tiles, int d, int xs, int js);  // the eight-wavefront shape
bool slab_shape_exists(int tiles, int d, int xs, int js, int waves);
hipError_t launch_stage_jfrag(const IntegArgs &a, int js, void *out, hipStream_t stream);
// Stages the couplings of the tasks list[0 .. n) of a batch (all with js
// coupling terms) into stages[task], ncps[task] chunks each; tasks, list,
// ncps and stages are device arrays.
hipError_t launch_stage_batched(int js, const IntegArgs *tasks, const int *list, int n, const int *ncps,
                                unsigned char *const *stages, hipStream_t stream);
hipError_t launch_integrate_slab(int tiles, int d, int xs, int js, int waves, const IntegArgs &a, const void *jfrag,
                                 hipStream_t stream);
hipError_t slab_occupancy(int tiles, int d, int xs, int js, int waves, size_t lds, int *blocks_per_cu);
hipError_t launch_integrate_slab_persistent(int tiles, int d, int xs, int js, int waves, size_t lds, int blocks,
                                            const IntegArgs *tasks, const int2 *items, int n_items, int *counter,
                                            const void *const *jfs, const int *ncps, hipStream_t stream);

// Learned early restart: trajectory features and the MLP.
hipError_t launch_features(int n, int d, int r, const void *j, int j_dtype, const float *x, uint64_t *prev,
                           float *feat, int feat_stride, int feat_off, hipStream_t stream);
hipError_t launch_sign_words(int n, int d, int r, const float *x, uint64_t *words, hipStream_t stream);
hipError_t launch_standardize(int groups, int group, const float *in, float *out, hipStream_t stream);
hipError_t launch_select_top(int groups, int group, int keep, const float *score, int32_t *idx, hipStream_t stream);
hipError_t launch_gather_replicas(int n, int d, int r_src, const float *x_src, const float *pump_src, int m,
                                  const int32_t *idx, float *x_dst, float *pump_dst, hipStream_t stream);
int mlp_param_count();
size_t mlp_backward_scratch_floats(int batch);
hipError_t launch_mlp_forward(int batch, const float *feat, const void *wb, float *logit, float *h1, float *h2,
                              hipStream_t stream);
hipError_t launch_mlp_backward(int batch, const float *feat, const float *label, const void *wb, const float *logit,
                               const float *h1, const float *h2, float *scratch, float *grad, float *loss,
                               hipStream_t stream);
hipError_t launch_mlp_adam(float *wm, void *wb, float *m, float *v, const float *grad, float lr, float b1, float b2,
                           float eps, int t, hipStream_t stream);
hipError_t launch_to_bf16(const float *src, void *dst, int n, hipStream_t stream);

hipError_t launch_readout(int n, int d, int r, const float *x, uint64_t *spins, double *extra,
                          uint8_t *diverged, hipStream_t stream);
hipError_t launch_ising_energy(int n, int r, const void *j, int j_dtype, const uint64_t *spins,
                               int32_t *e_i32, double *e_f64, hipStream_t stream);
hipError_t launch_hs_energy(int n, int d, int r, const void *j, int j_dtype, const float *x,
                            double *e_hs, hipStream_t stream);

}  // namespace chym

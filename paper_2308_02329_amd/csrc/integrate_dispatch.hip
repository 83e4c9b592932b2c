// Host-side dispatch of the register-resident integrator variants.
#include "integrate_slab.h"

namespace chym {

typedef KernelSet KernelFn;

static KernelFn lookup(int tiles, int d, int xs, int js) {
#define CHYM_PICK(D, XS, JS) \
    if (d == D && xs == XS && js == JS) return lookup_resident_##D##_##XS##_##JS(tiles);
    CHYM_PICK(1, 3, 1) CHYM_PICK(1, 1, 1) CHYM_PICK(1, 3, 3)
    CHYM_PICK(2, 3, 1) CHYM_PICK(2, 1, 1) CHYM_PICK(2, 3, 3)
    CHYM_PICK(3, 3, 1) CHYM_PICK(3, 1, 1) CHYM_PICK(3, 3, 3)
    CHYM_PICK(4, 3, 1) CHYM_PICK(4, 1, 1) CHYM_PICK(4, 3, 3)
#undef CHYM_PICK
    return KernelSet{nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
}

int resident_tile_limit(int d, int xs, int js) {
    return (d >= 1 && d <= 4) ? resident_max_tiles(d, xs, js) : 0;
}

// ------------------------------------------------------------ slab kernels
static SlabKernels lookup_slab_shape(int tpw, int waves, int d, int xs, int js, bool cp) {
#define CHYM_PICK(D, XS, JS) \
    if (d == D && xs == XS && js == JS) return lookup_slab_##D##_##XS##_##JS(tpw, waves, cp);
    CHYM_PICK(1, 3, 1) CHYM_PICK(1, 1, 1) CHYM_PICK(1, 3, 3)
    CHYM_PICK(2, 3, 1) CHYM_PICK(2, 1, 1) CHYM_PICK(2, 3, 3)
    CHYM_PICK(3, 3, 1) CHYM_PICK(3, 1, 1) CHYM_PICK(3, 3, 3)
    CHYM_PICK(4, 3, 1) CHYM_PICK(4, 1, 1) CHYM_PICK(4, 3, 3)
#undef CHYM_PICK
    return SlabKernels{nullptr, nullptr, 0};
}

// Tiles per wavefront of the slab kernel for a tile count and block size
// (eight or sixteen wavefronts); 0 when no shape holds that many tiles.
int slab_tpw_for(int tiles, int waves) {
    const int per = (tiles + waves - 1) / waves;
    if (waves == 8) return per <= 4 ? 4 : (per <= 8 ? 8 : 0);
    if (waves == 16) return per <= 1 ? 1 : (per <= 2 ? 2 : (per <= 4 ? 4 : 0));
    return 0;
}

// The float32 form takes component passes where the operand of all d
// components exceeds the LDS budget (the bf16 form's always fits).
static bool slab_component_passes(int tiles, int d, int xs) {
    return xs == 3 && d > 1 && (size_t)((tiles + 1) / 2) * d * xs * 64 * sizeof(bf16x8) > kSlabMaxLds;
}

static SlabKernels lookup_slab(int tiles, int d, int xs, int js, int waves) {
    const int tpw = slab_tpw_for(tiles, waves);
    if (tpw == 0) return SlabKernels{nullptr, nullptr, 0};
    return lookup_slab_shape(tpw, waves, d, xs, js, slab_component_passes(tiles, d, xs));
}

size_t slab_lds_bytes(int tiles, int d, int xs) {
    const int dp = slab_component_passes(tiles, d, xs) ? 1 : d;
    return (size_t)((tiles + 1) / 2) * dp * xs * 64 * sizeof(bf16x8);
}

// The fragments, plus kSlabRingChunks chunks of padding: the streamed-J
// kernel's prefetch ring refills unconditionally, so around the last tile it
// loads (and discards) up to that many chunks past the staged data.  Their
// offsets travel in the scalar operand of the buffer load, which the range
// check of the buffer resource does not cover; the padding keeps those loads
// inside the workspace.
size_t slab_jfrag_bytes(int tiles, int js) {
    return stage_frag_offset(tiles) + ((size_t)tiles * ((tiles + 1) / 2) + kSlabRingChunks) * js * 64 * sizeof(bf16x8);
}

bool slab_variant_exists(int tiles, int d, int xs, int js) { return slab_shape_exists(tiles, d, xs, js, 8); }

bool slab_shape_exists(int tiles, int d, int xs, int js, int waves) {
    return slab_lds_bytes(tiles, d, xs) <= kSlabMaxLds && lookup_slab(tiles, d, xs, js, waves).single != nullptr;
}

// Decides the staging format of the couplings, checked element by element:
// E2M1 codes when every coupling is -1, 0 or +1; else E4M3 bytes when every
// row is a set of E4M3 values times one power of two (the row scale, chosen
// as in the FP8 quantizer; FP8 storage always qualifies); else bf16.
// Writes the header and the row scales.  Run by one block of 1024 threads:
// wavefront w takes rows w, w + 16, ...  (Batches only: a single problem's
// staging is always bf16, k_stage_bf16_header.)
__device__ __forceinline__ void stage_prep_block(const IntegArgs &a, int tiles, unsigned char *__restrict__ stage) {
    __shared__ int s_ok, s_pm1;
    if (threadIdx.x == 0) {
        s_ok = 1;
        s_pm1 = 1;
    }
    __syncthreads();
    float *scale = reinterpret_cast<float *>(stage + kStageHeader);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int n = a.n;
    bool ok = true, pm1 = true;
    for (int p = w; p < tiles * 16; p += 16) {
        float sc = 1.0f;
        if (p < n) {
            if (a.j_dtype == CHYM_J_FP8) {
                const uint32_t e = reinterpret_cast<const uint8_t *>(a.j)[(size_t)n * n + p];
                sc = e == 0xffu ? __builtin_nanf("") : ldexpf(1.0f, (int)e - 127);
                for (int q = lane; q < n; q += 64) {
                    const float v = coupling(a.j, a.j_dtype, n, p, q);
                    if (!(v == 0.0f || v == 1.0f || v == -1.0f)) pm1 = false;
                }
            } else {
                float amax = 0.0f;
                bool fin = true;
                for (int q = lane; q < n; q += 64) {
                    const float v = coupling(a.j, a.j_dtype, n, p, q);
                    fin = fin && __builtin_isfinite(v);
                    amax = fmaxf(amax, fabsf(v));
                    if (!(v == 0.0f || v == 1.0f || v == -1.0f)) pm1 = false;
                }
                for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
                const int e = e4m3_row_exponent(amax);
                if (!__all(fin) || e < -126 || e > 127) {
                    ok = false;
                } else {
                    sc = ldexpf(1.0f, e);
                    for (int q = lane; q < n; q += 64) {
                        const float v = coupling(a.j, a.j_dtype, n, p, q);
                        if (ldexpf(e4m3_value(e4m3_code(ldexpf(v, -e))), e) != v) ok = false;
                    }
                }
            }
        }
        if (lane == 0) scale[p] = sc;
    }
    if (!ok) atomicAnd(&s_ok, 0);
    if (!pm1) atomicAnd(&s_pm1, 0);
    __syncthreads();
    if (threadIdx.x == 0)
        *reinterpret_cast<int *>(stage) = s_pm1 ? kStageE2M1
                                                : ((a.j_dtype == CHYM_J_FP8 || s_ok) ? kStageE4M3 : kStageBf16);
}

// A single problem's staging header: bf16 fragments.
__global__ void k_stage_bf16_header(unsigned char *__restrict__ stage) {
    if (threadIdx.x == 0) *reinterpret_cast<int *>(stage) = kStageBf16;
}

// The same for the tasks list[0 .. n) of a batch, one block each.
__global__ __launch_bounds__(1024) void k_stage_prep_batched(const IntegArgs *__restrict__ tasks,
                                                             const int *__restrict__ list,
                                                             unsigned char *const *__restrict__ stages) {
    const int t = list[blockIdx.x];
    const IntegArgs a = tasks[t];
    stage_prep_block(a, (a.n + 15) / 16, stages[t]);
}

hipError_t launch_stage_batched(int js, const IntegArgs *tasks, const int *list, int n, const int *ncps,
                                unsigned char *const *stages, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    constexpr int kBlocksPerTask = 32;  // 8192 threads share a task's fragment slots
    if (js == 3) {
        hipLaunchKernelGGL(k_stage_jfrag_batched<3>, dim3(n * kBlocksPerTask), dim3(256), 0, stream, tasks, list,
                           kBlocksPerTask, ncps, stages);
    } else {
        hipLaunchKernelGGL(k_stage_prep_batched, dim3(n), dim3(1024), 0, stream, tasks, list, stages);
        hipLaunchKernelGGL(k_stage_jfrag_batched<1>, dim3(n * kBlocksPerTask), dim3(256), 0, stream, tasks, list,
                           kBlocksPerTask, ncps, stages);
    }
    return hipGetLastError();
}

hipError_t launch_stage_jfrag(const IntegArgs &a, int js, void *out, hipStream_t stream) {
    const int nt = (a.n + 15) / 16;
    const int ncp = (nt + 1) / 2;
    const int total = nt * ncp * 64;
    const int grid = (total + 255) / 256;
    unsigned char *stage = reinterpret_cast<unsigned char *>(out);
    if (js == 3) {
        hipLaunchKernelGGL(k_stage_jfrag<3>, dim3(grid), dim3(256), 0, stream, a, ncp, stage);
    } else {
        hipLaunchKernelGGL(k_stage_bf16_header, dim3(1), dim3(64), 0, stream, stage);
        hipLaunchKernelGGL(k_stage_jfrag<1>, dim3(grid), dim3(256), 0, stream, a, ncp, stage);
    }
    return hipGetLastError();
}

static hipError_t slab_prepare(const void *fn, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_integrate_slab(int tiles, int d, int xs, int js, int waves, const IntegArgs &a, const void *jfrag,
                                 hipStream_t stream) {
    SlabKernels k = lookup_slab(tiles, d, xs, js, waves);
    if (!k.single) return hipErrorInvalidDeviceFunction;
    const size_t lds = slab_lds_bytes(tiles, d, xs);
    hipError_t e = slab_prepare(reinterpret_cast<const void *>(k.single), lds);
    if (e != hipSuccess) return e;
    const int blocks = (a.r + 15) / 16;
    hipLaunchKernelGGL(k.single, dim3(blocks), dim3(64 * k.waves), lds, stream, a,
                       reinterpret_cast<const unsigned char *>(jfrag),
                       (tiles + 1) / 2);
    return hipGetLastError();
}

hipError_t slab_occupancy(int tiles, int d, int xs, int js, int waves, size_t lds, int *blocks_per_cu) {
    *blocks_per_cu = 0;
    SlabKernels k = lookup_slab(tiles, d, xs, js, waves);
    if (!k.persistent) return hipErrorInvalidDeviceFunction;
    hipError_t e = slab_prepare(reinterpret_cast<const void *>(k.persistent), lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k.persistent, 64 * k.waves, lds);
}

hipError_t launch_integrate_slab_persistent(int tiles, int d, int xs, int js, int waves, size_t lds, int blocks,
                                            const IntegArgs *tasks, const int2 *items, int n_items, int *counter,
                                            const void *const *jfs, const int *ncps, hipStream_t stream) {
    SlabKernels k = lookup_slab(tiles, d, xs, js, waves);
    if (!k.persistent) return hipErrorInvalidDeviceFunction;
    hipError_t e = slab_prepare(reinterpret_cast<const void *>(k.persistent), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k.persistent, dim3(blocks), dim3(64 * k.waves), lds, stream, tasks, items, n_items, counter,
                       reinterpret_cast<const unsigned char *const *>(jfs), ncps);
    return hipGetLastError();
}

// Synthetic problem for timing runs: J = +-1 by a hash of (p, q) (symmetric,
// zero diagonal), pump 1.2, alpha 1.
__device__ __forceinline__ uint32_t mix32(uint32_t v) {
    v ^= v >> 16;
    v *= 0x7feb352dU;
    v ^= v >> 15;
    v *= 0x846ca68bU;
    v ^= v >> 16;
    return v;
}

__global__ void k_fill_probe(void *j, int j_dtype, int n, float *pump, int r, float *alpha, int na) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nn = (size_t)n * n;
    if (i < nn) {
        const int p = (int)(i / n), q = (int)(i % n);
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        const float v = p == q ? 0.0f : ((mix32((uint32_t)(lo * 65537 + hi)) & 1) ? 1.0f : -1.0f);
        if (j_dtype == CHYM_J_I8) reinterpret_cast<int8_t *>(j)[i] = (int8_t)v;
        else reinterpret_cast<float *>(j)[i] = v;
    }
    if (i < (size_t)r) pump[i] = 1.2f;
    if (i < (size_t)na) alpha[i] = 1.0f;
}

__global__ void k_fill_state(float *x, size_t nx) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += (size_t)gridDim.x * blockDim.x)
        x[i] = ((float)(mix32((uint32_t)i) & 0xffff) - 32768.0f) * 3e-8f;
}

hipError_t launch_fill_probe(void *j, int j_dtype, int n, float *pump, int r, float *alpha, int na,
                             hipStream_t stream) {
    size_t m = (size_t)n * n;
    if ((size_t)r > m) m = r;
    if ((size_t)na > m) m = na;
    hipLaunchKernelGGL(k_fill_probe, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, j, j_dtype, n, pump,
                       r, alpha, na);
    return hipGetLastError();
}

hipError_t launch_fill_state(float *x, size_t nx, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_state, dim3(2048), dim3(256), 0, stream, x, nx);
    return hipGetLastError();
}

// Eight consecutive values per thread through the kernels' own split.
__global__ void k_split3(const float *x, int64_t n8, bf16x8 *hi, bf16x8 *mid, bf16x8 *lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    float v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = x[i * 8 + s];
    XSplit<3> out;
    split8<3>(v, out);
    hi[i] = out.t[0];
    mid[i] = out.t[1];
    lo[i] = out.t[2];
}

hipError_t launch_split3(const float *x, int64_t n, uint16_t *hi, uint16_t *mid, uint16_t *lo, hipStream_t stream) {
    const int64_t n8 = n / 8;
    if (n8 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split3, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, stream, x, n8,
                       reinterpret_cast<bf16x8 *>(hi), reinterpret_cast<bf16x8 *>(mid), reinterpret_cast<bf16x8 *>(lo));
    return hipGetLastError();
}

__global__ void k_zero_counters(int *c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

hipError_t launch_integrate(int tiles, int d, int xs, int js, int waves_per_block, const IntegArgs &a,
                            hipStream_t stream, bool *supported) {
    KernelFn fn = lookup(tiles, d, xs, js);
    *supported = fn.single != nullptr;
    if (!fn.single) return hipSuccess;
    const int reps_per_block = 16 * waves_per_block;
    const int blocks = (a.r + reps_per_block - 1) / reps_per_block;
    hipLaunchKernelGGL(fn.single, dim3(blocks), dim3(64 * waves_per_block), 0, stream, a);
    return hipGetLastError();
}

bool integrate_variant_exists(int tiles, int d, int xs, int js) { return lookup(tiles, d, xs, js).single != nullptr; }

hipError_t launch_integrate_map(int tiles, int d, int xs, int waves_per_block, const IntegArgs &a,
                                hipStream_t stream, bool *supported) {
    KernelFn fn = lookup(tiles, d, xs, 1);
    *supported = fn.single_map != nullptr;
    if (!fn.single_map) return hipSuccess;
    const int reps_per_block = 16 * waves_per_block;
    const int blocks = (a.r + reps_per_block - 1) / reps_per_block;
    hipLaunchKernelGGL(fn.single_map, dim3(blocks), dim3(64 * waves_per_block), 0, stream, a);
    return hipGetLastError();
}

bool map_variant_exists(int tiles, int d, int xs) { return lookup(tiles, d, xs, 1).persistent_map != nullptr; }

hipError_t map_persistent_occupancy(int tiles, int d, int xs, int *blocks_per_cu) {
    KernelFn fn = lookup(tiles, d, xs, 1);
    *blocks_per_cu = 0;
    if (!fn.persistent_map) return hipErrorInvalidDeviceFunction;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn.persistent_map, 256, 0);
}

hipError_t launch_integrate_map_persistent(int tiles, int d, int xs, int blocks, const IntegArgs *tasks,
                                           const int2 *items, int n_items, int *counter, hipStream_t stream) {
    KernelFn fn = lookup(tiles, d, xs, 1);
    if (!fn.persistent_map) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL(fn.persistent_map, dim3(blocks), dim3(256), 0, stream, tasks, items, n_items, counter);
    return hipGetLastError();
}

static void (*lds_kernel(const KernelFn &fn, int kind))(const IntegArgs *, const int2 *, int, int *) {
    switch (kind) {
        case kKernelPipe: return fn.persistent_pipe;
        case kKernelLdsJ1: return fn.persistent_lds1;
        case kKernelLdsJ3: return fn.persistent_lds3;
        default: return fn.persistent_lds;
    }
}

static bool uses_lds(int kind) {
    return kind == kKernelLdsJ || kind == kKernelLdsJ1 || kind == kKernelPipe || kind == kKernelLdsJ3;
}

bool persistent_kind_exists(int tiles, int d, int xs, int js, int kind) {
    KernelFn fn = lookup(tiles, d, xs, js);
    if (!fn.persistent) return false;
    return uses_lds(kind) ? lds_kernel(fn, kind) != nullptr : true;
}

static hipError_t prepare_lds(const KernelFn &fn, int kind) {
    if (fn.lds_bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(lds_kernel(fn, kind)),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fn.lds_bytes);
}

hipError_t persistent_occupancy(int tiles, int d, int xs, int js, int kind, int waves_per_block, int *blocks_per_cu) {
    KernelFn fn = lookup(tiles, d, xs, js);
    *blocks_per_cu = 0;
    if (!fn.persistent) return hipErrorInvalidDeviceFunction;
    if (uses_lds(kind)) {
        if (!lds_kernel(fn, kind)) return hipErrorInvalidDeviceFunction;
        hipError_t e = prepare_lds(fn, kind);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, lds_kernel(fn, kind), 64 * waves_per_block,
                                                            fn.lds_bytes);
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn.persistent, 64 * waves_per_block, 0);
}

hipError_t launch_zero_counters(int *counters, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_counters, dim3((n + 255) / 256), dim3(256), 0, stream, counters, n);
    return hipGetLastError();
}

hipError_t launch_integrate_persistent(int tiles, int d, int xs, int js, int kind, int waves_per_block, int blocks,
                                       const IntegArgs *tasks, const int2 *items, int n_items, int *counter,
                                       hipStream_t stream) {
    KernelFn fn = lookup(tiles, d, xs, js);
    if (!fn.persistent) return hipErrorInvalidDeviceFunction;
    if (uses_lds(kind)) {
        if (!lds_kernel(fn, kind)) return hipErrorInvalidDeviceFunction;
        hipError_t e = prepare_lds(fn, kind);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(lds_kernel(fn, kind), dim3(blocks), dim3(64 * waves_per_block), fn.lds_bytes, stream,
                           tasks, items, n_items, counter);
    } else {
        hipLaunchKernelGGL(fn.persistent, dim3(blocks), dim3(64 * waves_per_block), 0, stream, tasks, items, n_items,
                           counter);
    }
    return hipGetLastError();
}

}  // namespace chym

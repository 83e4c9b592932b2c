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
    return KernelSet{nullptr, nullptr, nullptr, nullptr, 0};
}

int resident_tile_limit(int d, int xs, int js) {
    return (d >= 1 && d <= 4) ? resident_max_tiles(d, xs, js) : 0;
}

// ------------------------------------------------------------ slab kernels
static SlabKernels lookup_slab(int tpw, int d, int xs, int js) {
#define CHYM_PICK(D, XS, JS) \
    if (d == D && xs == XS && js == JS) return lookup_slab_##D##_##XS##_##JS(tpw);
    CHYM_PICK(1, 3, 1) CHYM_PICK(1, 1, 1) CHYM_PICK(1, 3, 3)
    CHYM_PICK(2, 3, 1) CHYM_PICK(2, 1, 1) CHYM_PICK(2, 3, 3)
    CHYM_PICK(3, 3, 1) CHYM_PICK(3, 1, 1) CHYM_PICK(3, 3, 3)
    CHYM_PICK(4, 3, 1) CHYM_PICK(4, 1, 1) CHYM_PICK(4, 3, 3)
#undef CHYM_PICK
    return SlabKernels{nullptr, nullptr};
}

int slab_tpw_for(int tiles) {
    const int per = (tiles + kSlabWaves - 1) / kSlabWaves;
    const int tpw = (per + 3) / 4 * 4;
    return tpw <= 8 ? tpw : 0;
}

size_t slab_lds_bytes(int tiles, int d, int xs) { return (size_t)((tiles + 1) / 2) * d * xs * 64 * sizeof(bf16x8); }

size_t slab_jfrag_bytes(int tiles, int js) {
    return (size_t)tiles * ((tiles + 1) / 2) * js * 64 * sizeof(bf16x8);
}

bool slab_variant_exists(int tiles, int d, int xs, int js) {
    const int tpw = slab_tpw_for(tiles);
    return tpw > 0 && slab_lds_bytes(tiles, d, xs) <= kSlabMaxLds && lookup_slab(tpw, d, xs, js).single != nullptr;
}

hipError_t launch_stage_jfrag(const IntegArgs &a, int js, void *out, hipStream_t stream) {
    const int nt = (a.n + 15) / 16;
    const int ncp = (nt + 1) / 2;
    const int total = nt * ncp * 64;
    const int grid = (total + 255) / 256;
    if (js == 3)
        hipLaunchKernelGGL(k_stage_jfrag<3>, dim3(grid), dim3(256), 0, stream, a, ncp, reinterpret_cast<bf16x8 *>(out));
    else
        hipLaunchKernelGGL(k_stage_jfrag<1>, dim3(grid), dim3(256), 0, stream, a, ncp, reinterpret_cast<bf16x8 *>(out));
    return hipGetLastError();
}

static hipError_t slab_prepare(const void *fn, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_integrate_slab(int tiles, int d, int xs, int js, const IntegArgs &a, const void *jfrag,
                                 hipStream_t stream) {
    const int tpw = slab_tpw_for(tiles);
    SlabKernels k = lookup_slab(tpw, d, xs, js);
    if (!k.single) return hipErrorInvalidDeviceFunction;
    const size_t lds = slab_lds_bytes(tiles, d, xs);
    hipError_t e = slab_prepare(reinterpret_cast<const void *>(k.single), lds);
    if (e != hipSuccess) return e;
    const int blocks = (a.r + 15) / 16;
    hipLaunchKernelGGL(k.single, dim3(blocks), dim3(64 * kSlabWaves), lds, stream, a,
                       reinterpret_cast<const bf16x8 *>(jfrag),
                       (tiles + 1) / 2);
    return hipGetLastError();
}

hipError_t slab_occupancy(int tiles, int d, int xs, int js, size_t lds, int *blocks_per_cu) {
    *blocks_per_cu = 0;
    SlabKernels k = lookup_slab(slab_tpw_for(tiles), d, xs, js);
    if (!k.persistent) return hipErrorInvalidDeviceFunction;
    hipError_t e = slab_prepare(reinterpret_cast<const void *>(k.persistent), lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k.persistent, 64 * kSlabWaves, lds);
}

hipError_t launch_integrate_slab_persistent(int tiles, int d, int xs, int js, size_t lds, int blocks,
                                            const IntegArgs *tasks, const int2 *items, int n_items, int *counter,
                                            const void *const *jfs, const int *ncps, hipStream_t stream) {
    SlabKernels k = lookup_slab(slab_tpw_for(tiles), d, xs, js);
    if (!k.persistent) return hipErrorInvalidDeviceFunction;
    hipError_t e = slab_prepare(reinterpret_cast<const void *>(k.persistent), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k.persistent, dim3(blocks), dim3(64 * kSlabWaves), lds, stream, tasks, items, n_items, counter,
                       reinterpret_cast<const bf16x8 *const *>(jfs), ncps);
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
    split8<3>(v, out, neg_pair());
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

static void (*lds_kernel(const KernelFn &fn, int kind))(const IntegArgs *, const int2 *, int, int *) {
    return kind == kKernelLdsJ1 ? fn.persistent_lds1 : fn.persistent_lds;
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
    if (kind == kKernelLdsJ || kind == kKernelLdsJ1) {
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
    if (kind == kKernelLdsJ || kind == kKernelLdsJ1) {
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

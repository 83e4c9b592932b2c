// Host-side dispatch of the register-resident integrator variants.
#include "integrate_kernel.h"

namespace chym {

typedef KernelPair KernelFn;

static KernelFn lookup(int tiles, int d, int xs, int js) {
#define CHYM_PICK(D, XS, JS) \
    if (d == D && xs == XS && js == JS) return lookup_resident_##D##_##XS##_##JS(tiles);
    CHYM_PICK(1, 3, 1) CHYM_PICK(1, 1, 1) CHYM_PICK(1, 3, 3)
    CHYM_PICK(2, 3, 1) CHYM_PICK(2, 1, 1) CHYM_PICK(2, 3, 3)
    CHYM_PICK(3, 3, 1) CHYM_PICK(3, 1, 1) CHYM_PICK(3, 3, 3)
    CHYM_PICK(4, 3, 1) CHYM_PICK(4, 1, 1) CHYM_PICK(4, 3, 3)
#undef CHYM_PICK
    return KernelPair{nullptr, nullptr};
}

int resident_tile_limit(int d, int xs, int js) {
    return (d >= 1 && d <= 4) ? resident_max_tiles(d, xs, js) : 0;
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

hipError_t persistent_occupancy(int tiles, int d, int xs, int js, int waves_per_block, int *blocks_per_cu) {
    KernelFn fn = lookup(tiles, d, xs, js);
    *blocks_per_cu = 0;
    if (!fn.persistent) return hipErrorInvalidDeviceFunction;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn.persistent, 64 * waves_per_block, 0);
}

hipError_t launch_zero_counters(int *counters, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_counters, dim3((n + 255) / 256), dim3(256), 0, stream, counters, n);
    return hipGetLastError();
}

hipError_t launch_integrate_persistent(int tiles, int d, int xs, int js, int waves_per_block, int blocks,
                                       const IntegArgs *tasks, const int2 *items, int n_items, int *counter,
                                       hipStream_t stream) {
    KernelFn fn = lookup(tiles, d, xs, js);
    if (!fn.persistent) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL(fn.persistent, dim3(blocks), dim3(64 * waves_per_block), 0, stream, tasks, items, n_items,
                       counter);
    return hipGetLastError();
}

}  // namespace chym

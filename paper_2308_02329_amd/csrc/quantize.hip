// FP8 storage of the coupling matrix: OCP E4M3 values with one OCP E8M0
// (power-of-two) exponent per row.  With a power-of-two row scale the
// factoring G_p = 2^e_p sum_q q_pq x_q is exact inside the bf16 matrix-core
// operand, so the integrator needs no extra work per step.
#include "chym_internal.h"

namespace chym {

// One wavefront per row: the row's exponent from its largest magnitude,
// then its codes.
__global__ __launch_bounds__(256) void k_quantize_fp8(int n, const float *__restrict__ j, uint8_t *__restrict__ out) {
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float *src = j + (size_t)row * n;
    float amax = 0.0f;
    bool finite = true;
    for (int q = lane; q < n; q += 64) {
        const float v = src[q];
        finite = finite && __builtin_isfinite(v);
        amax = fmaxf(amax, fabsf(v));
    }
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    finite = __all(finite);
    const int e = e4m3_row_exponent(amax);
    const bool ok = finite && e >= -127 && e <= 127;
    uint8_t *dst = out + (size_t)row * n;
    for (int q = lane; q < n; q += 64) dst[q] = ok ? (uint8_t)e4m3_code(ldexpf(src[q], -e)) : (uint8_t)0x7fu;
    if (lane == 0) out[(size_t)n * n + row] = ok ? (uint8_t)(e + 127) : (uint8_t)0xffu;
}

hipError_t launch_quantize_fp8(int n, const float *j, uint8_t *out, hipStream_t stream) {
    const int grid = (n + 3) / 4;
    hipLaunchKernelGGL(k_quantize_fp8, dim3(grid), dim3(256), 0, stream, n, j, out);
    return hipGetLastError();
}

}  // namespace chym

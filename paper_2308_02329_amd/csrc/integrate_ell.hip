// Sparse-coupling (ELL) CHYM integrator for gfx950.
//
// For graphs with few couplings per row (3-regular: 3; the paper's 20%
// Erdos-Renyi graphs: ~0.2 N) the dense matrix-core contraction does N/w
// times the necessary work.  Here a block owns rb replicas of one problem
// (rb a power of two, as many as let the double-buffered state fit in LDS)
// for the whole run: the state x[p][replica][mu] lives in LDS, each step
// every (row, replica) unit gathers its w couplings (G_mu = sum_k val x_col)
// in float32 from the current buffer and writes the Euler update of Eq. (2)'s
// continuous limit into the other buffer; one block barrier per step.
// Units are ordered row-major with the replica fastest, so the lanes of a
// wavefront read the same coupling row (broadcast) and contiguous state.
// Blocks of 1024 threads (sixteen wavefronts per CU cover the LDS latency);
// the coupling rows and the block's pumps are staged in LDS too when the
// rows fit a fixed budget (read from global memory otherwise).  A persistent
// form takes (task, replica block) items of many problems from a counter.
//
// Short rows (w <= kEllRegW, e.g. 3-regular graphs) with few units per
// thread (<= kEllRegUnits): a thread keeps its units' rows, pumps and own
// state in registers for the whole run, so a step reads from LDS only the
// neighbours' state (w independent loads per component) instead of the row,
// then the neighbours, then its own state; the arithmetic and its order are
// the same, so the results are identical.
#include "chym_internal.h"

namespace chym {

constexpr size_t kEllMaxLds = 159 * 1024;
constexpr size_t kEllRowBudget = 32 * 1024;  // LDS for the coupling rows
constexpr int kEllThreads = 1024;
constexpr int kEllRegW = 3;      // register path: at most this many couplings per row
constexpr int kEllRegUnits = 4;  // and this many (row, replica) units per thread

// Floats per (row, replica) unit in LDS: d, with d = 3 padded to 4, so that
// a unit is one 4-, 8- or 16-byte access and the lanes of a wavefront, which
// read consecutive units of a row, touch consecutive banks.
__host__ __device__ constexpr int ell_unit_floats(int d) { return d == 3 ? 4 : d; }

// Replicas per block: the largest power of two up to 16 whose double-buffered
// state fits LDS and that leaves at most kEllRegUnits units per thread (so
// that short rows take the register path at every size).
__host__ __device__ inline int ell_rb(int n, int d) {
    for (int rb = 16; rb >= 1; rb >>= 1)
        if (2 * (size_t)n * rb * ell_unit_floats(d) * sizeof(float) + kEllRowBudget + 64 <= kEllMaxLds &&
            (rb == 1 || (size_t)n * rb <= (size_t)kEllRegUnits * kEllThreads))
            return rb;
    return 0;
}

int ell_replicas_per_block(int n, int d) { return ell_rb(n, d); }

__host__ __device__ inline int ell_log2(int rb) {
    int l = 0;
    while ((1 << l) < rb) ++l;
    return l;
}

size_t ell_lds_bytes(int n, int d) {
    return 2 * (size_t)n * ell_rb(n, d) * ell_unit_floats(d) * sizeof(float) + 16 * sizeof(float) + kEllRowBudget;
}

// The D values of unit u of an LDS state buffer, as one access.
template <int D>
__device__ __forceinline__ void ell_get(const float *buf, size_t u, float (&v)[D]) {
    if constexpr (D == 1) {
        v[0] = buf[u];
    } else if constexpr (D == 2) {
        const float2 t = reinterpret_cast<const float2 *>(buf)[u];
        v[0] = t.x;
        v[1] = t.y;
    } else {
        const float4 t = reinterpret_cast<const float4 *>(buf)[u];
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        if constexpr (D == 4) v[3] = t.w;
    }
}

template <int D>
__device__ __forceinline__ void ell_put(float *buf, size_t u, const float (&v)[D]) {
    if constexpr (D == 1) {
        buf[u] = v[0];
    } else if constexpr (D == 2) {
        reinterpret_cast<float2 *>(buf)[u] = float2{v[0], v[1]};
    } else {
        reinterpret_cast<float4 *>(buf)[u] = float4{v[0], v[1], v[2], D == 4 ? v[D - 1] : 0.0f};
    }
}

// Integrates replicas rep0 .. rep0 + 2^lrb - 1 of problem a; called by all
// threads of the block (block barriers inside).
template <int D>
__device__ __forceinline__ void ell_block(const IntegArgs &a, int rep0, int lrb, float *sm) {
    const int n = a.n;
    const int r = a.r;
    const int rb = 1 << lrb;
    const int units = n << lrb;
    float *xa = sm;
    constexpr int UF = ell_unit_floats(D);
    float *xb = sm + (size_t)units * UF;
    float *pl = xb + (size_t)units * UF;                 // pumps of the block's replicas [16]
    int *rl = reinterpret_cast<int *>(pl + 16);          // coupling rows [n][2 w], if they fit
    const EllView e = ell_view(a.j, n);
    const bool staged = (size_t)n * 2 * e.w * sizeof(int) <= kEllRowBudget;
    if (staged) {
        const int *src = e.row(0);
        for (int i = threadIdx.x; i < n * 2 * e.w; i += blockDim.x) rl[i] = src[i];
    }
    if (threadIdx.x < rb) pl[threadIdx.x] = rep0 + (int)threadIdx.x < r ? a.pump[rep0 + threadIdx.x] : 1.0f;

    for (int u = threadIdx.x; u < units; u += blockDim.x) {
        const int p = u >> lrb;
        const int rep = rep0 + (u & (rb - 1));
        float v[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) v[mu] = rep < r ? a.x[((size_t)p * r + rep) * D + mu] : 0.0f;
        ell_put<D>(xa, u, v);
    }
    __syncthreads();

    const float nbd = -(a.dt * a.btil);
    const float ned = -(a.dt * a.eta);
    const float dte = a.dt * a.eps;
    const int upt = (units + (int)blockDim.x - 1) / (int)blockDim.x;
    if (e.w <= kEllRegW && upt <= kEllRegUnits) {
        // register path: unit i of this thread is u = threadIdx.x + i blockDim.x
        int nq[kEllRegUnits][kEllRegW];
        float nv[kEllRegUnits][kEllRegW];
        float xv[kEllRegUnits][D];
        float base[kEllRegUnits];
#pragma unroll
        for (int i = 0; i < kEllRegUnits; ++i) {
            const int u = (int)threadIdx.x + i * (int)blockDim.x;
            const bool own = i < upt && u < units;
            const int *row = own ? (staged ? rl + (size_t)(u >> lrb) * 2 * e.w : e.row(u >> lrb)) : nullptr;
#pragma unroll
            for (int kk = 0; kk < kEllRegW; ++kk) {
                nq[i][kk] = (own && kk < e.w) ? row[kk] : -1;
                nv[i][kk] = (own && kk < e.w) ? __int_as_float(row[e.w + kk]) : 0.0f;
            }
            const int jr = u & (rb - 1);
            base[i] = (own && rep0 + jr < r) ? fmaf(a.dt, pl[jr] - 1.0f, 1.0f) : 0.0f;
            if (own) {
                ell_get<D>(xa, u, xv[i]);
            } else {
#pragma unroll
                for (int mu = 0; mu < D; ++mu) xv[i][mu] = 0.0f;
            }
        }
        for (int k = 0; k < a.steps; ++k) {
            const float *al = a.alpha + (size_t)(a.start_step + k) * D;
            float ga[D];
#pragma unroll
            for (int mu = 0; mu < D; ++mu) ga[mu] = dte * al[mu];
#pragma unroll
            for (int i = 0; i < kEllRegUnits; ++i) {
                const int u = (int)threadIdx.x + i * (int)blockDim.x;
                if (i < upt && u < units) {
                    const int jr = u & (rb - 1);
                    float G[D];
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) G[mu] = 0.0f;
#pragma unroll
                    for (int kk = 0; kk < kEllRegW; ++kk) {
                        const int q = nq[i][kk];
                        if ((unsigned)q < (unsigned)n) {
                            float xq[D];
                            ell_get<D>(xa, ((size_t)q << lrb) + jr, xq);
#pragma unroll
                            for (int mu = 0; mu < D; ++mu) G[mu] = fmaf(nv[i][kk], xq[mu], G[mu]);
                        }
                    }
                    float x2[D];
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) x2[mu] = xv[i][mu] * xv[i][mu];
                    float S = x2[0];
#pragma unroll
                    for (int mu = 1; mu < D; ++mu) S = S + x2[mu];
                    const float cc = fmaf(nbd, S, base[i]);
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) {
                        const float y = xv[i][mu] * fmaf(ned, x2[mu], cc);
                        xv[i][mu] = fmaf(ga[mu], G[mu], y);
                    }
                    ell_put<D>(xb, u, xv[i]);
                }
            }
            __syncthreads();
            float *t = xa;
            xa = xb;
            xb = t;
        }
    } else
    for (int k = 0; k < a.steps; ++k) {
        const float *al = a.alpha + (size_t)(a.start_step + k) * D;
        float ga[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) ga[mu] = dte * al[mu];
        // one (row, replica) unit; row = its coupling row (LDS or global)
        auto unit = [&](int u, const int *__restrict__ row) __attribute__((always_inline)) {
            const int jr = u & (rb - 1);
            const int rep = rep0 + jr;
            const float base = rep < r ? fmaf(a.dt, pl[jr] - 1.0f, 1.0f) : 0.0f;  // 1 + dt (r_i - 1)
            float xv[D], G[D];
            ell_get<D>(xa, u, xv);
#pragma unroll
            for (int mu = 0; mu < D; ++mu) G[mu] = 0.0f;
            for (int kk = 0; kk < e.w; ++kk) {
                const int q = row[kk];
                if ((unsigned)q < (unsigned)n) {
                    const float jv = __int_as_float(row[e.w + kk]);
                    float xq[D];
                    ell_get<D>(xa, ((size_t)q << lrb) + jr, xq);
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) G[mu] = fmaf(jv, xq[mu], G[mu]);
                }
            }
            float x2[D];
#pragma unroll
            for (int mu = 0; mu < D; ++mu) x2[mu] = xv[mu] * xv[mu];
            float S = x2[0];
#pragma unroll
            for (int mu = 1; mu < D; ++mu) S = S + x2[mu];
            const float cc = fmaf(nbd, S, base);
            float xn[D];
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                const float y = xv[mu] * fmaf(ned, x2[mu], cc);
                xn[mu] = fmaf(ga[mu], G[mu], y);
            }
            ell_put<D>(xb, u, xn);
        };
        if (staged) {
            for (int u = threadIdx.x; u < units; u += blockDim.x) unit(u, rl + (size_t)(u >> lrb) * 2 * e.w);
        } else {
            for (int u = threadIdx.x; u < units; u += blockDim.x) unit(u, e.row(u >> lrb));
        }
        __syncthreads();
        float *t = xa;
        xa = xb;
        xb = t;
    }

    for (int u = threadIdx.x; u < units; u += blockDim.x) {
        const int p = u >> lrb;
        const int rep = rep0 + (u & (rb - 1));
        if (rep < r) {
            float v[D];
            ell_get<D>(xa, u, v);
#pragma unroll
            for (int mu = 0; mu < D; ++mu) a.x[((size_t)p * r + rep) * D + mu] = v[mu];
        }
    }
}

template <int D>
__global__ __launch_bounds__(kEllThreads) void k_integrate_ell(IntegArgs a, int lrb) {
    extern __shared__ __align__(16) float sm[];
    ell_block<D>(a, blockIdx.x << lrb, lrb, sm);
}

// Many problems of one D: blocks pop (task, replica block) items from the
// counter (zero at launch) until n_items are taken; a task's block size is
// ell_rb(n, D), as for its single launch, so the results are the same.
template <int D>
__global__ __launch_bounds__(kEllThreads) void k_integrate_ell_persistent(const IntegArgs *__restrict__ tasks,
                                                                          const int2 *__restrict__ items,
                                                                          int n_items, int *__restrict__ counter) {
    extern __shared__ __align__(16) float sm[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();  // the previous item's LDS use is over
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        const int2 w = items[it];
        const IntegArgs a = tasks[w.x];
        const int lrb = ell_log2(ell_rb(a.n, D));
        ell_block<D>(a, w.y << lrb, lrb, sm);
    }
}

hipError_t launch_integrate_ell(const IntegArgs &a, hipStream_t stream) {
    const int rb = ell_rb(a.n, a.d);
    if (rb == 0) return hipErrorInvalidValue;
    const int lrb = ell_log2(rb);
    const size_t lds = ell_lds_bytes(a.n, a.d);
    const int blocks = (a.r + rb - 1) / rb;
    void (*fn)(IntegArgs, int) = a.d == 1 ? k_integrate_ell<1>
                                 : a.d == 2 ? k_integrate_ell<2>
                                 : a.d == 3 ? k_integrate_ell<3>
                                            : k_integrate_ell<4>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kEllThreads), lds, stream, a, lrb);
    return hipGetLastError();
}

typedef void (*EllPersistentFn)(const IntegArgs *, const int2 *, int, int *);

static EllPersistentFn ell_persistent_fn(int d) {
    return d == 1 ? k_integrate_ell_persistent<1>
           : d == 2 ? k_integrate_ell_persistent<2>
           : d == 3 ? k_integrate_ell_persistent<3>
                    : k_integrate_ell_persistent<4>;
}

static hipError_t ell_persistent_prepare(EllPersistentFn fn, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

hipError_t ell_persistent_occupancy(int d, size_t lds, int *blocks_per_cu) {
    EllPersistentFn fn = ell_persistent_fn(d);
    *blocks_per_cu = 0;
    hipError_t e = ell_persistent_prepare(fn, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, kEllThreads, lds);
}

hipError_t launch_integrate_ell_persistent(int d, int blocks, size_t lds, const IntegArgs *tasks, const int2 *items,
                                           int n_items, int *counter, hipStream_t stream) {
    EllPersistentFn fn = ell_persistent_fn(d);
    hipError_t e = ell_persistent_prepare(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kEllThreads), lds, stream, tasks, items, n_items, counter);
    return hipGetLastError();
}

}  // namespace chym

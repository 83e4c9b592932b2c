// Readout and scoring kernels: sign readout of the Ising spins, exact Ising
// energy, and the float64 hyperspin energy of Eq. (3).
#include <algorithm>

#include "chym_internal.h"

namespace chym {

// Readout of one replica by one thread.  Walks the rows once: packs the
// spin bits (sigma_p = +1 iff x_{p,1} >= 0), and computes the largest share
// of the extra components and the divergence flag in the same pass.
__device__ void readout_one(int n, int d, int r, int rep, const float *__restrict__ x, uint64_t *__restrict__ spins,
                            double *__restrict__ extra, uint8_t *__restrict__ diverged) {
    const int w = (n + 63) >> 6;
    {
        uint64_t word = 0;
        float m = 0.0f;  // float32: the share needs no more (its reference runs in float64, rtol 1e-6)
        int bad = 0;
        for (int p = 0; p < n; ++p) {
            const float *xp = x + ((size_t)p * r + rep) * d;
            const float v0 = xp[0];
            if (v0 >= 0.0f) word |= 1ull << (p & 63);
            float tot = 0.0f, ext = 0.0f;
            for (int mu = 0; mu < d; ++mu) {
                const float v = xp[mu];
                const float v2 = v * v;
                tot = tot + v2;
                if (mu > 0) ext = ext + v2;
                if (!isfinite(v) || fabsf(v) > 1e3f) bad = 1;
            }
            if (tot > 0.0f && ext / tot > m) m = ext / tot;
            if ((p & 63) == 63 || p == n - 1) {
                if (spins) spins[(size_t)rep * w + (p >> 6)] = word;
                word = 0;
            }
        }
        if (extra) extra[rep] = (double)m;
        if (diverged) diverged[rep] = (uint8_t)bad;
    }
}

__global__ __launch_bounds__(256) void k_readout(int n, int d, int r, const float *__restrict__ x,
                                                 uint64_t *__restrict__ spins, double *__restrict__ extra,
                                                 uint8_t *__restrict__ diverged) {
    for (int rep = blockIdx.x * blockDim.x + threadIdx.x; rep < r; rep += gridDim.x * blockDim.x)
        readout_one(n, d, r, rep, x, spins, extra, diverged);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int spin_of(const uint64_t *s, int p) {
    return ((s[p >> 6] >> (p & 63)) & 1ull) ? 1 : -1;
}

// Ising energy of one replica by one wavefront:
// E = -sum_q sigma_q sum_p J_pq sigma_p.  Lanes own columns q (coalesced
// reads of each row of J); the sigma_p are uniform across the wave.  Integer
// J: exact int32; other J: float64 of the stored values.
__device__ void ising_one(int n, int rep, const void *__restrict__ j, int j_dtype, const uint64_t *__restrict__ spins,
                          int32_t *__restrict__ e_i32, double *__restrict__ e_f64) {
    const int lane = threadIdx.x & 63;
    const int w = (n + 63) >> 6;
    const uint64_t *s = spins + (size_t)rep * w;
    if (j_dtype == CHYM_J_ELL) {
        // lanes own rows p: E = -sum_p sigma_p sum_k val[p][k] sigma_{col[p][k]}
        const EllView e = ell_view(j, n);
        double acc = 0.0;
        for (int p = lane; p < n; p += 64) {
            const int *row = e.row(p);
            double h = 0.0;
            for (int k = 0; k < e.w; ++k) {
                const int q = row[k];
                if ((unsigned)q < (unsigned)n) h += (double)__int_as_float(row[e.w + k]) * (double)spin_of(s, q);
            }
            acc += (double)spin_of(s, p) * h;
        }
        acc = wave_sum(acc);
        if (lane == 0 && e_f64) e_f64[rep] = -acc;
    } else if (j_dtype == CHYM_J_I8) {
        const int8_t *J = reinterpret_cast<const int8_t *>(j);
        int acc = 0;
        for (int q = lane; q < n; q += 64) {
            int h = 0;
            for (int p = 0; p < n; ++p) h += (int)J[(size_t)p * n + q] * spin_of(s, p);
            acc += spin_of(s, q) * h;
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            if (e_i32) e_i32[rep] = -acc;
            if (e_f64) e_f64[rep] = -(double)acc;
        }
    } else {
        double acc = 0.0;
        for (int q = lane; q < n; q += 64) {
            double h = 0.0;
            for (int p = 0; p < n; ++p) h += (double)coupling(j, j_dtype, n, p, q) * (double)spin_of(s, p);
            acc += (double)spin_of(s, q) * h;
        }
        acc = wave_sum(acc);
        if (lane == 0 && e_f64) e_f64[rep] = -acc;
    }
}

// Ising energy of up to 64 replicas of one problem with int8 couplings, one
// replica per lane (lanes with mine = false compute nothing and store
// nothing); W >= ceil(n / 64) spin words per replica, n <= 64 W.  Row p of J
// is read 64 columns at a time, one column per lane, and the ballots of
// J = +1 and J = -1 over the wavefront give the row's masks P and M for those
// columns.  With sigma_q = 2 b_q - 1 (b the spin bit) the +-1 entries add
// 2 popc(b & P) - popc(P) - 2 popc(b & M) + popc(M) to sum_q J_pq sigma_q,
// and the entries of other magnitude (ballot X) are added one by one: the
// result is the exact int32 energy, the same as the row walk of ising_one.
template <int W>
__device__ void ising_lanes(int n, int rep, bool mine, const int8_t *__restrict__ J,
                            const uint64_t *__restrict__ spins, int32_t *__restrict__ e_i32,
                            double *__restrict__ e_f64) {
    const int lane = threadIdx.x & 63;
    const int w = (n + 63) >> 6;
    uint64_t b[W];
#pragma unroll
    for (int k = 0; k < W; ++k) b[k] = (mine && k < w) ? spins[(size_t)rep * w + k] : 0ull;
    int acc = 0;
#pragma unroll
    for (int kp = 0; kp < W; ++kp) {
        const int pend = min(64, n - 64 * kp);
        for (int pp = 0; pp < pend; ++pp) {
            const int8_t *row = J + (size_t)(64 * kp + pp) * n;
            int h = 0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                if (64 * k >= n) break;
                const int q = 64 * k + lane;
                const int v = q < n ? (int)row[q] : 0;
                const uint64_t P = __ballot(v == 1);
                const uint64_t M = __ballot(v == -1);
                uint64_t X = __ballot(v > 1 || v < -1);
                h += 2 * (__popcll(b[k] & P) - __popcll(b[k] & M)) - (__popcll(P) - __popcll(M));
                while (X) {
                    const int t = __ffsll((unsigned long long)X) - 1;
                    X &= X - 1;
                    const int jv = __shfl(v, t, 64);
                    h += ((b[k] >> t) & 1ull) ? jv : -jv;
                }
            }
            acc += ((b[kp] >> pp) & 1ull) ? h : -h;
        }
    }
    if (mine) {
        if (e_i32) e_i32[rep] = -acc;
        if (e_f64) e_f64[rep] = -(double)acc;
    }
}

// Largest n of the lane-per-replica path (16 spin words).
constexpr int kIsingLanesMaxN = 1024;

__device__ __forceinline__ void ising_lanes_any(int n, int rep, bool mine, const int8_t *J, const uint64_t *spins,
                                                int32_t *e_i32, double *e_f64) {
    const int w = (n + 63) >> 6;
    if (w <= 1) ising_lanes<1>(n, rep, mine, J, spins, e_i32, e_f64);
    else if (w <= 2) ising_lanes<2>(n, rep, mine, J, spins, e_i32, e_f64);
    else if (w <= 4) ising_lanes<4>(n, rep, mine, J, spins, e_i32, e_f64);
    else if (w <= 8) ising_lanes<8>(n, rep, mine, J, spins, e_i32, e_f64);
    else ising_lanes<16>(n, rep, mine, J, spins, e_i32, e_f64);
}

__device__ __forceinline__ bool ising_by_lanes(int n, int j_dtype) {
    return j_dtype == CHYM_J_I8 && n <= kIsingLanesMaxN;
}

// One problem, int8 couplings, n <= kIsingLanesMaxN: wavefront w takes
// replicas 64 w .. 64 w + 63.
__global__ __launch_bounds__(256) void k_ising_energy_lanes(int n, int r, const int8_t *__restrict__ J,
                                                            const uint64_t *__restrict__ spins,
                                                            int32_t *__restrict__ e_i32, double *__restrict__ e_f64) {
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave * 64 >= r) return;
    const int rep = wave * 64 + (threadIdx.x & 63);
    ising_lanes_any(n, rep, rep < r, J, spins, e_i32, e_f64);
}

__global__ __launch_bounds__(256) void k_ising_energy(int n, int r, const void *__restrict__ j, int j_dtype,
                                                      const uint64_t *__restrict__ spins,
                                                      int32_t *__restrict__ e_i32, double *__restrict__ e_f64) {
    const int rep = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (rep >= r) return;
    ising_one(n, rep, j, j_dtype, spins, e_i32, e_f64);
}

// Dense part of E_hs for one replica with int8 couplings: sum over the
// lane's columns q of sum_p J_pq (u_p . u_q), u in LDS [n][D].  Four rows at
// a time into four partial sums (independent chains).
template <int D>
__device__ double hs_dense_i8(int n, const int8_t *__restrict__ J, const double *u) {
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
#pragma unroll 1
    for (int q = lane; q < n; q += 64) {
        double uq[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) uq[mu] = u[q * D + mu];
        double h[4] = {0.0, 0.0, 0.0, 0.0};
        int p = 0;
#pragma unroll 1
        for (; p + 4 <= n; p += 4) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double dot = 0.0;
#pragma unroll
                for (int mu = 0; mu < D; ++mu) dot = fma(u[(p + i) * D + mu], uq[mu], dot);
                h[i] = fma((double)J[(size_t)(p + i) * n + q], dot, h[i]);
            }
        }
#pragma unroll 1
        for (; p < n; ++p) {
            double dot = 0.0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) dot = fma(u[p * D + mu], uq[mu], dot);
            h[0] = fma((double)J[(size_t)p * n + q], dot, h[0]);
        }
        acc += (h[0] + h[1]) + (h[2] + h[3]);
    }
    return acc;
}

// Hyperspin energy of one replica by one wavefront, u = its private LDS
// area [n][d].  The unit vectors u_p = x_p / |x_p| (0 for a zero hyperspin)
// are formed in float64, then E_hs = -sum_q sum_p J_pq (u_p . u_q) with
// lanes owning columns q.
__device__ void hs_one(int n, int d, int r, int rep, const void *__restrict__ j, int j_dtype,
                       const float *__restrict__ x, double *__restrict__ e_hs, double *u) {
    const int lane = threadIdx.x & 63;
    for (int q = lane; q < n; q += 64) {
        const float *xq = x + ((size_t)q * r + rep) * d;
        double s = 0.0;
        for (int mu = 0; mu < d; ++mu) {
            const double v = (double)xq[mu];
            s = s + v * v;
        }
        const double nrm = sqrt(s);
        for (int mu = 0; mu < d; ++mu) u[q * d + mu] = nrm > 0.0 ? (double)xq[mu] / nrm : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double acc = 0.0;
    if (j_dtype == CHYM_J_ELL) {
        const EllView e = ell_view(j, n);
        for (int p = lane; p < n; p += 64) {
            const int *row = e.row(p);
            double h = 0.0;
            for (int k = 0; k < e.w; ++k) {
                const int q = row[k];
                if ((unsigned)q >= (unsigned)n) continue;
                double dot = 0.0;
                for (int mu = 0; mu < d; ++mu) dot = dot + u[p * d + mu] * u[q * d + mu];
                h = h + (double)__int_as_float(row[e.w + k]) * dot;
            }
            acc += h;
        }
    } else if (j_dtype == CHYM_J_I8) {
        const int8_t *J8 = reinterpret_cast<const int8_t *>(j);
        switch (d) {
            case 1: acc = hs_dense_i8<1>(n, J8, u); break;
            case 2: acc = hs_dense_i8<2>(n, J8, u); break;
            case 3: acc = hs_dense_i8<3>(n, J8, u); break;
            default: acc = hs_dense_i8<4>(n, J8, u); break;
        }
    } else {
        for (int q = lane; q < n; q += 64) {
            double h = 0.0;
            for (int p = 0; p < n; ++p) {
                double dot = 0.0;
                for (int mu = 0; mu < d; ++mu) dot = dot + u[p * d + mu] * u[q * d + mu];
                const double jv = (double)coupling(j, j_dtype, n, p, q);
                h = h + jv * dot;
            }
            acc += h;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) e_hs[rep] = -acc;
}

__global__ __launch_bounds__(64) void k_hs_energy(int n, int d, int r, const void *__restrict__ j, int j_dtype,
                                                  const float *__restrict__ x, double *__restrict__ e_hs) {
    extern __shared__ double u[];  // [n][d]
    const int rep = blockIdx.x;
    if (rep >= r) return;
    hs_one(n, d, r, rep, j, j_dtype, x, e_hs, u);
}

// ------------------------------------------------------- batched scoring
// Global replica index g of a batch maps to (task, replica) through the
// prefix table first[t] = sum of r over tasks < t (first[n_tasks] = total).
__device__ __forceinline__ int task_of(const int64_t *__restrict__ first, int n_tasks, int64_t g) {
    int lo = 0, hi = n_tasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_readout_batched(const ScoreArgs *__restrict__ t, const int64_t *__restrict__ first,
                                                         int n_tasks) {
    const int64_t total = first[n_tasks];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int k = task_of(first, n_tasks, g);
        const ScoreArgs &a = t[k];
        if (!a.spins && !a.extra && !a.diverged) continue;
        readout_one(a.n, a.d, a.r, (int)(g - first[k]), a.x, a.spins, a.extra, a.diverged);
    }
}

// Each wavefront takes 64 consecutive global replicas at a time and walks the
// tasks they belong to: int8 problems with n <= kIsingLanesMaxN one replica
// per lane, the others one replica per wavefront.
__global__ __launch_bounds__(256) void k_ising_batched(const ScoreArgs *__restrict__ t, const int64_t *__restrict__ first,
                                                       int n_tasks) {
    const int64_t total = first[n_tasks];
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t g0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; g0 < total;
         g0 += waves * 64) {
        const int64_t g1 = min(g0 + 64, total);  // end of this group
        const int k0 = __builtin_amdgcn_readfirstlane(task_of(first, n_tasks, g0));
        const int k1 = __builtin_amdgcn_readfirstlane(task_of(first, n_tasks, g1 - 1));
        for (int k = k0; k <= k1; ++k) {
            const ScoreArgs &a = t[k];
            if (!a.e_i32 && !a.e_f64) continue;
            const int64_t lo = max(first[k], g0), hi = min(first[k + 1], g1);
            if (ising_by_lanes(a.n, a.j_dtype)) {
                const int64_t g = g0 + lane;
                const bool mine = g >= lo && g < hi;
                ising_lanes_any(a.n, mine ? (int)(g - first[k]) : 0, mine, reinterpret_cast<const int8_t *>(a.j),
                                a.spins, a.e_i32, a.e_f64);
            } else {
                for (int64_t g = lo; g < hi; ++g)
                    ising_one(a.n, (int)(g - first[k]), a.j, a.j_dtype, a.spins, a.e_i32, a.e_f64);
            }
        }
    }
}

// Replicas per block pass of k_hs_batched, and the LDS area for one int8
// coupling matrix (n <= 128) staged once per block pass and task.
constexpr int kHsBlockReplicas = 64;
constexpr int kHsJBytes = 128 * 128;

// LDS: one [max n*d] float64 area per wavefront, then (jl_bytes > 0) an int8
// J area of jl_bytes.  Each block takes kHsBlockReplicas consecutive global
// replicas at a time and walks the tasks they span; an int8 task with
// n * n <= jl_bytes is read from the block's LDS copy of J instead of global
// memory.  Block-uniform control flow around the barriers: the pass, the
// task and its LDS decision are the same for every thread of the block.
__global__ __launch_bounds__(256) void k_hs_batched(const ScoreArgs *__restrict__ t, const int64_t *__restrict__ first,
                                                    int n_tasks, int max_nd, int jl_bytes) {
    extern __shared__ double u_all[];
    const int nw = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    double *u = u_all + (size_t)wave * max_nd;
    int8_t *jl = reinterpret_cast<int8_t *>(u_all + (size_t)nw * max_nd);
    const int64_t total = first[n_tasks];
    for (int64_t b0 = (int64_t)blockIdx.x * kHsBlockReplicas; b0 < total;
         b0 += (int64_t)gridDim.x * kHsBlockReplicas) {
        const int64_t b1 = min(b0 + (int64_t)kHsBlockReplicas, total);
        int k = __builtin_amdgcn_readfirstlane(task_of(first, n_tasks, b0));
        for (int64_t s0 = b0; s0 < b1; ++k) {
            const int64_t s1 = min(first[k + 1], b1);
            if (s1 <= s0) continue;  // empty task
            const ScoreArgs &a = t[k];
            if (a.e_hs) {
                const bool staged = a.j_dtype == CHYM_J_I8 && a.n * a.n <= jl_bytes;
                if (staged) {
                    __syncthreads();  // the previous task's readers are done
                    const int8_t *J = reinterpret_cast<const int8_t *>(a.j);
                    for (int i = threadIdx.x; i < a.n * a.n; i += blockDim.x) jl[i] = J[i];
                    __syncthreads();
                }
                for (int64_t g = s0 + wave; g < s1; g += nw) {
                    // two call sites, so that the staged one reads J with LDS instructions
                    if (staged) hs_one(a.n, a.d, a.r, (int)(g - first[k]), jl, a.j_dtype, a.x, a.e_hs, u);
                    else hs_one(a.n, a.d, a.r, (int)(g - first[k]), a.j, a.j_dtype, a.x, a.e_hs, u);
                    __builtin_amdgcn_wave_barrier();  // u is rewritten by the next replica
                }
            }
            s0 = s1;
        }
    }
}

hipError_t launch_readout(int n, int d, int r, const float *x, uint64_t *spins, double *extra, uint8_t *diverged,
                          hipStream_t stream) {
    const int block = 256;
    int grid = (r + block - 1) / block;
    if (grid > 65535) grid = 65535;
    hipLaunchKernelGGL(k_readout, dim3(grid), dim3(block), 0, stream, n, d, r, x, spins, extra, diverged);
    return hipGetLastError();
}

hipError_t launch_ising_energy(int n, int r, const void *j, int j_dtype, const uint64_t *spins, int32_t *e_i32,
                               double *e_f64, hipStream_t stream) {
    const int waves = 4;
    if (j_dtype == CHYM_J_I8 && n <= kIsingLanesMaxN) {
        const int grid = (r + 64 * waves - 1) / (64 * waves);
        if (grid == 0) return hipSuccess;
        hipLaunchKernelGGL(k_ising_energy_lanes, dim3(grid), dim3(64 * waves), 0, stream, n, r,
                           reinterpret_cast<const int8_t *>(j), spins, e_i32, e_f64);
        return hipGetLastError();
    }
    const int grid = (r + waves - 1) / waves;
    hipLaunchKernelGGL(k_ising_energy, dim3(grid), dim3(64 * waves), 0, stream, n, r, j, j_dtype, spins, e_i32,
                       e_f64);
    return hipGetLastError();
}

hipError_t launch_hs_energy(int n, int d, int r, const void *j, int j_dtype, const float *x, double *e_hs,
                            hipStream_t stream) {
    const size_t lds = sizeof(double) * (size_t)n * d;
    hipLaunchKernelGGL(k_hs_energy, dim3(r), dim3(64), lds, stream, n, d, r, j, j_dtype, x, e_hs);
    return hipGetLastError();
}

hipError_t launch_score_batched(const ScoreArgs *tasks, const int64_t *first, int n_tasks, int64_t total_replicas,
                                int max_nd, bool any_readout, bool any_ising, bool any_hs, int cus,
                                hipStream_t stream) {
    if (total_replicas <= 0) return hipSuccess;
    const int grid_cap = 16 * (cus > 0 ? cus : 256);
    if (any_readout) {
        int grid = (int)std::min<int64_t>((total_replicas + 255) / 256, grid_cap);
        hipLaunchKernelGGL(k_readout_batched, dim3(grid), dim3(256), 0, stream, tasks, first, n_tasks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (any_ising) {
        int grid = (int)std::min<int64_t>((total_replicas + 255) / 256, grid_cap);
        hipLaunchKernelGGL(k_ising_batched, dim3(grid), dim3(256), 0, stream, tasks, first, n_tasks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (any_hs) {
        const int waves = max_nd <= 2048 ? 4 : 1;
        const size_t lds_u = sizeof(double) * (size_t)max_nd * waves;
        const int jl_bytes = lds_u + kHsJBytes <= 64 * 1024 ? kHsJBytes : 0;
        const size_t lds = lds_u + (size_t)jl_bytes;
        int grid = (int)std::min<int64_t>((total_replicas + kHsBlockReplicas - 1) / kHsBlockReplicas, grid_cap);
        hipLaunchKernelGGL(k_hs_batched, dim3(grid), dim3(64 * waves), lds, stream, tasks, first, n_tasks, max_nd,
                           jl_bytes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace chym

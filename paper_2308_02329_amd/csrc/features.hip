// Trajectory features for the learned early restart, the per-batch
// standardization, top-k selection and replica gather that the restart loop
// needs, and the small MLP that maps the features to a success logit.
//
// Features (per replica, at one checkpoint), all about the first component,
// the one the anneal keeps and the readout reads: its Rayleigh quotient per
// spin -(x_1^T J x_1) / (n x_1^T x_1), the Ising energy per spin of the
// current sign readout, the first component's share of the squared norm
// sum_p x_{p,1}^2 / sum_{p,mu} x_{p,mu}^2, and the fraction of spins whose
// sign flipped since the previous checkpoint.  Runs of one problem and pump
// reach the same hyperspin configuration up to a rotation, so quantities
// invariant under rotations (the hyperspin energy, the norms) do not tell
// them apart; the first component's orientation does.  One wavefront per
// replica, float32 sums in a fixed order.
//
// MLP: 32 -> 128 -> 128 -> 1, ReLU, sigmoid output, binary cross-entropy.
// Weights are kept as float32 master copies (updated by Adam) and as a bf16
// copy that the forward and backward passes use.  The two hidden layers run
// on the matrix cores in bf16 with float32 accumulation: a layer's input
// (the features, then the first layer's activations) is rounded to bf16
// (nearest even), its bias added in float32; the output layer is a float32
// dot product.  The backward pass differentiates that network (the
// weight gradients use the rounded layer inputs) in float32.
#include <algorithm>

#include "chym_internal.h"

namespace chym {

constexpr int kFeat = CHYM_FEATURES;  // feature columns per replica

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// LDS per wavefront: the first components x_{p,1} [n] and the signs as +-1 [n].
__global__ __launch_bounds__(64) void k_features(int n, int d, int r, const void *__restrict__ j, int j_dtype,
                                                 const float *__restrict__ x, uint64_t *__restrict__ prev,
                                                 float *__restrict__ feat, int feat_stride, int feat_off) {
    extern __shared__ float shf[];
    float *x1 = shf;       // [n]
    float *sg = shf + n;   // [n]
    const int lane = threadIdx.x;
    const int rep = blockIdx.x;
    if (rep >= r) return;
    const int w = (n + 63) >> 6;
    float s1 = 0.0f, sall = 0.0f;
    int flips = 0;
    for (int q = lane; q < n; q += 64) {
        const float *xq = x + ((size_t)q * r + rep) * d;
        float s = 0.0f;
        for (int mu = 0; mu < d; ++mu) s = fmaf(xq[mu], xq[mu], s);
        sall += s;
        s1 = fmaf(xq[0], xq[0], s1);
        x1[q] = xq[0];
        const bool up = xq[0] >= 0.0f;
        sg[q] = up ? 1.0f : -1.0f;
        const bool was = (prev[(size_t)rep * w + (q >> 6)] >> (q & 63)) & 1ull;
        flips += (up != was);
    }
    __syncthreads();
    // column sums: G_q = sum_p J_pq x_{p,1}, h_q = sum_p J_pq sigma_p, so that
    // x_1^T J x_1 = sum_q x_{q,1} G_q and sigma^T J sigma = sum_q sigma_q h_q
    float quad = 0.0f, eis = 0.0f;
    for (int q = lane; q < n; q += 64) {
        float gq = 0.0f, hq = 0.0f;
        for (int p = 0; p < n; ++p) {
            const float jv = coupling(j, j_dtype, n, p, q);
            gq = fmaf(jv, x1[p], gq);
            hq = fmaf(jv, sg[p], hq);
        }
        quad = fmaf(x1[q], gq, quad);
        eis = fmaf(sg[q], hq, eis);
    }
    quad = wsum(quad);
    eis = wsum(eis);
    s1 = wsum(s1);
    sall = wsum(sall);
    flips = wsum(flips);
    // new sign words (one per 64 spins, built by the lanes that own them)
    __syncthreads();
    for (int wd = 0; wd < w; ++wd) {
        const int q = wd * 64 + lane;
        const bool up = q < n && sg[q] > 0.0f;
        const uint64_t bits = __ballot(up);
        if (lane == 0) prev[(size_t)rep * w + wd] = bits;
    }
    if (lane == 0) {
        float *f = feat + (size_t)rep * feat_stride + feat_off;
        f[0] = s1 > 0.0f ? -quad / ((float)n * s1) : 0.0f;
        f[1] = -eis / (float)n;
        f[2] = sall > 0.0f ? s1 / sall : 0.0f;
        f[3] = (float)flips / (float)n;
    }
}

// Standardizes every feature column within each group of `group`
// consecutive replicas (one pump's batch of runs): (f - mean) / sd, with the
// mean and the population standard deviation of the group, 0 where sd = 0.
// One block per group; sums in a fixed order (per-thread strides, then a
// tree), so the result is deterministic.
__global__ __launch_bounds__(256) void k_standardize(int group, const float *__restrict__ in,
                                                     float *__restrict__ out) {
    __shared__ float red[256];
    const size_t base = (size_t)blockIdx.x * group * kFeat;
    for (int c = 0; c < kFeat; ++c) {
        float sum = 0.0f;
        for (int i = threadIdx.x; i < group; i += blockDim.x) sum += in[base + (size_t)i * kFeat + c];
        red[threadIdx.x] = sum;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        const float mean = red[0] / (float)group;
        __syncthreads();
        float ss = 0.0f;
        for (int i = threadIdx.x; i < group; i += blockDim.x) {
            const float v = in[base + (size_t)i * kFeat + c] - mean;
            ss = fmaf(v, v, ss);
        }
        red[threadIdx.x] = ss;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        const float sd = sqrtf(red[0] / (float)group);
        __syncthreads();
        for (int i = threadIdx.x; i < group; i += blockDim.x) {
            const float v = in[base + (size_t)i * kFeat + c];
            out[base + (size_t)i * kFeat + c] = sd > 0.0f ? (v - mean) / sd : 0.0f;
        }
    }
}

// Order-preserving map of a float to an unsigned key (NaN lowest).
__device__ __forceinline__ uint32_t score_key(float v) {
    if (v != v) return 0u;
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

template <int B>
__device__ __forceinline__ int block_count(bool pred, int *red) {
    const uint64_t m = __ballot(pred);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wv] = __popcll(m);
    __syncthreads();
    int tot = 0;
    for (int i = 0; i < B / 64; ++i) tot += red[i];
    __syncthreads();
    return tot;
}

// Exclusive prefix count of pred over the block in thread order, and the total.
template <int B>
__device__ __forceinline__ int block_scan(bool pred, int *red, int *total) {
    const uint64_t m = __ballot(pred);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (ln == 0) red[wv] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
    for (int i = 0; i < B / 64; ++i) {
        if (i < wv) before += red[i];
        tot += red[i];
    }
    __syncthreads();
    *total = tot;
    return before + __popcll(m & ((ln == 0) ? 0ull : (~0ull >> (64 - ln))));
}

// For each group of `group` consecutive scores, the indices of its `keep`
// highest scores (equal scores: the lower index first; NaN lowest), written
// in ascending order to idx[g * keep ...] as global replica indices.  One
// block per group: a bisection over the 32-bit keys finds the keep-th
// largest key, then one ordered pass writes the indices.
__global__ __launch_bounds__(1024) void k_select_top(int group, int keep, const float *__restrict__ score,
                                                     int32_t *__restrict__ idx) {
    __shared__ int red[16];
    const size_t base = (size_t)blockIdx.x * group;
    uint32_t lo = 0u, hi = 0xffffffffu;  // invariant: count(key >= lo) >= keep
    while (lo < hi) {
        const uint32_t mid = lo + (uint32_t)(((uint64_t)hi - lo + 1) >> 1);
        int cnt = 0;
        for (int i0 = 0; i0 < group; i0 += 1024) {
            const int i = i0 + threadIdx.x;
            cnt += block_count<1024>(i < group && score_key(score[base + i]) >= mid, red);
        }
        if (cnt >= keep) lo = mid;
        else hi = mid - 1u;
    }
    const uint32_t t = lo;
    int above = 0;  // keys strictly above t: all kept
    for (int i0 = 0; i0 < group; i0 += 1024) {
        const int i = i0 + threadIdx.x;
        above += block_count<1024>(i < group && score_key(score[base + i]) > t, red);
    }
    int eq_left = keep - above;  // keys equal to t still to keep, lowest index first
    int out = 0;
    for (int i0 = 0; i0 < group; i0 += 1024) {
        const int i = i0 + threadIdx.x;
        const uint32_t k = i < group ? score_key(score[base + i]) : 0u;
        int eq_tot = 0;
        const int eq_before = block_scan<1024>(i < group && k == t, red, &eq_tot);
        const bool take = i < group && (k > t || (k == t && eq_before < eq_left));
        int tot = 0;
        const int pos = block_scan<1024>(take, red, &tot);
        if (take) idx[(size_t)blockIdx.x * keep + out + pos] = (int32_t)(base + i);
        out += tot;
        eq_left -= eq_tot < eq_left ? eq_tot : eq_left;
    }
}

// x_dst[p][j][mu] = x_src[p][idx[j]][mu] and pump_dst[j] = pump_src[idx[j]].
__global__ __launch_bounds__(256) void k_gather_replicas(int n, int d, int r_src, const float *__restrict__ x_src,
                                                         const float *__restrict__ pump_src, int m,
                                                         const int32_t *__restrict__ idx, float *__restrict__ x_dst,
                                                         float *__restrict__ pump_dst) {
    const size_t tot = (size_t)n * m * d;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int mu = (int)(e % d);
        const size_t jq = e / d;
        const int jr = (int)(jq % m);
        const size_t p = jq / m;
        x_dst[e] = x_src[(p * r_src + idx[jr]) * d + mu];
        if (p == 0 && mu == 0 && pump_dst) pump_dst[jr] = pump_src[idx[jr]];
    }
}

// Sign words of the initial state (the reference of the first checkpoint).
__global__ __launch_bounds__(64) void k_sign_words(int n, int d, int r, const float *__restrict__ x,
                                                   uint64_t *__restrict__ words) {
    const int lane = threadIdx.x;
    const int rep = blockIdx.x;
    if (rep >= r) return;
    const int w = (n + 63) >> 6;
    for (int wd = 0; wd < w; ++wd) {
        const int q = wd * 64 + lane;
        const bool up = q < n && x[((size_t)q * r + rep) * d] >= 0.0f;
        const uint64_t bits = __ballot(up);
        if (lane == 0) words[(size_t)rep * w + wd] = bits;
    }
}

hipError_t launch_features(int n, int d, int r, const void *j, int j_dtype, const float *x, uint64_t *prev,
                           float *feat, int feat_stride, int feat_off, hipStream_t stream) {
    const size_t lds = sizeof(float) * 2 * (size_t)n;
    hipLaunchKernelGGL(k_features, dim3(r), dim3(64), lds, stream, n, d, r, j, j_dtype, x, prev, feat, feat_stride,
                       feat_off);
    return hipGetLastError();
}

hipError_t launch_sign_words(int n, int d, int r, const float *x, uint64_t *words, hipStream_t stream) {
    hipLaunchKernelGGL(k_sign_words, dim3(r), dim3(64), 0, stream, n, d, r, x, words);
    return hipGetLastError();
}

hipError_t launch_standardize(int groups, int group, const float *in, float *out, hipStream_t stream) {
    if (groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_standardize, dim3(groups), dim3(256), 0, stream, group, in, out);
    return hipGetLastError();
}

hipError_t launch_select_top(int groups, int group, int keep, const float *score, int32_t *idx, hipStream_t stream) {
    if (groups <= 0 || keep <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_top, dim3(groups), dim3(1024), 0, stream, group, keep, score, idx);
    return hipGetLastError();
}

hipError_t launch_gather_replicas(int n, int d, int r_src, const float *x_src, const float *pump_src, int m,
                                  const int32_t *idx, float *x_dst, float *pump_dst, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    const size_t tot = (size_t)n * m * d;
    const unsigned blocks = (unsigned)std::min<size_t>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(k_gather_replicas, dim3(blocks), dim3(256), 0, stream, n, d, r_src, x_src, pump_src, m, idx,
                       x_dst, pump_dst);
    return hipGetLastError();
}

// ------------------------------------------------------------------ MLP
// Parameter block layout (float32 master and bf16 copy use the same order):
//   W1 [H1][F], b1 [H1], W2 [H2][H1], b2 [H2], w3 [H2], b3 [1]
constexpr int kF = 32, kH1 = 128, kH2 = 128;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH1 * kF;
constexpr int kOffW2 = kOffB1 + kH1;
constexpr int kOffB2 = kOffW2 + kH2 * kH1;
constexpr int kOffW3 = kOffB2 + kH2;
constexpr int kOffB3 = kOffW3 + kH2;
constexpr int kParams = kOffB3 + 1;
static_assert(kParams == CHYM_MLP_PARAMS && kF == CHYM_FEATURES, "parameter block must match chym.h");

__device__ __forceinline__ float bf(const __bf16 *w, int i) { return (float)w[i]; }

typedef __attribute__((ext_vector_type(2))) float mlp_f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 mlp_bf16x2;
typedef __attribute__((ext_vector_type(4))) __bf16 mlp_bf16x4;

__device__ __forceinline__ mlp_bf16x2 mlp_pack(float a, float b) {
    return __builtin_convertvector((mlp_f32x2){a, b}, mlp_bf16x2);
}

__device__ __forceinline__ bf16x8 mlp_join(mlp_bf16x2 a, mlp_bf16x2 b, mlp_bf16x2 c, mlp_bf16x2 d) {
    const mlp_bf16x4 lo = __builtin_shufflevector(a, b, 0, 1, 2, 3);
    const mlp_bf16x4 hi = __builtin_shufflevector(c, d, 0, 1, 2, 3);
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ mlp_bf16x4 mlp_load4(const __bf16 *p) { return *reinterpret_cast<const mlp_bf16x4 *>(p); }

// Forward pass on the matrix cores, one wavefront per 16 samples (the batch
// tail padded with zero features, its outputs not written).  Both hidden
// layers are computed transposed, H^T = W X^T, with v_mfma_f32_16x16x32_bf16:
// the weights are the A operand (16 units x 32 inputs per fragment), the
// layer input the B operand (32 inputs x 16 samples), and lane (j, g) of a
// 16 x 16 result holds units 4 g + v of sample j.  The second layer's K
// chunk c is the rows lane (j, g) already holds in result tiles 2c and 2c+1
// (slot s: unit 32 c + 16 (s >> 2) + 4 g + (s & 3)), with W2's columns read in
// that order, so its B operand comes from the lane's own registers.  Writes
// the logit, and h1 (the rounded first-layer activations, the second layer's
// input) and h2 when given, [batch][128] each.
__global__ __launch_bounds__(256) void k_mlp_forward(int batch, const float *__restrict__ feat,
                                                     const __bf16 *__restrict__ wb, float *__restrict__ logit,
                                                     float *__restrict__ h1, float *__restrict__ h2) {
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    const int s0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16;
    if (s0 >= batch) return;  // wave-uniform
    const int smp = s0 + j;
    const bool ok = smp < batch;
    // layer 1: B operand = features 8 g .. 8 g + 7 of sample j, rounded to bf16
    bf16x8 bx;
    {
        float v[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = ok ? feat[(size_t)smp * kF + 8 * g + s] : 0.0f;
        bx = mlp_join(mlp_pack(v[0], v[1]), mlp_pack(v[2], v[3]), mlp_pack(v[4], v[5]), mlp_pack(v[6], v[7]));
    }
    f32x4 a1[8];
#pragma unroll
    for (int I = 0; I < 8; ++I) {
        const mlp_bf16x4 b = mlp_load4(wb + kOffB1 + 16 * I + 4 * g);
        a1[I] = f32x4{(float)b[0], (float)b[1], (float)b[2], (float)b[3]};
        // A fragment: W1 row 16 I + j, inputs 8 g .. 8 g + 7
        const bf16x8 aw = *reinterpret_cast<const bf16x8 *>(wb + kOffW1 + (16 * I + j) * kF + 8 * g);
        a1[I] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx, a1[I], 0, 0, 0);
    }
    // ReLU, then the rounded activations (the second layer's input)
    mlp_bf16x2 hp[8][2];
#pragma unroll
    for (int I = 0; I < 8; ++I) {
        float r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = a1[I][v] > 0.0f ? a1[I][v] : 0.0f;
        hp[I][0] = mlp_pack(r[0], r[1]);
        hp[I][1] = mlp_pack(r[2], r[3]);
        if (h1 && ok) {
            float4 o;
            o.x = (float)hp[I][0][0];
            o.y = (float)hp[I][0][1];
            o.z = (float)hp[I][1][0];
            o.w = (float)hp[I][1][1];
            *reinterpret_cast<float4 *>(h1 + (size_t)smp * kH1 + 16 * I + 4 * g) = o;
        }
    }
    // layer 2
    f32x4 a2[8];
#pragma unroll
    for (int I = 0; I < 8; ++I) {
        const mlp_bf16x4 b = mlp_load4(wb + kOffB2 + 16 * I + 4 * g);
        a2[I] = f32x4{(float)b[0], (float)b[1], (float)b[2], (float)b[3]};
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bf16x8 bh = mlp_join(hp[2 * c][0], hp[2 * c][1], hp[2 * c + 1][0], hp[2 * c + 1][1]);
#pragma unroll
        for (int I = 0; I < 8; ++I) {
            const __bf16 *row = wb + kOffW2 + (16 * I + j) * kH1 + 32 * c + 4 * g;
            const mlp_bf16x4 lo = mlp_load4(row), hi = mlp_load4(row + 16);
            const bf16x8 aw = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
            a2[I] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bh, a2[I], 0, 0, 0);
        }
    }
    // ReLU and the output layer: float32 dot with w3 over the lane's units,
    // then over the four lanes of the sample
    float part = 0.0f;
#pragma unroll
    for (int I = 0; I < 8; ++I) {
        const mlp_bf16x4 w3 = mlp_load4(wb + kOffW3 + 16 * I + 4 * g);
        float r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            r[v] = a2[I][v] > 0.0f ? a2[I][v] : 0.0f;
            part = fmaf((float)w3[v], r[v], part);
        }
        if (h2 && ok) *reinterpret_cast<float4 *>(h2 + (size_t)smp * kH2 + 16 * I + 4 * g) = float4{r[0], r[1], r[2], r[3]};
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g == 0 && ok) logit[smp] = (float)wb[kOffB3] + part;
}

// Backward pass of the mean binary cross-entropy over the batch, in three
// deterministic stages:
//  1. k_mlp_backward_act, one sample per thread: dz = (sigmoid(z) - y) / B,
//     d2 = dz w3 * [h2 > 0], d1 = (W2^T d2) * [h1 > 0], and the loss term;
//  2. k_mlp_wgrad, NS samples per block: the block's partial weight
//     gradients (sums over its samples of outer products), one parameter
//     per thread at a time, operands staged in LDS;
//  3. k_mlp_reduce: the partials summed over blocks in block order.
__global__ __launch_bounds__(128) void k_mlp_backward_act(int batch, const float *__restrict__ label,
                                                          const __bf16 *__restrict__ wb,
                                                          const float *__restrict__ logit,
                                                          const float *__restrict__ h1, const float *__restrict__ h2,
                                                          float *__restrict__ dzs, float *__restrict__ d1s,
                                                          float *__restrict__ d2s, float *__restrict__ loss) {
    extern __shared__ float w[];  // W2 [kH2][kH1], then w3 [kH2]
    for (int i = threadIdx.x; i < kH2 * kH1; i += blockDim.x) w[i] = bf(wb, kOffW2 + i);
    for (int i = threadIdx.x; i < kH2; i += blockDim.x) w[kH2 * kH1 + i] = bf(wb, kOffW3 + i);
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    const float z = logit[s];
    const float y = label[s];
    const float p = 1.0f / (1.0f + expf(-z));
    const float dz = (p - y) / (float)batch;
    dzs[s] = dz;
    loss[s] = (z > 0.0f ? z + log1pf(expf(-z)) : log1pf(expf(z))) - y * z;
    float d1[kH1];
#pragma unroll
    for (int i = 0; i < kH1; ++i) d1[i] = 0.0f;
    for (int o = 0; o < kH2; ++o) {
        const float d2 = h2[(size_t)s * kH2 + o] > 0.0f ? dz * w[kH2 * kH1 + o] : 0.0f;
        d2s[(size_t)s * kH2 + o] = d2;
#pragma unroll
        for (int i = 0; i < kH1; ++i) d1[i] = fmaf(d2, w[o * kH1 + i], d1[i]);
    }
#pragma unroll
    for (int i = 0; i < kH1; ++i) d1s[(size_t)s * kH1 + i] = h1[(size_t)s * kH1 + i] > 0.0f ? d1[i] : 0.0f;
}

constexpr int kNS = 16;  // samples per block of the weight-gradient stage

__global__ __launch_bounds__(256) void k_mlp_wgrad(int batch, const float *__restrict__ feat,
                                                   const float *__restrict__ h1, const float *__restrict__ h2,
                                                   const float *__restrict__ dzs, const float *__restrict__ d1s,
                                                   const float *__restrict__ d2s, float *__restrict__ partial) {
    __shared__ float sx[kNS][kF], sh1[kNS][kH1], sh2[kNS][kH2], sd1[kNS][kH1], sd2[kNS][kH2], sdz[kNS];
    const int s0 = blockIdx.x * kNS;
    const int ns = batch - s0 < kNS ? batch - s0 : kNS;
    for (int i = threadIdx.x; i < kNS * kH1; i += blockDim.x) {
        const int a = i / kH1, b = i % kH1;
        const bool ok = a < ns;
        sh1[a][b] = ok ? h1[(size_t)(s0 + a) * kH1 + b] : 0.0f;
        sh2[a][b] = ok ? h2[(size_t)(s0 + a) * kH2 + b] : 0.0f;
        sd1[a][b] = ok ? d1s[(size_t)(s0 + a) * kH1 + b] : 0.0f;
        sd2[a][b] = ok ? d2s[(size_t)(s0 + a) * kH2 + b] : 0.0f;
    }
    for (int i = threadIdx.x; i < kNS * kF; i += blockDim.x) {
        const int a = i / kF, b = i % kF;
        // the first layer's input as the forward pass rounds it
        sx[a][b] = a < ns ? (float)(__bf16)feat[(size_t)(s0 + a) * kF + b] : 0.0f;
    }
    for (int i = threadIdx.x; i < kNS; i += blockDim.x) sdz[i] = i < ns ? dzs[s0 + i] : 0.0f;
    __syncthreads();
    float *out = partial + (size_t)blockIdx.x * kParams;
    for (int pi = threadIdx.x; pi < kParams; pi += blockDim.x) {
        float acc = 0.0f;
        if (pi < kOffB1) {  // W1[o][k] = sum d1[o] x[k]
            const int o = pi / kF, k = pi % kF;
            for (int a = 0; a < kNS; ++a) acc = fmaf(sd1[a][o], sx[a][k], acc);
        } else if (pi < kOffW2) {
            const int o = pi - kOffB1;
            for (int a = 0; a < kNS; ++a) acc += sd1[a][o];
        } else if (pi < kOffB2) {  // W2[o][i] = sum d2[o] h1[i]
            const int o = (pi - kOffW2) / kH1, i = (pi - kOffW2) % kH1;
            for (int a = 0; a < kNS; ++a) acc = fmaf(sd2[a][o], sh1[a][i], acc);
        } else if (pi < kOffW3) {
            const int o = pi - kOffB2;
            for (int a = 0; a < kNS; ++a) acc += sd2[a][o];
        } else if (pi < kOffB3) {  // w3[o] = sum dz h2[o]
            const int o = pi - kOffW3;
            for (int a = 0; a < kNS; ++a) acc = fmaf(sdz[a], sh2[a][o], acc);
        } else {
            for (int a = 0; a < kNS; ++a) acc += sdz[a];
        }
        out[pi] = acc;
    }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(int blocks, const float *__restrict__ partial,
                                                    float *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    float acc = 0.0f;
    for (int b = 0; b < blocks; ++b) acc += partial[(size_t)b * kParams + i];
    grad[i] = acc;
}

// Adam (Kingma & Ba) on the float32 master weights; refreshes the bf16 copy.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ wm, __bf16 *__restrict__ wb,
                                                  float *__restrict__ m, float *__restrict__ v,
                                                  const float *__restrict__ grad, float lr, float b1, float b2,
                                                  float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float wi = wm[i] - lr * mh / (sqrtf(vh) + eps);
    wm[i] = wi;
    wb[i] = (__bf16)wi;
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *__restrict__ src, __bf16 *__restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (__bf16)src[i];
}

int mlp_param_count() { return kParams; }

hipError_t launch_mlp_forward(int batch, const float *feat, const void *wb, float *logit, float *h1, float *h2,
                              hipStream_t stream) {
    if (batch <= 0) return hipSuccess;
    const int waves = (batch + 15) / 16;  // 16 samples per wavefront, 4 wavefronts per block
    hipLaunchKernelGGL(k_mlp_forward, dim3((waves + 3) / 4), dim3(256), 0, stream, batch, feat,
                       reinterpret_cast<const __bf16 *>(wb), logit, h1, h2);
    return hipGetLastError();
}

// Backward scratch: dz [B], d1 [B][H1], d2 [B][H2], per-block partial
// gradients [ceil(B / kNS)][kParams].
size_t mlp_backward_scratch_floats(int batch) {
    return (size_t)batch * (1 + kH1 + kH2) + (size_t)((batch + kNS - 1) / kNS) * kParams;
}

hipError_t launch_mlp_backward(int batch, const float *feat, const float *label, const void *wb, const float *logit,
                               const float *h1, const float *h2, float *scratch, float *grad, float *loss,
                               hipStream_t stream) {
    if (batch <= 0) return hipSuccess;
    float *dzs = scratch;
    float *d1s = dzs + batch;
    float *d2s = d1s + (size_t)batch * kH1;
    float *partial = d2s + (size_t)batch * kH2;
    const int block = 128;
    const size_t lds = sizeof(float) * (kH2 * kH1 + kH2);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp_backward_act),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_backward_act, dim3((batch + block - 1) / block), dim3(block), lds, stream, batch, label,
                       reinterpret_cast<const __bf16 *>(wb), logit, h1, h2, dzs, d1s, d2s, loss);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int wblocks = (batch + kNS - 1) / kNS;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(wblocks), dim3(256), 0, stream, batch, feat, h1, h2, dzs, d1s, d2s, partial);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, stream, wblocks, partial, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *wm, void *wb, float *m, float *v, const float *grad, float lr, float b1, float b2,
                           float eps, int t, hipStream_t stream) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, stream, wm,
                       reinterpret_cast<__bf16 *>(wb), m, v, grad, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, void *dst, int n, hipStream_t stream) {
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, stream, src, reinterpret_cast<__bf16 *>(dst),
                       n);
    return hipGetLastError();
}

}  // namespace chym

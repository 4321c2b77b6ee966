// Learned weight proposer (form F3): front-gap features, a small MLP
// (D -> 128 -> 128 -> 1, exact-erf GELU, bf16 weights, fp32 activations and
// accumulation), its mean binary cross-entropy gradient, Adam, top-k
// selection and the labels "this weight vector produced a new non-dominated
// point".  The paper has no learned component; the proposer chooses which
// scalarisation weight vectors (Eq. 7) the sampler runs next.
//
// Parameter layout (flat): W1 [H][D], b1 [H], W2 [H][H], b2 [H], w3 [H], b3.

#include <cmath>

#include "radix.hpp"

namespace qaia {
namespace {

constexpr int kH = 128;
constexpr int kB = 256;
constexpr int kMaxD = 16;

struct ParamOffsets {
    int64_t W1, b1, W2, b2, w3, b3, total;
};
__host__ __device__ inline ParamOffsets offsets(int D) {
    ParamOffsets o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)kH * D;
    o.W2 = o.b1 + kH;
    o.b2 = o.W2 + (int64_t)kH * kH;
    o.w3 = o.b2 + kH;
    o.b3 = o.w3 + kH;
    o.total = o.b3 + 1;
    return o;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round half to even (finite values)
    return (uint16_t)(u >> 16);
}
// 1 + erf(z / sqrt 2) is evaluated as erfc(-z / sqrt 2): for negative z the
// sum would cancel (at z = -5 it is 1.5e-6, below the float32 spacing of the
// erf value near -1), the complementary function keeps full relative accuracy.
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * erfcf(-z * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * erfcf(-z * 0.70710678118654752f) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------- MLP passes
//
// One block of 256 threads (four waves) handles 32 samples.  Layer 1
// (D -> 128, tiny) runs on the vector units; the 128 x 128 contractions run
// on the matrix cores as fp32 32x32x2 MFMAs (the bf16 weights widen exactly to
// fp32, so activations and accumulation stay fp32):
//   forward : Z2 = A1 W2^T, wave w takes the 32 units 32w .. 32w+31;
//   backward: dZ1 = dZ2 W2 (wave w: hidden units 32w ..), and
//             dW2 = dZ2^T A1 (wave w: rows u = 32w .., all 128 columns).
// For every MFMA the A and B fragments of a lane come from the same k
// position (k = 2t + lane / 32), which pairs them for any internal k order.
// Accumulator slot i of lane l holds row (i/4)*8 + (l/32)*4 + i%4, column l%32.
// Training writes the block's gradient contribution (every parameter) to
// partial[block]; a second kernel sums the blocks in a fixed order.
constexpr int kS = 32;          // samples per block
constexpr int kP = kH + 2;      // LDS pitch (floats) of the 128-wide tiles: a 32-lane strided read and its
                                // neighbour column fall on disjoint banks

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int acc_row(int half, int i) { return (i >> 2) * 8 + half * 4 + (i & 3); }

template <bool TRAIN>
__global__ __launch_bounds__(kB) void mlp_fused_kernel(const uint16_t *__restrict__ P, int D,
                                                       const float *__restrict__ X, int64_t N,
                                                       const float *__restrict__ y, float *__restrict__ logits,
                                                       float *__restrict__ partial) {
    __shared__ float w2[kH * kP];          // W2[u][h] at u * kP + h
    __shared__ float w1[kH][kMaxD + 1];
    __shared__ float xs[kS][kMaxD + 1];
    __shared__ float a1[kS * kP];          // A1[s][h]
    __shared__ float g1[TRAIN ? kS * kP : 1];   // gelu'(z1)[s][h]
    __shared__ float dz2[TRAIN ? kS * kP : 1];  // dZ2[s][u]
    __shared__ float dz1[TRAIN ? kS * kP : 1];  // dZ1[s][h]
    __shared__ float lpart[4][kS];
    __shared__ float dz3[kS];
    const ParamOffsets o = offsets(D);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5, lr = lane & 31;
    const int64_t s0 = (int64_t)blockIdx.x * kS;
    const int ns = (int)(N - s0 < kS ? N - s0 : kS);
    if ((((uintptr_t)(P + o.W2)) & 15) == 0) {
        // eight bf16 weights per 16-byte load (W2 starts at 128 (D + 1) elements)
        const uint4 *src = (const uint4 *)(P + o.W2);
        for (int i = tid; i < kH * kH / 8; i += kB) {
            const uint4 w = src[i];
            float *dst = w2 + ((i * 8) >> 7) * kP + ((i * 8) & (kH - 1));
            const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                dst[2 * e] = __uint_as_float(u[e] << 16);
                dst[2 * e + 1] = __uint_as_float(u[e] & 0xFFFF0000u);
            }
        }
    } else {
        for (int i = tid; i < kH * kH; i += kB) w2[(i >> 7) * kP + (i & (kH - 1))] = bf16_to_f32(P[o.W2 + i]);
    }
    for (int i = tid; i < kH * kMaxD; i += kB) {
        const int h = i / kMaxD, d = i % kMaxD;
        w1[h][d] = d < D ? bf16_to_f32(P[o.W1 + (int64_t)h * D + d]) : 0.0f;
    }
    for (int i = tid; i < kS * kMaxD; i += kB) {
        const int s = i / kMaxD, d = i % kMaxD;
        xs[s][d] = (s < ns && d < D) ? X[(s0 + s) * D + d] : 0.0f;
    }
    __syncthreads();
    // layer 1: thread t takes sample t % 32 and hidden units 16 (t / 32) ..
    {
        const int s = tid & (kS - 1), hg = tid >> 5;
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
            const int h = hg * 16 + j;
            float z = bf16_to_f32(P[o.b1 + h]);
            for (int d = 0; d < D; ++d) z = fmaf(w1[h][d], xs[s][d], z);
            a1[s * kP + h] = gelu(z);
            if constexpr (TRAIN) g1[s * kP + h] = gelu_grad(z);
        }
    }
    __syncthreads();
    // layer 2 on the matrix cores: this wave's 32 units
    const int u = wave * 32 + lr;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll 8
    for (int t = 0; t < kH / 2; ++t) {
        const int k = 2 * t + half;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[lr * kP + k], w2[u * kP + k], acc, 0, 0, 0);
    }
    const float b2u = bf16_to_f32(P[o.b2 + u]), w3u = bf16_to_f32(P[o.w3 + u]);
    float z2[16], part[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        z2[i] = acc[i] + b2u;
        part[i] = w3u * gelu(z2[i]);
    }
    // head: sum over this wave's units (the 32 lanes of each half), per row
#pragma unroll
    for (int i = 0; i < 16; ++i)
        for (int off = 16; off > 0; off >>= 1) part[i] += __shfl_xor(part[i], off, 64);
    if (lr == 0)
#pragma unroll
        for (int i = 0; i < 16; ++i) lpart[wave][acc_row(half, i)] = part[i];
    __syncthreads();
    if (tid < kS) {
        // the four waves' unit ranges in a fixed order
        const float z = bf16_to_f32(P[o.b3]) + ((lpart[0][tid] + lpart[1][tid]) + (lpart[2][tid] + lpart[3][tid]));
        if (tid < ns && logits) logits[s0 + tid] = z;
        if constexpr (TRAIN) dz3[tid] = tid < ns ? (1.0f / (1.0f + expf(-z)) - y[s0 + tid]) / (float)N : 0.0f;
    }
    if constexpr (!TRAIN) return;
    __syncthreads();
    float *pg = partial + (int64_t)blockIdx.x * o.total;
    // dZ2 = dz3 w3 gelu'(z2); gb2[u] = sum_s dZ2, gw3[u] = sum_s dz3 a2
    {
        float gb2 = 0.0f, gw3 = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int s = acc_row(half, i);
            const float d3 = dz3[s];
            const float d2 = d3 * w3u * gelu_grad(z2[i]);
            dz2[s * kP + u] = d2;
            gb2 += d2;
            gw3 = fmaf(d3, gelu(z2[i]), gw3);
        }
        gb2 += __shfl_xor(gb2, 32, 64);
        gw3 += __shfl_xor(gw3, 32, 64);
        if (half == 0) {
            pg[o.b2 + u] = gb2;
            pg[o.w3 + u] = gw3;
        }
        if (tid == 0) {
            float g3 = 0.0f;
            for (int s = 0; s < kS; ++s) g3 += dz3[s];
            pg[o.b3] = g3;
        }
    }
    __syncthreads();
    // dZ1 = (dZ2 W2) * gelu'(z1): this wave's hidden units h = 32w + lr
    {
        const int h = wave * 32 + lr;
        f32x16 d;
#pragma unroll
        for (int i = 0; i < 16; ++i) d[i] = 0.0f;
#pragma unroll 8
        for (int t = 0; t < kH / 2; ++t) {
            const int k = 2 * t + half;  // the unit index u
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(dz2[lr * kP + k], w2[k * kP + h], d, 0, 0, 0);
        }
        float gb1 = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int s = acc_row(half, i);
            const float v = d[i] * g1[s * kP + h];
            dz1[s * kP + h] = v;
            gb1 += v;
        }
        gb1 += __shfl_xor(gb1, 32, 64);
        if (half == 0) pg[o.b1 + h] = gb1;
    }
    // dW2 = dZ2^T A1: rows u = 32w + .., columns h in four 32-wide tiles, k = sample
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        f32x16 g;
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = 0.0f;
#pragma unroll
        for (int t = 0; t < kS / 2; ++t) {
            const int s = 2 * t + half;
            g = __builtin_amdgcn_mfma_f32_32x32x2f32(dz2[s * kP + wave * 32 + lr], a1[s * kP + c * 32 + lr], g, 0, 0,
                                                     0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) pg[o.W2 + (int64_t)(wave * 32 + acc_row(half, i)) * kH + c * 32 + lr] = g[i];
    }
    __syncthreads();
    // dW1[h][d] = sum_s dZ1[s][h] x[s][d]: thread t takes hidden unit t / 2 and eight inputs
    {
        const int h = tid >> 1, d0 = (tid & 1) * 8;
        float g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int s = 0; s < kS; ++s) {
            const float v = dz1[s * kP + h];
#pragma unroll
            for (int j = 0; j < 8; ++j) g[j] = fmaf(v, xs[s][d0 + j], g[j]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (d0 + j < D) pg[o.W1 + (int64_t)h * D + d0 + j] = g[j];
    }
}

// the gradient is the sum of the blocks' contributions, in block order (deterministic)
__global__ void grads_reduce_kernel(const float *__restrict__ partial, int slices, int64_t total,
                                    float *__restrict__ grad) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= total) return;
    float g = 0.0f;
    for (int j = 0; j < slices; ++j) g += partial[(int64_t)j * total + p];
    grad[p] = g;
}

// Adam (Kingma and Ba, 2015) on fp32 master weights; refreshes the bf16 copy
__global__ void adam_kernel(float *__restrict__ master, uint16_t *__restrict__ P,
                            float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float w = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    master[i] = w;
    P[i] = f32_to_bf16(w);
}

// ---------------------------------------------------------------- features

// per objective nadir (min) and ideal (max) of the front; one block
__global__ void front_range_kernel(const int64_t *__restrict__ front, int64_t Pn, int m,
                                   int64_t *__restrict__ lohi) {
    __shared__ int64_t lo_sh[8][kB / 64], hi_sh[8][kB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < m; ++k) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int64_t j = threadIdx.x; j < Pn; j += kB) {
            const int64_t v = front[j * m + k];
            lo = v < lo ? v : lo;
            hi = v > hi ? v : hi;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const int64_t ol = __shfl_xor(lo, off), oh = __shfl_xor(hi, off);
            lo = ol < lo ? ol : lo;
            hi = oh > hi ? oh : hi;
        }
        if (lane == 0) {
            lo_sh[k][wave] = lo;
            hi_sh[k][wave] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x < m) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int w = 0; w < kB / 64; ++w) {
            lo = lo_sh[threadIdx.x][w] < lo ? lo_sh[threadIdx.x][w] : lo;
            hi = hi_sh[threadIdx.x][w] > hi ? hi_sh[threadIdx.x][w] : hi;
        }
        lohi[threadIdx.x] = lo;
        lohi[8 + threadIdx.x] = hi;
    }
}

// normalised front y^ (range 0 maps to 1)
__global__ void front_norm_kernel(const int64_t *__restrict__ front, int64_t Pn, int m,
                                  const int64_t *__restrict__ lohi, float *__restrict__ yh) {
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= Pn * m) return;
    const int k = (int)(idx % m);
    const int64_t lo = lohi[k], hi = lohi[8 + k];
    const double r = (double)hi - (double)lo;
    yh[idx] = r > 0.0 ? (float)(((double)front[idx] - (double)lo) / r) : 1.0f;
}

// per front point: distance to the nearest other point and the fraction of
// points within 0.05 (itself included); the front passes through LDS in
// chunks shared by the block
constexpr int kLChunk = 2048;

__global__ __launch_bounds__(kB) void front_local_kernel(const float *__restrict__ yh, int64_t Pn, int m,
                                                         float *__restrict__ nn, float *__restrict__ frac) {
    __shared__ float stage[kLChunk * 8];
    const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    const bool active = j < Pn;
    float me[8];
    for (int k = 0; k < m; ++k) me[k] = active ? yh[j * m + k] : 0.0f;
    float best = INFINITY;
    int64_t close = 0;
    for (int64_t base = 0; base < Pn; base += kLChunk) {
        const int cnt = (int)(Pn - base < kLChunk ? Pn - base : kLChunk);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * m; i += kB) stage[i] = yh[base * m + i];
        __syncthreads();
        if (active)
            for (int i = 0; i < cnt; ++i) {
                float d2 = 0.0f;
                for (int k = 0; k < m; ++k) {
                    const float d = stage[i * m + k] - me[k];
                    d2 = fmaf(d, d, d2);
                }
                const float d = sqrtf(d2);
                if (base + i != j && d < best) best = d;
                if (d <= 0.05f) ++close;
            }
    }
    if (!active) return;
    nn[j] = Pn > 1 ? best : 0.0f;
    frac[j] = (float)close / (float)Pn;
}

template <int M>
__device__ float angle(const float (&a)[M], const float *b) {
    // 2 atan2(|a^ - b^|, |a^ + b^|): accurate for nearly parallel vectors
    float na = 0.0f, nb = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        na = fmaf(a[k], a[k], na);
        nb = fmaf(b[k], b[k], nb);
    }
    na = sqrtf(na);
    nb = sqrtf(nb);
    float dm = 0.0f, dp = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const float u = a[k] / na, v = b[k] / nb;
        dm = fmaf(u - v, u - v, dm);
        dp = fmaf(u + v, u + v, dp);
    }
    return 2.0f * atan2f(sqrtf(dm), sqrtf(dp));
}

// one thread per candidate weight vector; the front and the last round's hit
// and miss vectors are staged through LDS in chunks shared by the block.  The
// smallest angle to a set is taken at the set member with the largest cosine
// (the angle decreases with the cosine) and then evaluated accurately once.
constexpr int kFChunk = 1024;

template <int M>
__device__ __forceinline__ void best_cosine(const float (&u)[M], const float *__restrict__ vecs, int64_t count,
                                            float *stage, bool active, int64_t &best) {
    float bc = -INFINITY;
    best = -1;
    for (int64_t base = 0; base < count; base += kFChunk) {
        const int cnt = (int)(count - base < kFChunk ? count - base : kFChunk);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += kB) {
            float nb = 0.0f;
#pragma unroll
            for (int k = 0; k < M; ++k) nb = fmaf(vecs[(base + i) * M + k], vecs[(base + i) * M + k], nb);
            const float inv = nb > 0.0f ? 1.0f / sqrtf(nb) : 0.0f;
#pragma unroll
            for (int k = 0; k < M; ++k) stage[i * M + k] = vecs[(base + i) * M + k] * inv;
        }
        __syncthreads();
        if (active)
            for (int i = 0; i < cnt; ++i) {
                float d = 0.0f;
#pragma unroll
                for (int k = 0; k < M; ++k) d = fmaf(u[k], stage[i * M + k], d);
                if (d > bc) {
                    bc = d;
                    best = base + i;
                }
            }
    }
}

template <int M>
__global__ __launch_bounds__(kB) void features_kernel(const float *__restrict__ yh, int64_t Pn,
                                                      const float *__restrict__ nn, const float *__restrict__ frac,
                                                      const float *__restrict__ cands, int64_t N,
                                                      const float *__restrict__ hits, int64_t Hn,
                                                      const float *__restrict__ misses, int64_t Mn,
                                                      float *__restrict__ feat) {
    __shared__ float stage[kFChunk * M];
    const int64_t c = (int64_t)blockIdx.x * kB + threadIdx.x;
    const bool active = c < N;
    float w[M], u[M];
    float nw = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        w[k] = active ? cands[c * M + k] : 0.0f;
        nw = fmaf(w[k], w[k], nw);
    }
    const float inv = nw > 0.0f ? 1.0f / sqrtf(nw) : 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) u[k] = w[k] * inv;
    float f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // max, second and eighth largest of v_j = c . yh_j over the front, and the maximiser
    float top[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) top[i] = -INFINITY;
    int64_t jstar = 0;
    for (int64_t base = 0; base < Pn; base += kFChunk) {
        const int cnt = (int)(Pn - base < kFChunk ? Pn - base : kFChunk);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * M; i += kB) stage[i] = yh[base * M + i];
        __syncthreads();
        if (active)
            for (int jj = 0; jj < cnt; ++jj) {
                float v = 0.0f;
#pragma unroll
                for (int k = 0; k < M; ++k) v = fmaf(w[k], stage[jj * M + k], v);
                if (v > top[0]) jstar = base + jj;  // first index on ties
                if (v > top[7]) {
                    int i = 7;
                    while (i > 0 && top[i - 1] < v) {
                        top[i] = top[i - 1];
                        --i;
                    }
                    top[i] = v;
                }
            }
    }
    if (Pn > 0) {
        f[0] = top[0];
        f[1] = Pn > 1 ? top[0] - top[1] : 0.0f;
        f[2] = top[0] - top[Pn < 8 ? Pn - 1 : 7];
        f[3] = nn[jstar];
        f[4] = frac[jstar];
    }
    int64_t bh, bm;
    best_cosine<M>(u, hits, Hn, stage, active, bh);
    best_cosine<M>(u, misses, Mn, stage, active, bm);
    if (!active) return;
    f[5] = bh >= 0 ? angle<M>(w, hits + bh * M) : 1.57079632679489662f;
    f[6] = bm >= 0 ? angle<M>(w, misses + bm * M) : 1.57079632679489662f;
    float dev = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) dev = fmaxf(dev, fabsf(w[k] - 1.0f / (float)M));
    f[7] = dev;
    // one MLP input row: the candidate followed by its eight features
    float *row = feat + c * (M + 8);
#pragma unroll
    for (int k = 0; k < M; ++k) row[k] = w[k];
#pragma unroll
    for (int i = 0; i < 8; ++i) row[M + i] = f[i];
}

// ---------------------------------------------------------------- selection and labels

// Gumbel-perturbed keys: the top k of score / tau + G (G standard Gumbel from
// the counter stream) is a sample of k items without replacement with
// probabilities proportional to exp(score / tau).
__global__ void gumbel_keys_kernel(const float *__restrict__ scores, int64_t N, float inv_tau, uint64_t seed,
                                   float *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= N) return;
    uint64_t z = seed + ((uint64_t)i + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    const float u = ((float)(uint32_t)(z >> 40) + 0.5f) * 0x1p-24f;  // (0, 1)
    keys[i] = scores[i] * inv_tau - logf(-logf(u));
}

// Sort keys of the top-k selection: descending score order as an ascending
// unsigned key (the IEEE bit pattern made monotone, then complemented; -0 is
// taken as +0), value = item index.  Block 0 also stores the item and digit
// pass counts the sort reads from device memory.
__global__ void topk_key_kernel(const float *__restrict__ s, int64_t N, uint64_t *__restrict__ key,
                                int32_t *__restrict__ val, int64_t *__restrict__ d_n, int32_t *__restrict__ d_passes) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i == 0) {
        *d_n = N;
        *d_passes = 4;
    }
    if (i >= N) return;
    const float f = s[i];
    uint32_t b = f == 0.0f ? 0u : __float_as_uint(f);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    key[i] = (uint64_t)(~b);
    val[i] = (int32_t)i;
}

__global__ void topk_out_kernel(const int32_t *__restrict__ val, int64_t k, int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < k) out[i] = val[i];
}

__global__ void labels_kernel(const int64_t *__restrict__ keep, const int64_t *__restrict__ num_keep,
                              int64_t archive, int R, int64_t W, float *__restrict__ labels) {
    const int64_t K = *num_keep;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < K; t += (int64_t)gridDim.x * kB) {
        const int64_t s = keep[t];
        if (s >= archive) {
            const int64_t w = (s - archive) / R;
            if (w < W) labels[w] = 1.0f;
        }
    }
}

__global__ void zero_f32_kernel(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void gather_rows_kernel(const uint32_t *__restrict__ src, int width,
                                   const int64_t *__restrict__ idx, const int64_t *__restrict__ count,
                                   int64_t cap, uint32_t *__restrict__ dst) {
    const int64_t K = *count < cap ? *count : cap;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < K * width; t += (int64_t)gridDim.x * kB) {
        const int64_t r = t / width, c = t % width;
        dst[t] = src[idx[r] * width + c];
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kB - 1) / kB); }

}  // namespace

int64_t mlp_param_count(int D) { return offsets(D).total; }

static int64_t grad_blocks(int64_t B) { return (B + kS - 1) / kS; }

size_t mlp_backward_ws_bytes(int D, int64_t B) {
    return align256(sizeof(float) * (size_t)std::max<int64_t>(grad_blocks(B), 1) *
                    (size_t)offsets(std::max(D, 1)).total);
}

size_t mlp_forward_ws_bytes(int64_t N) {
    (void)N;
    return 256;  // the fused forward keeps everything on chip
}

void launch_mlp_forward(const uint16_t *P, int D, const float *X, int64_t N, float *logits, void *ws,
                        hipStream_t st) {
    (void)ws;
    QAIA_CHECK(D >= 1 && D <= kMaxD, QAIA_INVALID_ARGUMENT, "input width must be in [1, 16]");
    if (N == 0) return;
    const int64_t blocks = grad_blocks(N);
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many samples");
    hipLaunchKernelGGL(mlp_fused_kernel<false>, dim3((unsigned)blocks), dim3(kB), 0, st, P, D, X, N,
                       (const float *)nullptr, logits, (float *)nullptr);
    QAIA_HIP(hipGetLastError());
}

void launch_mlp_backward(const uint16_t *P, int D, const float *X, const float *y, int64_t B,
                         float *grad, float *loss_logits, void *ws, hipStream_t st) {
    QAIA_CHECK(D >= 1 && D <= kMaxD, QAIA_INVALID_ARGUMENT, "input width must be in [1, 16]");
    QAIA_CHECK(B >= 1, QAIA_INVALID_ARGUMENT, "batch must be >= 1");
    const int64_t total = offsets(D).total, blocks = grad_blocks(B);
    QAIA_CHECK(blocks <= 65535, QAIA_INVALID_ARGUMENT, "batch too large");
    float *partial = (float *)ws;
    hipLaunchKernelGGL(mlp_fused_kernel<true>, dim3((unsigned)blocks), dim3(kB), 0, st, P, D, X, B, y, loss_logits,
                       partial);
    hipLaunchKernelGGL(grads_reduce_kernel, dim3(blocks_for(total)), dim3(kB), 0, st, partial, (int)blocks, total,
                       grad);
    QAIA_HIP(hipGetLastError());
}

void launch_adam(float *master, uint16_t *P, float *m, float *v, const float *g, int64_t n, int step,
                 float lr, float b1, float b2, float eps, hipStream_t st) {
    QAIA_CHECK(step >= 1, QAIA_INVALID_ARGUMENT, "Adam step counts from 1");
    const float c1 = (float)(1.0 - std::pow((double)b1, step));
    const float c2 = (float)(1.0 - std::pow((double)b2, step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(kB), 0, st, master, P, m, v, g, n, lr, b1,
                       b2, eps, c1, c2);
    QAIA_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- training loop

namespace {
__global__ void train_count_kernel(int64_t *c, int64_t n) {
    if (threadIdx.x == 0) *c = n;
}
}  // namespace

struct TrainLayout {
    size_t zeros, perm, xp, yp, grad, count, bw, tk, total;
};

static TrainLayout train_layout(int D, int64_t n, int64_t B) {
    TrainLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t nz = (size_t)std::max<int64_t>(n, 1);
    L.zeros = take(sizeof(float) * nz);
    L.perm = take(sizeof(int64_t) * nz);
    L.xp = take(sizeof(float) * nz * (size_t)D);
    L.yp = take(sizeof(float) * nz);
    L.grad = take(sizeof(float) * (size_t)offsets(D).total);
    L.count = take(sizeof(int64_t));
    L.bw = take(mlp_backward_ws_bytes(D, B));
    L.tk = take(topk_ws_bytes(n));
    L.total = off;
    return L;
}

size_t mlp_train_ws_bytes(int D, int64_t n, int64_t batch) {
    return train_layout(std::max(D, 1), std::max<int64_t>(n, 1), std::min(std::max<int64_t>(batch, 1), std::max<int64_t>(n, 1))).total;
}

// `steps` Adam steps on minibatches of min(batch, n) rows: minibatch t is
// window t mod (n / B) of a random permutation of the rows, drawn afresh at
// the start of every pass as the Gumbel top-k of n equal scores with seed
// `seed + 104729 * (first_step + t)`; the Adam step counter runs from
// first_step.
void launch_mlp_train(float *master, uint16_t *P, float *m1, float *m2, int D, const float *X, const float *y,
                      int64_t n, int64_t batch, int steps, int first_step, float lr, uint64_t seed, void *ws,
                      size_t ws_bytes, hipStream_t st) {
    QAIA_CHECK(D >= 1 && D <= kMaxD, QAIA_INVALID_ARGUMENT, "input width must be in [1, 16]");
    QAIA_CHECK(n >= 1 && batch >= 1 && steps >= 0 && first_step >= 1, QAIA_INVALID_ARGUMENT,
               "need n >= 1, batch >= 1, steps >= 0, first_step >= 1");
    const int64_t B = std::min(batch, n), per_pass = n / B;
    const TrainLayout L = train_layout(D, n, B);
    QAIA_CHECK(ws_bytes >= L.total, QAIA_WORKSPACE_TOO_SMALL, "training workspace too small");
    char *b = (char *)ws;
    float *zeros = (float *)(b + L.zeros), *xp = (float *)(b + L.xp), *yp = (float *)(b + L.yp);
    float *grad = (float *)(b + L.grad);
    int64_t *perm = (int64_t *)(b + L.perm), *cnt = (int64_t *)(b + L.count);
    const int64_t total = offsets(D).total;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks_for(n)), dim3(kB), 0, st, zeros, n);
    hipLaunchKernelGGL(train_count_kernel, dim3(1), dim3(64), 0, st, cnt, n);
    QAIA_HIP(hipGetLastError());
    for (int t = 0; t < steps; ++t) {
        const int64_t win = t % per_pass;
        if (win == 0) {
            launch_topk(zeros, n, n, 1.0f, seed + 104729ull * (uint64_t)(first_step + t), perm, b + L.tk,
                        topk_ws_bytes(n), st);
            launch_gather_rows((const uint32_t *)X, D, perm, cnt, n, (uint32_t *)xp, st);
            launch_gather_rows((const uint32_t *)y, 1, perm, cnt, n, (uint32_t *)yp, st);
        }
        launch_mlp_backward(P, D, xp + win * B * D, yp + win * B, B, grad, nullptr, b + L.bw, st);
        launch_adam(master, P, m1, m2, grad, total, first_step + t, lr, 0.9f, 0.999f, 1e-8f, st);
    }
}

size_t features_ws_bytes(int64_t Pn, int m) {
    return align256(16 * sizeof(int64_t)) + align256(sizeof(float) * (size_t)std::max<int64_t>(Pn, 1) * m) +
           2 * align256(sizeof(float) * (size_t)std::max<int64_t>(Pn, 1));
}

void launch_features(const int64_t *front, int64_t Pn, int m, const float *cands, int64_t N,
                     const float *hits, int64_t Hn, const float *misses, int64_t Mn, float *feat,
                     void *ws, size_t ws_bytes, hipStream_t st) {
    QAIA_CHECK(m >= 1 && m <= 8, QAIA_INVALID_ARGUMENT, "m must be in [1, 8]");
    QAIA_CHECK(ws_bytes >= features_ws_bytes(Pn, m), QAIA_WORKSPACE_TOO_SMALL, "feature workspace too small");
    if (N == 0) return;
    char *b = (char *)ws;
    int64_t *lohi = (int64_t *)b;
    size_t off = align256(16 * sizeof(int64_t));
    float *yh = (float *)(b + off);
    off += align256(sizeof(float) * (size_t)std::max<int64_t>(Pn, 1) * m);
    float *nn = (float *)(b + off);
    off += align256(sizeof(float) * (size_t)std::max<int64_t>(Pn, 1));
    float *frac = (float *)(b + off);
    if (Pn > 0) {
        hipLaunchKernelGGL(front_range_kernel, dim3(1), dim3(kB), 0, st, front, Pn, m, lohi);
        hipLaunchKernelGGL(front_norm_kernel, dim3(blocks_for(Pn * m)), dim3(kB), 0, st, front, Pn, m, lohi, yh);
        hipLaunchKernelGGL(front_local_kernel, dim3(blocks_for(Pn)), dim3(kB), 0, st, yh, Pn, m, nn, frac);
    }
#define QAIA_FEATURES(MM)                                                                                     \
    case MM:                                                                                                  \
        hipLaunchKernelGGL(features_kernel<MM>, dim3(blocks_for(N)), dim3(kB), 0, st, yh, Pn, nn, frac, cands, N, \
                           hits, Hn, misses, Mn, feat);                                                       \
        break;
    switch (m) {
        QAIA_FEATURES(1)
        QAIA_FEATURES(2)
        QAIA_FEATURES(3)
        QAIA_FEATURES(4)
        QAIA_FEATURES(5)
        QAIA_FEATURES(6)
        QAIA_FEATURES(7)
        QAIA_FEATURES(8)
        default: throw Error{QAIA_UNSUPPORTED, "features support 1..8 objectives"};
    }
#undef QAIA_FEATURES
    QAIA_HIP(hipGetLastError());
}

size_t topk_ws_bytes(int64_t N) {
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    return align256(sizeof(float) * n) + 2 * align256(sizeof(uint64_t) * n) + 2 * align256(sizeof(int32_t) * n) +
           align256(4 * radix_hist_words(N)) + align256(4 * 256) + align256(64);
}

void launch_topk(const float *scores, int64_t N, int64_t k, float temperature, uint64_t seed, int64_t *idx_out,
                 void *ws, size_t ws_bytes, hipStream_t st) {
    QAIA_CHECK(N >= 1 && N < (int64_t(1) << 31), QAIA_INVALID_ARGUMENT, "N must be in [1, 2^31)");
    QAIA_CHECK(k >= 0 && k <= N, QAIA_INVALID_ARGUMENT, "k must be in [0, N]");
    QAIA_CHECK(ws_bytes >= topk_ws_bytes(N), QAIA_WORKSPACE_TOO_SMALL, "top-k workspace too small");
    QAIA_CHECK(temperature >= 0.0f && std::isfinite(temperature), QAIA_INVALID_ARGUMENT,
               "temperature must be finite and >= 0");
    char *b = (char *)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = b + off;
        off += align256(bytes);
        return p;
    };
    float *pert = (float *)take(sizeof(float) * (size_t)N);
    uint64_t *keyA = (uint64_t *)take(sizeof(uint64_t) * (size_t)N), *keyB = (uint64_t *)take(sizeof(uint64_t) * (size_t)N);
    int32_t *valA = (int32_t *)take(sizeof(int32_t) * (size_t)N), *valB = (int32_t *)take(sizeof(int32_t) * (size_t)N);
    uint32_t *hist = (uint32_t *)take(4 * radix_hist_words(N)), *total = (uint32_t *)take(4 * 256);
    char *small = take(64);
    int64_t *d_n = (int64_t *)small;
    int32_t *d_passes = (int32_t *)(small + 8);
    const float *src = scores;
    if (temperature > 0.0f) {
        hipLaunchKernelGGL(gumbel_keys_kernel, dim3(blocks_for(N)), dim3(kB), 0, st, scores, N, 1.0f / temperature,
                           seed, pert);
        src = pert;
    }
    // stable: equal scores keep increasing index order; four passes leave the result in A
    hipLaunchKernelGGL(topk_key_kernel, dim3(blocks_for(N)), dim3(kB), 0, st, src, N, keyA, valA, d_n, d_passes);
    QAIA_HIP(hipGetLastError());
    for (int pass = 0; pass < 4; ++pass) {
        const bool even = (pass & 1) == 0;
        radix_pass(even ? keyA : keyB, even ? valA : valB, even ? keyB : keyA, even ? valB : valA, N, d_n, d_passes,
                   pass, hist, total, st);
    }
    if (k > 0) {
        hipLaunchKernelGGL(topk_out_kernel, dim3(blocks_for(k)), dim3(kB), 0, st, valA, k, idx_out);
        QAIA_HIP(hipGetLastError());
    }
}

void launch_labels(const int64_t *keep, const int64_t *num_keep, int64_t archive, int R, int64_t W,
                   float *labels, hipStream_t st) {
    QAIA_CHECK(R >= 1 && W >= 0 && archive >= 0, QAIA_INVALID_ARGUMENT, "bad label arguments");
    if (W == 0) return;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks_for(W)), dim3(kB), 0, st, labels, W);
    hipLaunchKernelGGL(labels_kernel, dim3(1024), dim3(kB), 0, st, keep, num_keep, archive, R, W, labels);
    QAIA_HIP(hipGetLastError());
}

void launch_gather_rows(const uint32_t *src, int width, const int64_t *idx, const int64_t *count,
                        int64_t cap, uint32_t *dst, hipStream_t st) {
    QAIA_CHECK(width >= 1 && cap >= 0, QAIA_INVALID_ARGUMENT, "bad gather arguments");
    hipLaunchKernelGGL(gather_rows_kernel, dim3(1024), dim3(kB), 0, st, src, width, idx, count, cap, dst);
    QAIA_HIP(hipGetLastError());
}

}  // namespace qaia

// Learned weight proposer (form F3): front-gap features, a small MLP
// (D -> 128 -> 128 -> 1, exact-erf GELU, bf16 weights, fp32 activations and
// accumulation), its mean binary cross-entropy gradient, Adam, top-k
// selection and the labels "this weight vector produced a new non-dominated
// point".  The paper has no learned component; the proposer chooses which
// scalarisation weight vectors (Eq. 7) the sampler runs next.
//
// Parameter layout (flat): W1 [H][D], b1 [H], W2 [H][H], b2 [H], w3 [H], b3.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "internal.hpp"

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
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------- MLP passes

// a1 = gelu(W1 x + b1), g1 = gelu'(.) (optional); one thread per (sample, unit)
__global__ void layer1_kernel(const uint16_t *__restrict__ P, int D, const float *__restrict__ X,
                              int64_t N, float *__restrict__ a1, float *__restrict__ g1) {
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= N * kH) return;
    const int64_t s = idx / kH;
    const int h = (int)(idx % kH);
    const ParamOffsets o = offsets(D);
    float z = bf16_to_f32(P[o.b1 + h]);
    for (int d = 0; d < D; ++d) z = fmaf(bf16_to_f32(P[o.W1 + (int64_t)h * D + d]), X[s * D + d], z);
    a1[idx] = gelu(z);
    if (g1) g1[idx] = gelu_grad(z);
}

// a2 = gelu(W2 a1 + b2), g2 = gelu'(.) (optional); one thread per (sample, unit)
__global__ void layer2_kernel(const uint16_t *__restrict__ P, int D, const float *__restrict__ a1,
                              int64_t N, float *__restrict__ a2, float *__restrict__ g2) {
    // transposed copy: lanes (consecutive units u) read consecutive words
    __shared__ float w2t[kH][kH];
    const ParamOffsets o = offsets(D);
    for (int i = threadIdx.x; i < kH * kH; i += kB) w2t[i % kH][i / kH] = bf16_to_f32(P[o.W2 + i]);
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= N * kH) return;
    const int64_t s = idx / kH;
    const int u = (int)(idx % kH);
    const float *a = a1 + s * kH;
    float z = bf16_to_f32(P[o.b2 + u]);
#pragma unroll 8
    for (int h = 0; h < kH; ++h) z = fmaf(w2t[h][u], a[h], z);
    a2[idx] = gelu(z);
    if (g2) g2[idx] = gelu_grad(z);
}

// logit = w3 . a2 + b3; with labels: dz3 = (sigmoid(logit) - y) / B and
// dz2 = dz3 w3 gelu'(z2); one thread per sample
__global__ void head_kernel(const uint16_t *__restrict__ P, int D, const float *__restrict__ a2,
                            const float *__restrict__ g2, int64_t N, const float *__restrict__ y,
                            float *__restrict__ logits, float *__restrict__ dz3,
                            float *__restrict__ dz2) {
    const int64_t s = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (s >= N) return;
    const ParamOffsets o = offsets(D);
    float z = bf16_to_f32(P[o.b3]);
    for (int u = 0; u < kH; ++u) z = fmaf(bf16_to_f32(P[o.w3 + u]), a2[s * kH + u], z);
    if (logits) logits[s] = z;
    if (y) {
        const float d = (1.0f / (1.0f + expf(-z)) - y[s]) / (float)N;
        dz3[s] = d;
        for (int u = 0; u < kH; ++u) dz2[s * kH + u] = d * bf16_to_f32(P[o.w3 + u]) * g2[s * kH + u];
    }
}

// dz1 = (W2^T dz2) * gelu'(z1); one thread per (sample, unit)
__global__ void back1_kernel(const uint16_t *__restrict__ P, int D, const float *__restrict__ dz2,
                             const float *__restrict__ g1, int64_t N, float *__restrict__ dz1) {
    __shared__ float w2[kH][kH];  // natural layout: lanes (consecutive h) read consecutive words
    const ParamOffsets o = offsets(D);
    for (int i = threadIdx.x; i < kH * kH; i += kB) w2[i / kH][i % kH] = bf16_to_f32(P[o.W2 + i]);
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= N * kH) return;
    const int64_t s = idx / kH;
    const int h = (int)(idx % kH);
    float a = 0.0f;
#pragma unroll 8
    for (int u = 0; u < kH; ++u) a = fmaf(w2[u][h], dz2[s * kH + u], a);
    dz1[idx] = a * g1[idx];
}

// parameter gradients in two passes: pass 1 gives each (parameter, slice of
// kSlice samples) one thread, pass 2 sums the slices in order (deterministic)
constexpr int kSlice = 64;

__global__ void grads_partial_kernel(int D, const float *__restrict__ X, const float *__restrict__ a1,
                                     const float *__restrict__ a2, const float *__restrict__ dz1,
                                     const float *__restrict__ dz2, const float *__restrict__ dz3, int64_t N,
                                     float *__restrict__ partial) {
    const ParamOffsets o = offsets(D);
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= o.total) return;
    const int64_t s0 = (int64_t)blockIdx.y * kSlice;
    const int64_t s1 = s0 + kSlice < N ? s0 + kSlice : N;
    float g = 0.0f;
    if (p < o.b1) {
        const int h = (int)(p / D), d = (int)(p % D);
        for (int64_t s = s0; s < s1; ++s) g = fmaf(dz1[s * kH + h], X[s * D + d], g);
    } else if (p < o.W2) {
        const int h = (int)(p - o.b1);
        for (int64_t s = s0; s < s1; ++s) g += dz1[s * kH + h];
    } else if (p < o.b2) {
        const int u = (int)((p - o.W2) / kH), h = (int)((p - o.W2) % kH);
        for (int64_t s = s0; s < s1; ++s) g = fmaf(dz2[s * kH + u], a1[s * kH + h], g);
    } else if (p < o.w3) {
        const int u = (int)(p - o.b2);
        for (int64_t s = s0; s < s1; ++s) g += dz2[s * kH + u];
    } else if (p < o.b3) {
        const int u = (int)(p - o.w3);
        for (int64_t s = s0; s < s1; ++s) g = fmaf(dz3[s], a2[s * kH + u], g);
    } else {
        for (int64_t s = s0; s < s1; ++s) g += dz3[s];
    }
    partial[(int64_t)blockIdx.y * o.total + p] = g;
}

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
// points within 0.05 (itself included)
__global__ void front_local_kernel(const float *__restrict__ yh, int64_t Pn, int m,
                                   float *__restrict__ nn, float *__restrict__ frac) {
    const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (j >= Pn) return;
    float best = INFINITY;
    int64_t close = 0;
    for (int64_t i = 0; i < Pn; ++i) {
        float d2 = 0.0f;
        for (int k = 0; k < m; ++k) {
            const float d = yh[i * m + k] - yh[j * m + k];
            d2 = fmaf(d, d, d2);
        }
        const float d = sqrtf(d2);
        if (i != j && d < best) best = d;
        if (d <= 0.05f) ++close;
    }
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

__global__ void iota64_kernel(int64_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = i;
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

size_t topk_temp(int64_t N) {
    size_t b = 0;
    hipcub::DeviceRadixSort::SortPairsDescending(nullptr, b, (const float *)nullptr, (float *)nullptr,
                                                 (const int64_t *)nullptr, (int64_t *)nullptr,
                                                 (int)std::max<int64_t>(N, 1), 0, 32, (hipStream_t)0);
    return b;
}

}  // namespace

int64_t mlp_param_count(int D) { return offsets(D).total; }

static int64_t grad_slices(int64_t B) { return (B + kSlice - 1) / kSlice; }

size_t mlp_backward_ws_bytes(int D, int64_t B) {
    // a1, g1, a2, g2, dz1, dz2 [B][H], dz3 [B], per-slice partial gradients [slices][params]
    return align256(sizeof(float) * (size_t)B * kH) * 6 + align256(sizeof(float) * (size_t)B) +
           align256(sizeof(float) * (size_t)grad_slices(B) * (size_t)offsets(std::max(D, 1)).total);
}

size_t mlp_forward_ws_bytes(int64_t N) { return align256(sizeof(float) * (size_t)N * kH) * 2; }

void launch_mlp_forward(const uint16_t *P, int D, const float *X, int64_t N, float *logits, void *ws,
                        hipStream_t st) {
    QAIA_CHECK(D >= 1 && D <= kMaxD, QAIA_INVALID_ARGUMENT, "input width must be in [1, 16]");
    if (N == 0) return;
    char *b = (char *)ws;
    float *a1 = (float *)b, *a2 = (float *)(b + align256(sizeof(float) * (size_t)N * kH));
    hipLaunchKernelGGL(layer1_kernel, dim3(blocks_for(N * kH)), dim3(kB), 0, st, P, D, X, N, a1, nullptr);
    hipLaunchKernelGGL(layer2_kernel, dim3(blocks_for(N * kH)), dim3(kB), 0, st, P, D, a1, N, a2, nullptr);
    hipLaunchKernelGGL(head_kernel, dim3(blocks_for(N)), dim3(kB), 0, st, P, D, a2, nullptr, N, nullptr,
                       logits, nullptr, nullptr);
    QAIA_HIP(hipGetLastError());
}

void launch_mlp_backward(const uint16_t *P, int D, const float *X, const float *y, int64_t B,
                         float *grad, float *loss_logits, void *ws, hipStream_t st) {
    QAIA_CHECK(D >= 1 && D <= kMaxD, QAIA_INVALID_ARGUMENT, "input width must be in [1, 16]");
    QAIA_CHECK(B >= 1, QAIA_INVALID_ARGUMENT, "batch must be >= 1");
    char *b = (char *)ws;
    const size_t S = align256(sizeof(float) * (size_t)B * kH);
    float *a1 = (float *)b, *g1 = (float *)(b + S), *a2 = (float *)(b + 2 * S), *g2 = (float *)(b + 3 * S);
    float *dz1 = (float *)(b + 4 * S), *dz2 = (float *)(b + 5 * S), *dz3 = (float *)(b + 6 * S);
    float *partial = (float *)(b + 6 * S + align256(sizeof(float) * (size_t)B));
    hipLaunchKernelGGL(layer1_kernel, dim3(blocks_for(B * kH)), dim3(kB), 0, st, P, D, X, B, a1, g1);
    hipLaunchKernelGGL(layer2_kernel, dim3(blocks_for(B * kH)), dim3(kB), 0, st, P, D, a1, B, a2, g2);
    hipLaunchKernelGGL(head_kernel, dim3(blocks_for(B)), dim3(kB), 0, st, P, D, a2, g2, B, y, loss_logits,
                       dz3, dz2);
    hipLaunchKernelGGL(back1_kernel, dim3(blocks_for(B * kH)), dim3(kB), 0, st, P, D, dz2, g1, B, dz1);
    const int64_t total = offsets(D).total, slices = grad_slices(B);
    QAIA_CHECK(slices <= 65535, QAIA_INVALID_ARGUMENT, "batch too large");
    hipLaunchKernelGGL(grads_partial_kernel, dim3(blocks_for(total), (unsigned)slices), dim3(kB), 0, st, D, X, a1,
                       a2, dz1, dz2, dz3, B, partial);
    hipLaunchKernelGGL(grads_reduce_kernel, dim3(blocks_for(total)), dim3(kB), 0, st, partial, (int)slices, total,
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
    return 2 * align256(sizeof(float) * n) + 2 * align256(sizeof(int64_t) * n) + align256(topk_temp(N));
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
    float *keys = (float *)(b + off);
    off += align256(sizeof(float) * (size_t)N);
    float *pert = (float *)(b + off);
    off += align256(sizeof(float) * (size_t)N);
    int64_t *iota = (int64_t *)(b + off);
    off += align256(sizeof(int64_t) * (size_t)N);
    int64_t *sorted = (int64_t *)(b + off);
    off += align256(sizeof(int64_t) * (size_t)N);
    size_t tb = topk_temp(N);
    hipLaunchKernelGGL(iota64_kernel, dim3(blocks_for(N)), dim3(kB), 0, st, iota, N);
    QAIA_HIP(hipGetLastError());
    // stable: equal scores keep increasing index order
    const float *src = scores;
    if (temperature > 0.0f) {
        hipLaunchKernelGGL(gumbel_keys_kernel, dim3(blocks_for(N)), dim3(kB), 0, st, scores, N, 1.0f / temperature,
                           seed, pert);
        src = pert;
    }
    QAIA_HIP(hipcub::DeviceRadixSort::SortPairsDescending(b + off, tb, src, keys, iota, sorted, (int)N, 0,
                                                          32, st));
    if (k > 0) QAIA_HIP(hipMemcpyAsync(idx_out, sorted, sizeof(int64_t) * (size_t)k, hipMemcpyDeviceToDevice, st));
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

// Non-dominated filtering of a sample pool (section "Pareto filtering",
// dominance of Eq. 4 in cut / maximisation space) with duplicate merging.
// A sampler's pool repeats the same cuts many times (at the 42-node
// four-objective workload, 10.24 M rows hold about ten thousand distinct
// vectors), so duplicates go first.
//
// 1. Duplicate merging.  Every row looks its vector up in an open-addressing
//    hash table; each distinct vector ends with one slot holding its smallest
//    sample index (the representative).  Rows are first merged per chunk of
//    1024 in an LDS table, so that only each chunk's distinct vectors reach
//    the global one.  The occupied slots are compacted into the list of
//    distinct vectors.
// 2. Pivots.  On an evenly strided sample of that list, the row with the
//    largest normalised weighted sum is taken for each of 256 fixed positive
//    directions (a maximiser of a positive weighted sum is non-dominated, so
//    the pivots sit on or near the front).
// 3. Pruning.  A listed row is dropped when some pivot p is >= it
//    componentwise and either differs from it or has a smaller sample index.
//    Such a row is dominated, or equal to an earlier row, so it is neither on
//    the front nor a representative; every representative of the front
//    survives, and every dominated survivor keeps a surviving dominator (the
//    representative of a front vector above it), so filtering the survivors
//    gives the pool's answer.  The survivors' per-objective ranges are
//    reduced on the way.
// 4. Order the survivors lexicographically descending: one stable radix sort
//    per objective, last objective first, on the key (max_k - y_k) of only as
//    many 8-bit digits as the survivors' range of objective k needs.  This
//    order is a linear extension of dominance (y' dominates y => y' >lex y).
// 5. Chunk pass: within chunks of 1024 consecutive (distinct) vectors, a
//    vector is dropped when an earlier one in its chunk is >= it
//    componentwise.
// 6. Global pass over the chunk survivors: a survivor is kept when no earlier
//    survivor is >= it componentwise.  Any dominator of it in an earlier
//    chunk is itself dominated-or-equal by a survivor of that chunk, so
//    comparing survivors with survivors is complete.  Early exit per block.
//    Lists of at most 32768 vectors skip 5 and 6: every pair of 256-row
//    tiles is one work item of a persistent grid that marks each vector with
//    an earlier vector >= it componentwise.
// 7. The kept sample indices are emitted in ascending order by a flagged
//    compaction over 0..M-1.
// The non-dominated ranks take steps 4-6 over every row (no merging or
// pruning; equal vectors become adjacent, smallest index first, and the first
// of each run represents it).
// Every step runs on the caller's stream and every count stays on the device
// (radix.hip: launches whose pass or tile is not needed return at once).
#include <climits>

#include "radix.hpp"

namespace qaia {

namespace {

constexpr int kB = 256;
constexpr int kChunk = 1024;
constexpr int kDirs = 256;          // pivot directions
constexpr int kSampleRows = 1 << 17;  // rows of the pivot sample (at most)
constexpr int kCandBlocks = 128;     // blocks of the pivot search
constexpr int64_t kPairMax = 1 << 15;  // longest list of the pair pass (128 tiles)
constexpr int kPairBlocks = 2048;      // persistent grid of the pair pass

unsigned grid_for_n(int64_t n, int per) {
    const int64_t g = (n + per - 1) / per;
    return (unsigned)(g > 1 ? g : 1);
}

__global__ void fill_u8_kernel(uint8_t *p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = v;
}

// lo[k] = INT64_MAX, hi[k] = INT64_MIN for the range reductions
__global__ void range_init_kernel(int64_t *lo, int64_t *hi, int n) {
    if ((int)threadIdx.x < n) {
        lo[threadIdx.x] = INT64_MAX;
        hi[threadIdx.x] = INT64_MIN;
    }
}

// Fixed positive direction d over m objectives: exponential variates of a
// counter hash, i.e. a Dirichlet(1, ..., 1) draw (only their spread over the
// simplex matters).
__device__ __forceinline__ float direction(int d, int k) {
    uint64_t z = ((uint64_t)d << 8 | (uint64_t)k) * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float u = ((float)(z >> 40) + 0.5f) * (1.0f / 16777216.0f);
    return -__logf(u);
}

// A row list: position i < n names row list[i] (the identity without a list);
// n is read from device memory when d_n is given.
struct RowList {
    const int32_t *list;
    const int64_t *d_n;
    int64_t n_host;
    __device__ __forceinline__ int64_t n() const { return d_n ? *d_n : n_host; }
    __device__ __forceinline__ int64_t row(int64_t i) const { return list ? (int64_t)list[i] : i; }
};

// The pivot sample: positions s * stride, s < ns, stride = ceil(n / kSampleRows).
__device__ __forceinline__ void sample_plan(int64_t n, int64_t &stride, int64_t &ns) {
    stride = n > kSampleRows ? (n + kSampleRows - 1) / kSampleRows : 1;
    ns = (n + stride - 1) / stride;
}

// Per-objective range of the sample rows.
template <int MM>
__global__ __launch_bounds__(kB) void sample_range_kernel(const int64_t *__restrict__ obj, RowList L,
                                                          int64_t *__restrict__ lo, int64_t *__restrict__ hi) {
    __shared__ int64_t rl[MM][kB], rh[MM][kB];
    int64_t stride, ns;
    sample_plan(L.n(), stride, ns);
    int64_t a[MM], b[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        a[k] = INT64_MAX;
        b[k] = INT64_MIN;
    }
    for (int64_t s = (int64_t)blockIdx.x * kB + threadIdx.x; s < ns; s += (int64_t)gridDim.x * kB) {
        const int64_t *y = obj + L.row(s * stride) * MM;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            a[k] = min(a[k], y[k]);
            b[k] = max(b[k], y[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        rl[k][threadIdx.x] = a[k];
        rh[k][threadIdx.x] = b[k];
    }
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                rl[k][threadIdx.x] = min(rl[k][threadIdx.x], rl[k][threadIdx.x + s]);
                rh[k][threadIdx.x] = max(rh[k][threadIdx.x], rh[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if ((int)threadIdx.x < MM) {
        atomicMin((long long *)&lo[threadIdx.x], (long long)rl[threadIdx.x][0]);
        atomicMax((long long *)&hi[threadIdx.x], (long long)rh[threadIdx.x][0]);
    }
}

// Block b scans its share of the sample; thread d keeps the best row of
// direction d (largest score, then smallest row index).
template <int MM>
__global__ __launch_bounds__(kB) void pivot_cand_kernel(const int64_t *__restrict__ obj, RowList L,
                                                        const int64_t *__restrict__ lo, const int64_t *__restrict__ hi,
                                                        float *__restrict__ cscore, int32_t *__restrict__ cidx) {
    __shared__ float yn[kB][MM];
    __shared__ int32_t yi[kB];
    int64_t stride, ns;
    sample_plan(L.n(), stride, ns);
    float w[MM];
    float scale[MM];
    double off[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        w[k] = direction(threadIdx.x, k);
        off[k] = (double)lo[k];
        const double span = (double)hi[k] - (double)lo[k];
        scale[k] = span > 0.0 ? (float)(1.0 / span) : 0.0f;
    }
    float best = -1.0f;
    int32_t bidx = INT32_MAX;
    const int64_t per = (ns + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = (int64_t)blockIdx.x * per, s1 = min(ns, s0 + per);
    for (int64_t c = s0; c < s1; c += kB) {
        const int64_t s = c + threadIdx.x;
        if (s < s1) {
            const int64_t r = L.row(s * stride);
#pragma unroll
            for (int k = 0; k < MM; ++k) yn[threadIdx.x][k] = (float)(((double)obj[r * MM + k] - off[k]) * scale[k]);
            yi[threadIdx.x] = (int32_t)r;
        }
        __syncthreads();
        const int cnt = (int)min<int64_t>(kB, s1 - c);
        for (int t = 0; t < cnt; ++t) {
            float sc = 0.0f;
#pragma unroll
            for (int k = 0; k < MM; ++k) sc = fmaf(w[k], yn[t][k], sc);
            if (sc > best || (sc == best && yi[t] < bidx)) {
                best = sc;
                bidx = yi[t];
            }
        }
        __syncthreads();
    }
    cscore[(int64_t)blockIdx.x * kB + threadIdx.x] = best;
    cidx[(int64_t)blockIdx.x * kB + threadIdx.x] = bidx;
}

// One block: the best candidate of each direction over the candidate blocks,
// distinct rows only, copied into the pivot table; np = their count.
template <int MM>
__global__ __launch_bounds__(kB) void pivot_reduce_kernel(const int64_t *__restrict__ obj,
                                                          const float *__restrict__ cscore,
                                                          const int32_t *__restrict__ cidx, int nblocks,
                                                          int64_t *__restrict__ piv, int32_t *__restrict__ pidx,
                                                          int64_t *__restrict__ np) {
    __shared__ int32_t sel[kB];
    __shared__ int32_t slot[kB];
    float best = -1.0f;
    int32_t bidx = INT32_MAX;
    for (int b = 0; b < nblocks; ++b) {
        const float s = cscore[(int64_t)b * kB + threadIdx.x];
        const int32_t i = cidx[(int64_t)b * kB + threadIdx.x];
        if (s > best || (s == best && i < bidx)) {
            best = s;
            bidx = i;
        }
    }
    sel[threadIdx.x] = bidx;
    __syncthreads();
    bool first = bidx != INT32_MAX;
    for (int t = 0; t < (int)threadIdx.x && first; ++t) first = sel[t] != bidx;
    slot[threadIdx.x] = first ? 1 : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int t = 0; t < kB; ++t) {
            const int f = slot[t];
            slot[t] = f ? c : -1;
            c += f;
        }
        *np = c;
    }
    __syncthreads();
    const int p = slot[threadIdx.x];
    if (p >= 0) {
        pidx[p] = bidx;
#pragma unroll
        for (int k = 0; k < MM; ++k) piv[(int64_t)p * MM + k] = obj[(int64_t)bidx * MM + k];
    }
}

// flag[i] = 1 unless a pivot is >= row L.row(i) componentwise and differs
// from it or has a smaller index; the kept rows' per-objective range goes to
// lo / hi.
template <int MM>
__global__ __launch_bounds__(kB) void prune_kernel(const int64_t *__restrict__ obj, RowList L,
                                                   const int64_t *__restrict__ piv, const int32_t *__restrict__ pidx,
                                                   const int64_t *__restrict__ d_np, uint8_t *__restrict__ flag,
                                                   int64_t *__restrict__ lo, int64_t *__restrict__ hi) {
    __shared__ int64_t pv[kDirs][MM];
    __shared__ int32_t pi[kDirs];
    __shared__ int64_t rl[MM][kB], rh[MM][kB];
    const int np = d_np ? (int)*d_np : 0;
    const int64_t n = L.n();
    for (int p = threadIdx.x; p < np; p += kB) {
        pi[p] = pidx[p];
#pragma unroll
        for (int k = 0; k < MM; ++k) pv[p][k] = piv[(int64_t)p * MM + k];
    }
    __syncthreads();
    int64_t a[MM], b[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        a[k] = INT64_MAX;
        b[k] = INT64_MIN;
    }
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const int64_t r = L.row(i);
        int64_t y[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) y[k] = obj[r * MM + k];
        bool drop = false;
        for (int p = 0; p < np && !drop; ++p) {
            bool ge = true, ne = false;
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                ge &= pv[p][k] >= y[k];
                ne |= pv[p][k] != y[k];
            }
            drop = ge && (ne || pi[p] < r);
        }
        flag[i] = drop ? 0 : 1;
        if (!drop) {
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                a[k] = min(a[k], y[k]);
                b[k] = max(b[k], y[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        rl[k][threadIdx.x] = a[k];
        rh[k][threadIdx.x] = b[k];
    }
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                rl[k][threadIdx.x] = min(rl[k][threadIdx.x], rl[k][threadIdx.x + s]);
                rh[k][threadIdx.x] = max(rh[k][threadIdx.x], rh[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if ((int)threadIdx.x < MM) {
        atomicMin((long long *)&lo[threadIdx.x], (long long)rl[threadIdx.x][0]);
        atomicMax((long long *)&hi[threadIdx.x], (long long)rh[threadIdx.x][0]);
    }
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) p[i] = v;
}

__device__ __forceinline__ uint64_t vec_hash_step(uint64_t h, int64_t y) {
    h = (h ^ (uint64_t)y) * 0xFF51AFD7ED558CCDull;
    return h ^ (h >> 32);
}

template <int MM>
__device__ __forceinline__ uint64_t vec_hash(const int64_t (&y)[MM]) {
    uint64_t h = 0x243F6A8885A308D3ull;
#pragma unroll
    for (int k = 0; k < MM; ++k) h = vec_hash_step(h, y[k]);
    h = (h ^ (h >> 29)) * 0xC4CEB9FE1A85EC53ull;
    return h ^ (h >> 32);
}

// Open addressing in the global table of `mask + 1` slots (more than the row
// count, so a free slot always exists), linear probing from the vector's
// hash: a free slot (-1) is claimed with a compare-and-swap; a slot naming a
// row with the same vector takes min(that row, me) with an atomic minimum.
// Slots never change vector, so every row of a vector reaches the same slot,
// which ends holding the smallest row index offered for it.
template <int MM>
__device__ __forceinline__ void table_insert(const int64_t *__restrict__ obj, const int64_t (&y)[MM], uint64_t h,
                                             int32_t me, int32_t *__restrict__ table, uint64_t mask) {
    uint64_t s = h & mask;
    while (true) {
        int32_t q = table[s];
        if (q < 0) {
            q = atomicCAS(&table[s], -1, me);
            if (q < 0) return;  // claimed
        }
        bool eq = true;
#pragma unroll
        for (int k = 0; k < MM; ++k) eq &= obj[(int64_t)q * MM + k] == y[k];
        if (eq) {
            if (me < q) atomicMin(&table[s], me);
            return;
        }
        s = (s + 1) & mask;
    }
}

constexpr int kDedupRows = 1024;   // rows per chunk of the in-block merge
constexpr int kDedupSlots = 2048;  // its LDS hash slots

// Duplicate merging in two levels.  A sampler's pool repeats its most
// frequent cut vectors hundreds of thousands of times, and one global table
// slot per vector made those rows queue on a few cache lines.  So each block
// first merges a chunk of 1024 consecutive rows in an LDS table (the same
// probing, on the chunk's vectors staged in LDS, keeping the smallest row of
// the chunk per vector), and only the chunk's distinct vectors, with those
// rows, go to the global table.  The global minimum over the chunks'
// minima is the vector's smallest row.
template <int MM>
__global__ __launch_bounds__(kB) void dedupe_kernel(const int64_t *__restrict__ obj, int64_t M,
                                                    int32_t *__restrict__ table, uint64_t mask) {
    __shared__ int64_t v[kDedupRows][MM];
    __shared__ int32_t loc[kDedupSlots];
    for (int64_t c0 = (int64_t)blockIdx.x * kDedupRows; c0 < M; c0 += (int64_t)gridDim.x * kDedupRows) {
        const int len = (int)((M - c0) < kDedupRows ? (M - c0) : kDedupRows);
        for (int i = threadIdx.x; i < kDedupSlots; i += kB) loc[i] = -1;
        for (int i = threadIdx.x; i < len * MM; i += kB) (&v[0][0])[i] = obj[c0 * MM + i];
        __syncthreads();
        for (int p = threadIdx.x; p < len; p += kB) {
            int64_t y[MM];
#pragma unroll
            for (int k = 0; k < MM; ++k) y[k] = v[p][k];
            uint32_t s = (uint32_t)vec_hash<MM>(y) & (kDedupSlots - 1);
            while (true) {
                int32_t q = loc[s];
                if (q < 0) {
                    q = atomicCAS(&loc[s], -1, p);
                    if (q < 0) break;  // claimed
                }
                bool eq = true;
#pragma unroll
                for (int k = 0; k < MM; ++k) eq &= v[q][k] == y[k];
                if (eq) {
                    if (p < q) atomicMin(&loc[s], p);
                    break;
                }
                s = (s + 1) & (kDedupSlots - 1);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kDedupSlots; i += kB) {
            const int32_t p = loc[i];
            if (p < 0) continue;
            int64_t y[MM];
#pragma unroll
            for (int k = 0; k < MM; ++k) y[k] = v[p][k];
            table_insert<MM>(obj, y, vec_hash<MM>(y), (int32_t)(c0 + p), table, mask);
        }
        __syncthreads();  // v and loc are rewritten for the next chunk
    }
}

// Sort keys of objective k for the list of n = *d_n rows: key = hi_k - y_k
// (unsigned, exact), value = row.  The list is the survivors for the last
// objective, else the previous round's output (in A after an even number of
// digit passes, else in B).  Block 0 stores this round's digit-pass count.
__global__ void sort_key_kernel(const int64_t *__restrict__ obj, int m, int k, const int32_t *__restrict__ first,
                                const int64_t *__restrict__ d_n, const int64_t *__restrict__ lo,
                                const int64_t *__restrict__ hi, uint64_t *__restrict__ keyA, int32_t *valA,
                                const int32_t *valB, int32_t *__restrict__ passes) {
    const int64_t n = *d_n;
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    const uint64_t top = (uint64_t)hi[k];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t span = n > 0 ? top - (uint64_t)lo[k] : 0;
        const int bits = span ? 64 - __clzll((long long)span) : 0;
        passes[k] = (bits + 7) / 8;
    }
    if (i >= n) return;
    const int32_t *src = k == m - 1 ? first : ((passes[k + 1] & 1) ? valB : valA);
    const int32_t r = src[i];
    keyA[i] = top - (uint64_t)obj[(int64_t)r * m + k];
    valA[i] = r;
}

// sorted[i] = the final round's output (objective 0's pass parity)
__global__ void settle_kernel(const int32_t *__restrict__ valA, const int32_t *__restrict__ valB,
                              const int32_t *__restrict__ passes, const int64_t *__restrict__ d_n,
                              int32_t *__restrict__ sorted) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < *d_n) sorted[i] = (passes[0] & 1) ? valB[i] : valA[i];
}

__global__ void unique_flag_kernel(const int64_t *__restrict__ obj, int m, const int32_t *__restrict__ idx,
                                   const int64_t *__restrict__ d_n, uint8_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= *d_n) return;
    uint8_t f = 1;
    if (i > 0) {
        const int64_t *a = obj + (int64_t)idx[i] * m, *b = obj + (int64_t)idx[i - 1] * m;
        f = 0;
        for (int k = 0; k < m; ++k) f |= a[k] != b[k];
    }
    flag[i] = f;
}

// Chunk pass over the list[0 .. U) of distinct vectors in lexicographic
// order: within each chunk of 1024, flag[p] = 0 when an earlier vector of the
// chunk is >= it componentwise.  Each thread holds four rows in registers and
// walks the chunk's earlier rows once for all four (one broadcast LDS read of
// a row serves four comparisons), stopping when all four are dominated.
template <int MM>
__global__ __launch_bounds__(kB) void chunk_nd_kernel(const int64_t *__restrict__ obj,
                                                      const int32_t *__restrict__ list,
                                                      const int64_t *__restrict__ d_U, uint8_t *__restrict__ flag) {
    constexpr int RPT = kChunk / kB;  // rows per thread
    __shared__ int64_t v[kChunk][MM];
    const int64_t U = *d_U;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    if (U <= kPairMax || c0 >= U) return;  // short lists take the pair pass
    const int len = (int)((U - c0) < kChunk ? (U - c0) : kChunk);
    for (int p = threadIdx.x; p < len; p += kB) {
        const int64_t *y = obj + (int64_t)list[c0 + p] * MM;
#pragma unroll
        for (int k = 0; k < MM; ++k) v[p][k] = y[k];
    }
    __syncthreads();
    int64_t y[RPT][MM];
    bool dom[RPT];
    int last = 0;  // rows before the thread's last live row
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = r * kB + threadIdx.x;
        dom[r] = j >= len;
        if (j < len) last = j;
#pragma unroll
        for (int k = 0; k < MM; ++k) y[r][k] = j < len ? v[j][k] : 0;
    }
    for (int i = 0; i < last; ++i) {
        int64_t w[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) w[k] = v[i][k];
        bool done = true;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!dom[r] && i < r * kB + (int)threadIdx.x) {
                bool ge = true;
#pragma unroll
                for (int k = 0; k < MM; ++k) ge &= w[k] >= y[r][k];
                dom[r] = ge;
            }
            done &= dom[r];
        }
        if (done) break;
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int j = r * kB + threadIdx.x;
        if (j < len) flag[c0 + j] = dom[r] ? 0 : 1;
    }
}

// Survivor pass over sidx[0 .. S) (chunk survivors, lexicographic order): a
// survivor is kept when no earlier survivor is >= it componentwise.  Tiles of
// 256 earlier survivors pass through LDS; a block stops once all its rows are
// dominated.
template <int MM>
__global__ __launch_bounds__(kB) void global_nd_kernel(const int64_t *__restrict__ obj,
                                                       const int32_t *__restrict__ sidx,
                                                       const int64_t *__restrict__ d_U,
                                                       const int64_t *__restrict__ d_S,
                                                       uint8_t *__restrict__ keep) {
    __shared__ int64_t v[kB][MM];
    if (*d_U <= kPairMax) return;  // short lists take the pair pass
    const int64_t S = *d_S;
    const int64_t j0 = (int64_t)blockIdx.x * kB;
    if (j0 >= S) return;
    const int64_t j = j0 + threadIdx.x;
    const bool mine = j < S;
    int64_t yj[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) yj[k] = mine ? obj[(int64_t)sidx[j] * MM + k] : 0;
    bool alive = mine;
    for (int64_t i0 = 0; i0 < j0 + kB && i0 < S; i0 += kB) {
        const int64_t ii = i0 + threadIdx.x;
        if (ii < S) {
            const int64_t *y = obj + (int64_t)sidx[ii] * MM;
#pragma unroll
            for (int k = 0; k < MM; ++k) v[threadIdx.x][k] = y[k];
        }
        __syncthreads();
        if (alive) {
            const int lim = (int)((j - i0) < kB ? (j - i0) : kB);  // earlier survivors only
            for (int t = 0; t < lim; ++t) {
                bool ge = true;
#pragma unroll
                for (int k = 0; k < MM; ++k) ge &= v[t][k] >= yj[k];
                if (ge) {
                    alive = false;
                    break;
                }
            }
        }
        if (!__syncthreads_or(alive ? 1 : 0)) break;
    }
    if (alive) keep[sidx[j]] = 1;
}

// Pair pass for lists of at most kPairMax vectors (the usual case once the
// pivots have pruned a pool): the chunk and survivor passes above leave most
// CUs idle on a few thousand rows (one block per chunk, one per 256
// survivors, each walking its earlier rows in sequence), so short lists are
// instead split into 256-row tiles and every tile pair (it, jt) with
// it <= jt is one work item of a persistent grid.  Row j of tile jt is marked
// (dom[j] = 1) when a row i < j of tile it is >= it componentwise: in the
// lexicographic order every dominator comes first, and the vectors are
// distinct, so "some earlier row is >= it" is exactly "dominated".  A row
// already marked by another pair skips its comparisons, and a pair whose rows
// are all marked is skipped; concurrent marks all store the same byte.
template <int MM>
__global__ __launch_bounds__(kB) void pair_nd_kernel(const int64_t *__restrict__ obj,
                                                     const int32_t *__restrict__ list,
                                                     const int64_t *__restrict__ d_n, uint8_t *dom) {
    const int64_t n = *d_n;
    if (n > kPairMax) return;
    const int T = (int)((n + kB - 1) / kB);
    const int P = T * (T + 1) / 2;
    __shared__ int64_t v[kB][MM];
    for (int p = blockIdx.x; p < P; p += gridDim.x) {
        // p = jt (jt + 1) / 2 + it, 0 <= it <= jt
        int jt = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
        while (jt * (jt + 1) / 2 > p) --jt;
        while ((jt + 1) * (jt + 2) / 2 <= p) ++jt;
        const int it = p - jt * (jt + 1) / 2;
        const int64_t j = (int64_t)jt * kB + threadIdx.x;
        const bool live = j < n && dom[j] == 0;
        if (!__syncthreads_or(live ? 1 : 0)) continue;
        const int64_t i = (int64_t)it * kB + threadIdx.x;
        if (i < n) {
            const int64_t *y = obj + (int64_t)list[i] * MM;
#pragma unroll
            for (int k = 0; k < MM; ++k) v[threadIdx.x][k] = y[k];
        }
        __syncthreads();
        if (live) {
            int64_t yj[MM];
            const int64_t *y = obj + (int64_t)list[j] * MM;
#pragma unroll
            for (int k = 0; k < MM; ++k) yj[k] = y[k];
            // tile it < jt is full (only the last tile can be partial)
            const int lim = it < jt ? kB : (int)threadIdx.x;
            for (int t = 0; t < lim; ++t) {
                bool ge = true;
#pragma unroll
                for (int k = 0; k < MM; ++k) ge &= v[t][k] >= yj[k];
                if (ge) {
                    dom[j] = 1;
                    break;
                }
            }
        }
        __syncthreads();  // v is rewritten by the next pair
    }
}

// keep[list[j]] = 1 for the unmarked rows of a short list.
__global__ __launch_bounds__(kB) void pair_keep_kernel(const int32_t *__restrict__ list,
                                                       const int64_t *__restrict__ d_n,
                                                       const uint8_t *__restrict__ dom, uint8_t *__restrict__ keep) {
    const int64_t n = *d_n;
    const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (n <= kPairMax && j < n && dom[j] == 0) keep[list[j]] = 1;
}

// Both routes are queued; the list length, known only on the device, picks
// the one that works (the other's launches return at once).
template <int MM>
void launch_nd_passes(const int64_t *obj, const int32_t *list, const int64_t *d_n, int64_t cap, uint8_t *flag,
                      int32_t *sidx, int64_t *d_s, uint32_t *cnt, uint8_t *keep, hipStream_t st) {
    const int64_t short_cap = std::min<int64_t>(cap, kPairMax);
    const int64_t tc = (short_cap + kB - 1) / kB;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for_n(short_cap, kB)), dim3(kB), 0, st, flag, short_cap, (uint8_t)0);
    hipLaunchKernelGGL(pair_nd_kernel<MM>, dim3((unsigned)std::max<int64_t>(std::min<int64_t>(tc * (tc + 1) / 2, kPairBlocks), 1)),
                       dim3(kB), 0, st, obj, list, d_n, flag);
    hipLaunchKernelGGL(pair_keep_kernel, dim3(grid_for_n(short_cap, kB)), dim3(kB), 0, st, list, d_n, flag, keep);
    QAIA_HIP(hipGetLastError());
    if (cap <= kPairMax) return;
    hipLaunchKernelGGL(chunk_nd_kernel<MM>, dim3(grid_for_n(cap, kChunk)), dim3(kB), 0, st, obj, list, d_n, flag);
    QAIA_HIP(hipGetLastError());
    select_flagged<int32_t, int32_t>(list, flag, d_n, cap, sidx, d_s, cnt, nullptr, st);
    hipLaunchKernelGGL(global_nd_kernel<MM>, dim3(grid_for_n(cap, kB)), dim3(kB), 0, st, obj, sidx, d_n, d_s, keep);
    QAIA_HIP(hipGetLastError());
}

// The non-dominated rows of the lexicographically ordered distinct vectors
// list[0 .. n) (n = *d_n <= cap): keep[row] = 1 (keep is not cleared here).
// sidx / d_s receive the chunk survivors.
void nd_passes(const int64_t *obj, int32_t m, const int32_t *list, const int64_t *d_n, int64_t cap, uint8_t *flag,
               int32_t *sidx, int64_t *d_s, uint32_t *cnt, uint8_t *keep, hipStream_t st) {
    switch (m) {
#define QAIA_ND(MM) \
    case MM: launch_nd_passes<MM>(obj, list, d_n, cap, flag, sidx, d_s, cnt, keep, st); break;
        QAIA_ND(1)
        QAIA_ND(2)
        QAIA_ND(3)
        QAIA_ND(4)
        QAIA_ND(5)
        QAIA_ND(6)
        QAIA_ND(7)
        QAIA_ND(8)
#undef QAIA_ND
        default: throw Error{QAIA_UNSUPPORTED, "the filter supports 1..8 objectives"};
    }
}

// ranks: rows of the current list that entered rank r leave the list
__global__ void rank_assign_kernel(const int32_t *__restrict__ list, const int64_t *__restrict__ d_n,
                                   uint8_t *__restrict__ keep, int32_t r, int32_t *__restrict__ rank,
                                   uint8_t *__restrict__ rem) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= *d_n) return;
    const int32_t s = list[p];
    const bool in_front = keep[s] != 0;
    if (in_front) {
        rank[s] = r;
        keep[s] = 0;
    }
    rem[p] = in_front ? 0 : 1;
}

__global__ void rank_fill_kernel(const int32_t *__restrict__ list, int64_t n, int32_t r, int32_t *__restrict__ rank) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p < n) rank[list[p]] = r;
}

// every sorted position takes the rank of its run's representative
__global__ void rank_spread_kernel(const int32_t *__restrict__ sorted, const int32_t *__restrict__ run,
                                   const int32_t *__restrict__ uidx, int64_t M, int32_t *__restrict__ rank) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= M) return;
    const int32_t rep = uidx[run[i] - 1];
    const int32_t s = sorted[i];
    if (s != rep) rank[s] = rank[rep];
}



// Per-objective minimum over the rows of a pool (the reference point of the
// hypervolume comparisons in section "Comparison to evolutionary
// algorithm-based heuristics" is the worst value of each objective).  Each
// thread folds a strided range of rows, the block reduces in LDS, and one
// atomic min per objective and block merges the blocks.
__global__ void objective_min_init_kernel(int64_t *lo, int m) {
    if ((int)threadIdx.x < m) lo[threadIdx.x] = INT64_MAX;
}

__global__ __launch_bounds__(kB) void objective_min_kernel(const int64_t *__restrict__ obj, int64_t M, int m,
                                                           int64_t *__restrict__ lo) {
    __shared__ int64_t red[8][kB];
    int64_t mn[8];
    for (int k = 0; k < 8; ++k) mn[k] = INT64_MAX;
    for (int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x; r < M; r += (int64_t)gridDim.x * kB)
        for (int k = 0; k < m; ++k) mn[k] = min(mn[k], obj[r * m + k]);
    for (int k = 0; k < m; ++k) red[k][threadIdx.x] = mn[k];
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < m; ++k) red[k][threadIdx.x] = min(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        __syncthreads();
    }
    if ((int)threadIdx.x < m) atomicMin((long long *)&lo[threadIdx.x], (long long)red[threadIdx.x][0]);
}


// Workspace of the filter and of the ranks.  The first 64 bytes hold the
// device counts: [0] unique vectors, [1] chunk survivors, [2] rows left after
// pruning, [3] pivots.
struct PLayout {
    size_t counts = 0, passes, lo, hi, slo, shi, piv, pidx, cscore, cidx;
    size_t flag, keep, surv, keyA, keyB, valA, valB, sorted, uidx, sidx, hist, total, cnt;
    size_t table = 0;         // filter only: the duplicate-merging hash table
    uint64_t table_slots = 0;
    size_t list2 = 0, rem = 0, run = 0;  // ranks only
    size_t total_bytes = 0;
};

PLayout layout(int64_t M, bool ranks = false) {
    PLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t Mz = (size_t)std::max<int64_t>(M, 1);
    L.counts = take(8 * 8);
    L.passes = take(4 * 8);
    L.lo = take(8 * 8);
    L.hi = take(8 * 8);
    L.slo = take(8 * 8);
    L.shi = take(8 * 8);
    L.piv = take(8 * 8 * kDirs);
    L.pidx = take(4 * kDirs);
    L.cscore = take(4 * kB * kCandBlocks);
    L.cidx = take(4 * kB * kCandBlocks);
    L.flag = take(Mz);
    L.keep = take(Mz);
    L.surv = take(4 * Mz);
    L.keyA = take(8 * Mz);
    L.keyB = take(8 * Mz);
    L.valA = take(4 * Mz);
    L.valB = take(4 * Mz);
    L.sorted = take(4 * Mz);
    L.uidx = take(4 * Mz);
    L.sidx = take(4 * Mz);
    L.hist = take(4 * radix_hist_words(M));
    L.total = take(4 * 256);
    if (!ranks) {
        // a power of two of at least 1.5 M slots (load factor <= 2/3)
        uint64_t c = 1024;
        while (c < (uint64_t)Mz + Mz / 2) c <<= 1;
        L.table_slots = c;
        L.table = take(4 * c);
    }
    // per-tile counts of the compactions: over M rows, or over the table's slots
    L.cnt = take(4 * select_cnt_words(std::max<int64_t>(M, (int64_t)L.table_slots)));
    if (ranks) {
        L.list2 = take(4 * Mz);
        L.rem = take(Mz);
        L.run = take(4 * Mz);
    }
    L.total_bytes = off;
    return L;
}

unsigned grid_for(int64_t n, int per = kB) {
    int64_t g = (n + per - 1) / per;
    return (unsigned)std::max<int64_t>(g, 1);
}

struct PView {
    int64_t *counts, *lo, *hi, *slo, *shi, *piv;
    int32_t *passes, *pidx, *cidx, *surv, *valA, *valB, *sorted, *uidx, *sidx, *table;
    uint64_t table_slots;
    float *cscore;
    uint8_t *flag, *keep;
    uint64_t *keyA, *keyB;
    uint32_t *hist, *total, *cnt;
};

PView view(void *ws, const PLayout &L) {
    char *b = (char *)ws;
    PView v;
    v.counts = (int64_t *)(b + L.counts);
    v.passes = (int32_t *)(b + L.passes);
    v.lo = (int64_t *)(b + L.lo);
    v.hi = (int64_t *)(b + L.hi);
    v.slo = (int64_t *)(b + L.slo);
    v.shi = (int64_t *)(b + L.shi);
    v.piv = (int64_t *)(b + L.piv);
    v.pidx = (int32_t *)(b + L.pidx);
    v.cscore = (float *)(b + L.cscore);
    v.cidx = (int32_t *)(b + L.cidx);
    v.flag = (uint8_t *)(b + L.flag);
    v.keep = (uint8_t *)(b + L.keep);
    v.surv = (int32_t *)(b + L.surv);
    v.keyA = (uint64_t *)(b + L.keyA);
    v.keyB = (uint64_t *)(b + L.keyB);
    v.valA = (int32_t *)(b + L.valA);
    v.valB = (int32_t *)(b + L.valB);
    v.sorted = (int32_t *)(b + L.sorted);
    v.uidx = (int32_t *)(b + L.uidx);
    v.sidx = (int32_t *)(b + L.sidx);
    v.hist = (uint32_t *)(b + L.hist);
    v.total = (uint32_t *)(b + L.total);
    v.cnt = (uint32_t *)(b + L.cnt);
    v.table = L.table_slots ? (int32_t *)(b + L.table) : nullptr;
    v.table_slots = L.table_slots;
    return v;
}

template <int MM>
void launch_prune(const int64_t *obj, RowList rows, int64_t cap, bool pivots, const PView &v, hipStream_t st) {
    if (pivots) {
        const unsigned sgrid = (unsigned)std::min<int64_t>(grid_for(std::min<int64_t>(cap, kSampleRows)), 512);
        hipLaunchKernelGGL(range_init_kernel, dim3(1), dim3(64), 0, st, v.slo, v.shi, MM);
        hipLaunchKernelGGL(sample_range_kernel<MM>, dim3(sgrid), dim3(kB), 0, st, obj, rows, v.slo, v.shi);
        hipLaunchKernelGGL(pivot_cand_kernel<MM>, dim3(kCandBlocks), dim3(kB), 0, st, obj, rows, v.slo, v.shi,
                           v.cscore, v.cidx);
        hipLaunchKernelGGL(pivot_reduce_kernel<MM>, dim3(1), dim3(kB), 0, st, obj, v.cscore, v.cidx, kCandBlocks,
                           v.piv, v.pidx, v.counts + 3);
    }
    hipLaunchKernelGGL(range_init_kernel, dim3(1), dim3(64), 0, st, v.lo, v.hi, MM);
    const unsigned grid = (unsigned)std::min<int64_t>(grid_for(cap), 4096);
    hipLaunchKernelGGL(prune_kernel<MM>, dim3(grid), dim3(kB), 0, st, obj, rows, v.piv, v.pidx,
                       pivots ? (const int64_t *)(v.counts + 3) : nullptr, v.flag, v.lo, v.hi);
    QAIA_HIP(hipGetLastError());
}

// Prune the listed rows (or, without pivots, only take their range), compact
// the remaining ones and sort them lexicographically descending (ties by
// position in the list): v.sorted[0 .. counts[2]).  cap bounds the list length.
void prune_and_sort(const int64_t *obj, RowList rows, int64_t cap, int32_t m, bool pivots, const PView &v,
                    hipStream_t st) {
    switch (m) {
#define QAIA_PRUNE(MM) \
    case MM: launch_prune<MM>(obj, rows, cap, pivots, v, st); break;
        QAIA_PRUNE(1)
        QAIA_PRUNE(2)
        QAIA_PRUNE(3)
        QAIA_PRUNE(4)
        QAIA_PRUNE(5)
        QAIA_PRUNE(6)
        QAIA_PRUNE(7)
        QAIA_PRUNE(8)
#undef QAIA_PRUNE
        default: throw Error{QAIA_UNSUPPORTED, "the filter supports 1..8 objectives"};
    }
    int64_t *d_S = v.counts + 2;
    select_flagged<int32_t, int32_t>(rows.list, v.flag, rows.d_n, cap, v.surv, d_S, v.cnt, nullptr, st);
    for (int k = m - 1; k >= 0; --k) {
        hipLaunchKernelGGL(sort_key_kernel, dim3(grid_for(cap)), dim3(kB), 0, st, obj, m, k, v.surv, d_S, v.lo, v.hi,
                           v.keyA, v.valA, v.valB, v.passes);
        QAIA_HIP(hipGetLastError());
        for (int pass = 0; pass < 8; ++pass) {
            const bool even = (pass & 1) == 0;
            radix_pass(even ? v.keyA : v.keyB, even ? v.valA : v.valB, even ? v.keyB : v.keyA,
                       even ? v.valB : v.valA, cap, d_S, v.passes + k, pass, v.hist, v.total, st);
        }
    }
    hipLaunchKernelGGL(settle_kernel, dim3(grid_for(cap)), dim3(kB), 0, st, v.valA, v.valB, v.passes, d_S, v.sorted);
    QAIA_HIP(hipGetLastError());
}

template <int MM>
void launch_dedupe(const int64_t *obj, int64_t M, const PView &v, hipStream_t st) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(2048), dim3(kB), 0, st, v.table, (int64_t)v.table_slots, (int32_t)-1);
    hipLaunchKernelGGL(dedupe_kernel<MM>, dim3((unsigned)std::min<int64_t>(grid_for(M, kDedupRows), 2048)), dim3(kB),
                       0, st, obj, M, v.table, v.table_slots - 1);
    QAIA_HIP(hipGetLastError());
}

}  // namespace

size_t pareto_ws_bytes(int64_t M, int32_t m) {
    (void)m;
    return layout(M).total_bytes;
}

void launch_pareto(const int64_t *obj, int64_t M, int32_t m, int64_t *keep_idx, int64_t *num_keep,
                   void *ws, size_t ws_bytes, hipStream_t st) {
    if (M == 0) {
        hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(kB), 0, st, num_keep, (int64_t)1, (int64_t)0);
        QAIA_HIP(hipGetLastError());
        return;
    }
    const PLayout L = layout(M);
    QAIA_CHECK(ws_bytes >= L.total_bytes, QAIA_WORKSPACE_TOO_SMALL,
               "pareto filter workspace needs " + std::to_string(L.total_bytes) + " bytes");
    const PView v = view(ws, L);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(M)), dim3(kB), 0, st, v.keep, M, (uint8_t)0);
    QAIA_HIP(hipGetLastError());
    // 1. merge duplicates: uidx[0 .. U) = the smallest row of every distinct vector
    switch (m) {
#define QAIA_DEDUPE(MM) \
    case MM: launch_dedupe<MM>(obj, M, v, st); break;
        QAIA_DEDUPE(1)
        QAIA_DEDUPE(2)
        QAIA_DEDUPE(3)
        QAIA_DEDUPE(4)
        QAIA_DEDUPE(5)
        QAIA_DEDUPE(6)
        QAIA_DEDUPE(7)
        QAIA_DEDUPE(8)
#undef QAIA_DEDUPE
        default: throw Error{QAIA_UNSUPPORTED, "the filter supports 1..8 objectives"};
    }
    select_flagged<int32_t, int32_t>(v.table, nullptr, nullptr, (int64_t)v.table_slots, v.uidx, v.counts + 0, v.cnt,
                                     nullptr, st);
    // 2. prune the distinct vectors against the pivots and sort the rest
    prune_and_sort(obj, RowList{v.uidx, v.counts + 0, 0}, M, m, true, v, st);
    const int64_t *d_S = v.counts + 2;
    // 3. the sorted survivors are distinct: chunk pass, survivor pass, ascending emission
    nd_passes(obj, m, v.sorted, d_S, M, v.flag, v.sidx, v.counts + 1, v.cnt, v.keep, st);
    select_flagged<int32_t, int64_t>(nullptr, v.keep, nullptr, M, keep_idx, num_keep, v.cnt, nullptr, st);
}

void launch_objective_min(const int64_t *obj, int64_t M, int32_t m, int64_t *lo, bool accumulate,
                          hipStream_t st) {
    if (!accumulate) hipLaunchKernelGGL(objective_min_init_kernel, dim3(1), dim3(64), 0, st, lo, m);
    if (M > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>((M + kB - 1) / kB, 2048);
        hipLaunchKernelGGL(objective_min_kernel, dim3(grid), dim3(kB), 0, st, obj, M, m, lo);
    }
    QAIA_HIP(hipGetLastError());
}

size_t pareto_ranks_ws_bytes(int64_t M, int32_t m) {
    (void)m;
    return layout(M, true).total_bytes;
}

// Non-dominated sorting by peeling: sort and de-duplicate as the filter does
// (without pruning: every row needs a rank), then repeatedly take the
// non-dominated set of the remaining unique vectors (chunk pass + survivor
// pass, as above) as the next rank and remove it; the list stays in
// lexicographic order, a linear extension of dominance, which the two passes
// rely on.  Duplicates take their representative's rank.
int32_t launch_pareto_ranks(const int64_t *obj, int64_t M, int32_t m, int32_t max_rank, int32_t *rank, void *ws,
                            size_t ws_bytes, hipStream_t st) {
    if (M == 0) return 0;
    const PLayout L = layout(M, true);
    QAIA_CHECK(ws_bytes >= L.total_bytes, QAIA_WORKSPACE_TOO_SMALL,
               "pareto ranks workspace needs " + std::to_string(L.total_bytes) + " bytes");
    QAIA_CHECK(M <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many rows");
    char *b = (char *)ws;
    const PView v = view(ws, L);
    uint8_t *rem = (uint8_t *)(b + L.rem);
    int32_t *list2 = (int32_t *)(b + L.list2), *run = (int32_t *)(b + L.run);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(M)), dim3(kB), 0, st, v.keep, M, (uint8_t)0);
    QAIA_HIP(hipGetLastError());
    prune_and_sort(obj, RowList{nullptr, nullptr, M}, M, m, false, v, st);  // every row survives: counts[2] = M
    int32_t *cur = v.sorted;
    const int64_t *d_M = v.counts + 2;
    hipLaunchKernelGGL(unique_flag_kernel, dim3(grid_for(M)), dim3(kB), 0, st, obj, m, cur, d_M, v.flag);
    QAIA_HIP(hipGetLastError());
    // uidx: the representatives; run[i]: 1 + index of position i's run
    select_flagged<int32_t, int32_t>(cur, v.flag, d_M, M, v.uidx, v.counts + 0, v.cnt, run, st);
    // the working list starts as the unique representatives (a copy, uidx is kept for the spread)
    int32_t *list = v.surv, *other = list2;
    QAIA_HIP(hipMemcpyAsync(list, v.uidx, sizeof(int32_t) * (size_t)M, hipMemcpyDeviceToDevice, st));
    int64_t n = 0;
    QAIA_HIP(hipMemcpyAsync(&n, v.counts + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    QAIA_HIP(hipStreamSynchronize(st));
    int32_t r = 0;
    while (n > 0) {
        if (r == max_rank) {
            hipLaunchKernelGGL(rank_fill_kernel, dim3(grid_for(n)), dim3(kB), 0, st, list, n, r, rank);
            QAIA_HIP(hipGetLastError());
            break;
        }
        // the list length n (= counts[0]) is also known on the host here
        nd_passes(obj, m, list, v.counts + 0, n, v.flag, v.sidx, v.counts + 1, v.cnt, v.keep, st);
        hipLaunchKernelGGL(rank_assign_kernel, dim3(grid_for(n)), dim3(kB), 0, st, list, v.counts + 0, v.keep, r, rank,
                           rem);
        QAIA_HIP(hipGetLastError());
        select_flagged<int32_t, int32_t>(list, rem, nullptr, n, other, v.counts + 0, v.cnt, nullptr, st);
        std::swap(list, other);
        QAIA_HIP(hipMemcpyAsync(&n, v.counts + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        QAIA_HIP(hipStreamSynchronize(st));
        ++r;
    }
    hipLaunchKernelGGL(rank_spread_kernel, dim3(grid_for(M)), dim3(kB), 0, st, cur, run, v.uidx, M, rank);
    QAIA_HIP(hipGetLastError());
    return r;
}

}  // namespace qaia

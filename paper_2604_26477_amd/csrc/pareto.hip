// Non-dominated filtering of a sample pool (section "Pareto filtering",
// dominance of Eq. 4 in cut / maximisation space) with duplicate merging.
//
// 1. Order all M objective vectors lexicographically descending with m
//    stable radix passes (last objective first).  This order is a linear
//    extension of dominance (y' dominates y  =>  y' >lex y), and equal
//    vectors become adjacent with the smallest sample index first.
// 2. Keep the first row of every run of equal vectors (the representative).
// 3. Chunk pass: within chunks of 1024 consecutive unique vectors, a vector
//    is dropped when an earlier one in its chunk is >= it componentwise.
// 4. Global pass over the chunk survivors: a survivor is kept when no earlier
//    survivor is >= it componentwise.  Any dominator of it in an earlier
//    chunk is itself dominated-or-equal by a survivor of that chunk, so
//    comparing survivors with survivors is complete.  Early exit per block.
// 5. The kept sample indices are emitted in ascending order by a flagged
//    selection over 0..M-1.
// Every step runs on the caller's stream; counts stay on the device.
#include <hipcub/hipcub.hpp>

#include "internal.hpp"

namespace qaia {

namespace {

constexpr int kB = 256;
constexpr int kChunk = 1024;

__global__ void iota_kernel(int32_t *idx, int64_t M) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < M) idx[i] = (int32_t)i;
}

__global__ void fill_u8_kernel(uint8_t *p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void gather_key_kernel(const int64_t *__restrict__ obj, int m, int k,
                                  const int32_t *__restrict__ idx, int64_t *__restrict__ key,
                                  int64_t M) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < M) key[i] = obj[(int64_t)idx[i] * m + k];
}

__global__ void unique_flag_kernel(const int64_t *__restrict__ obj, int m,
                                   const int32_t *__restrict__ idx, uint8_t *__restrict__ flag,
                                   int64_t M) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= M) return;
    uint8_t f = 1;
    if (i > 0) {
        const int64_t *a = obj + (int64_t)idx[i] * m, *b = obj + (int64_t)idx[i - 1] * m;
        f = 0;
        for (int k = 0; k < m; ++k) f |= a[k] != b[k];
    }
    flag[i] = f;
}

// chunk-local pass over the unique vectors uidx[0..U)
__global__ __launch_bounds__(kB) void chunk_nd_kernel(const int64_t *__restrict__ obj, int m,
                                                      const int32_t *__restrict__ uidx,
                                                      const int64_t *__restrict__ d_U,
                                                      int64_t M, uint8_t *__restrict__ flag) {
    __shared__ int64_t v[8][kChunk];
    const int64_t U = *d_U;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    // positions U..M-1 still hold flags of the uniqueness pass: clear them so
    // the following selection sees survivors only
    for (int p = threadIdx.x; p < kChunk; p += kB) {
        const int64_t pos = c0 + p;
        if (pos >= U && pos < M) flag[pos] = 0;
    }
    if (c0 >= U) return;
    const int len = (int)((U - c0) < kChunk ? (U - c0) : kChunk);
    for (int p = threadIdx.x; p < len; p += kB) {
        const int64_t *y = obj + (int64_t)uidx[c0 + p] * m;
        for (int k = 0; k < m; ++k) v[k][p] = y[k];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < len; j += kB) {
        int64_t yj[8];
        for (int k = 0; k < m; ++k) yj[k] = v[k][j];
        bool dom = false;
        for (int i = 0; i < j && !dom; ++i) {
            bool ge = true;
            for (int k = 0; k < m; ++k) ge &= v[k][i] >= yj[k];
            dom = ge;
        }
        flag[c0 + j] = dom ? 0 : 1;
    }
}

// global pass over the chunk survivors sidx[0..S)
__global__ __launch_bounds__(kB) void global_nd_kernel(const int64_t *__restrict__ obj, int m,
                                                       const int32_t *__restrict__ sidx,
                                                       const int64_t *__restrict__ d_S,
                                                       uint8_t *__restrict__ keep) {
    __shared__ int64_t v[8][kB];
    const int64_t S = *d_S;
    const int64_t j0 = (int64_t)blockIdx.x * kB;
    if (j0 >= S) return;
    const int64_t j = j0 + threadIdx.x;
    const bool mine = j < S;
    int64_t yj[8];
    for (int k = 0; k < m; ++k) yj[k] = mine ? obj[(int64_t)sidx[j] * m + k] : 0;
    bool alive = mine;
    for (int64_t i0 = 0; i0 < j0 + kB && i0 < S; i0 += kB) {
        const int64_t ii = i0 + threadIdx.x;
        if (ii < S) {
            const int64_t *y = obj + (int64_t)sidx[ii] * m;
            for (int k = 0; k < m; ++k) v[k][threadIdx.x] = y[k];
        }
        __syncthreads();
        if (alive) {
            const int64_t lim = (j - i0) < kB ? (j - i0) : kB;  // earlier survivors only
            for (int64_t t = 0; t < lim; ++t) {
                bool ge = true;
                for (int k = 0; k < m; ++k) ge &= v[k][t] >= yj[k];
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

__global__ void u8_to_i32_kernel(const uint8_t *__restrict__ f, int32_t *__restrict__ o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) o[i] = f[i];
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

struct PLayout {
    size_t idxA, idxB, keyA, keyB, flag, uidx, sidx, keep, counts, temp, temp_bytes, total;
    size_t list2 = 0, rem = 0, run = 0;  // ranks only
};

size_t temp_bytes_needed(int64_t M) {
    size_t sort_b = 0, sel_b = 0, sel2_b = 0;
    hipcub::DeviceRadixSort::SortPairsDescending(nullptr, sort_b, (const int64_t *)nullptr,
                                                 (int64_t *)nullptr, (const int32_t *)nullptr,
                                                 (int32_t *)nullptr, (int)M, 0, 64, (hipStream_t)0);
    hipcub::DeviceSelect::Flagged(nullptr, sel_b, (const int32_t *)nullptr,
                                  (const uint8_t *)nullptr, (int32_t *)nullptr,
                                  (int64_t *)nullptr, M, (hipStream_t)0);
    hipcub::CountingInputIterator<int64_t> it(0);
    hipcub::DeviceSelect::Flagged(nullptr, sel2_b, it, (const uint8_t *)nullptr,
                                  (int64_t *)nullptr, (int64_t *)nullptr, M, (hipStream_t)0);
    return std::max(sort_b, std::max(sel_b, sel2_b));
}

PLayout layout(int64_t M, bool ranks = false) {
    PLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t Mz = (size_t)std::max<int64_t>(M, 1);
    L.idxA = take(4 * Mz);
    L.idxB = take(4 * Mz);
    L.keyA = take(8 * Mz);
    L.keyB = take(8 * Mz);
    L.flag = take(Mz);
    L.uidx = take(4 * Mz);
    L.sidx = take(4 * Mz);
    L.keep = take(Mz);
    L.counts = take(8 * 4);
    L.temp_bytes = temp_bytes_needed(std::max<int64_t>(M, 1));
    if (ranks) {
        L.list2 = take(4 * Mz);
        L.rem = take(Mz);
        L.run = take(4 * Mz);
        size_t scan_b = 0;
        hipcub::DeviceScan::InclusiveSum(nullptr, scan_b, (const int32_t *)nullptr, (int32_t *)nullptr,
                                         (int)std::max<int64_t>(M, 1), (hipStream_t)0);
        L.temp_bytes = std::max(L.temp_bytes, scan_b);
    }
    L.temp = take(L.temp_bytes);
    L.total = off;
    return L;
}

unsigned grid_for(int64_t n, int per = kB) {
    int64_t g = (n + per - 1) / per;
    return (unsigned)std::max<int64_t>(g, 1);
}

}  // namespace

size_t pareto_ws_bytes(int64_t M, int32_t m) {
    (void)m;
    return layout(M).total;
}

#define QAIA_CUB(call) QAIA_HIP(call)

void launch_pareto(const int64_t *obj, int64_t M, int32_t m, int64_t *keep_idx, int64_t *num_keep,
                   void *ws, size_t ws_bytes, hipStream_t st) {
    if (M == 0) {
        hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(kB), 0, st, num_keep, (int64_t)1,
                           (int64_t)0);
        QAIA_HIP(hipGetLastError());
        return;
    }
    const PLayout L = layout(M);
    QAIA_CHECK(ws_bytes >= L.total, QAIA_WORKSPACE_TOO_SMALL,
               "pareto filter workspace needs " + std::to_string(L.total) + " bytes");
    char *b = (char *)ws;
    int32_t *idxA = (int32_t *)(b + L.idxA), *idxB = (int32_t *)(b + L.idxB);
    int64_t *keyA = (int64_t *)(b + L.keyA), *keyB = (int64_t *)(b + L.keyB);
    uint8_t *flag = (uint8_t *)(b + L.flag), *keep = (uint8_t *)(b + L.keep);
    int32_t *uidx = (int32_t *)(b + L.uidx), *sidx = (int32_t *)(b + L.sidx);
    int64_t *counts = (int64_t *)(b + L.counts);
    void *temp = b + L.temp;
    size_t tb = L.temp_bytes;

    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(M)), dim3(kB), 0, st, idxA, M);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(M)), dim3(kB), 0, st, keep, M, (uint8_t)0);
    QAIA_HIP(hipGetLastError());
    int32_t *cur = idxA, *nxt = idxB;
    for (int k = m - 1; k >= 0; --k) {
        hipLaunchKernelGGL(gather_key_kernel, dim3(grid_for(M)), dim3(kB), 0, st, obj, m, k, cur,
                           keyA, M);
        QAIA_HIP(hipGetLastError());
        size_t t = tb;
        QAIA_CUB(hipcub::DeviceRadixSort::SortPairsDescending(temp, t, keyA, keyB, cur, nxt, (int)M,
                                                              0, 64, st));
        std::swap(cur, nxt);
    }
    hipLaunchKernelGGL(unique_flag_kernel, dim3(grid_for(M)), dim3(kB), 0, st, obj, m, cur, flag, M);
    QAIA_HIP(hipGetLastError());
    {
        size_t t = tb;
        QAIA_CUB(hipcub::DeviceSelect::Flagged(temp, t, cur, flag, uidx, counts + 0, M, st));
    }
    hipLaunchKernelGGL(chunk_nd_kernel, dim3(grid_for(M, kChunk)), dim3(kB), 0, st, obj, m, uidx,
                       counts + 0, M, flag);
    QAIA_HIP(hipGetLastError());
    {
        size_t t = tb;
        QAIA_CUB(hipcub::DeviceSelect::Flagged(temp, t, uidx, flag, sidx, counts + 1, M, st));
    }
    hipLaunchKernelGGL(global_nd_kernel, dim3(grid_for(M)), dim3(kB), 0, st, obj, m, sidx,
                       counts + 1, keep);
    QAIA_HIP(hipGetLastError());
    {
        size_t t = tb;
        hipcub::CountingInputIterator<int64_t> it(0);
        QAIA_CUB(hipcub::DeviceSelect::Flagged(temp, t, it, keep, keep_idx, num_keep, M, st));
    }
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
    return layout(M, true).total;
}

// Non-dominated sorting by peeling: sort and de-duplicate as the filter does,
// then repeatedly take the non-dominated set of the remaining unique vectors
// (chunk pass + survivor pass, as above) as the next rank and remove it; the
// list stays in lexicographic order, a linear extension of dominance, which
// the two passes rely on.  Duplicates take their representative's rank.
int32_t launch_pareto_ranks(const int64_t *obj, int64_t M, int32_t m, int32_t max_rank, int32_t *rank, void *ws,
                            size_t ws_bytes, hipStream_t st) {
    if (M == 0) return 0;
    const PLayout L = layout(M, true);
    QAIA_CHECK(ws_bytes >= L.total, QAIA_WORKSPACE_TOO_SMALL,
               "pareto ranks workspace needs " + std::to_string(L.total) + " bytes");
    QAIA_CHECK(M <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many rows");
    char *b = (char *)ws;
    int32_t *idxA = (int32_t *)(b + L.idxA), *idxB = (int32_t *)(b + L.idxB);
    int64_t *keyA = (int64_t *)(b + L.keyA), *keyB = (int64_t *)(b + L.keyB);
    uint8_t *flag = (uint8_t *)(b + L.flag), *keep = (uint8_t *)(b + L.keep), *rem = (uint8_t *)(b + L.rem);
    int32_t *uidx = (int32_t *)(b + L.uidx), *sidx = (int32_t *)(b + L.sidx), *list2 = (int32_t *)(b + L.list2);
    int32_t *run = (int32_t *)(b + L.run);
    int64_t *counts = (int64_t *)(b + L.counts);
    void *temp = b + L.temp;
    const size_t tb = L.temp_bytes;

    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(M)), dim3(kB), 0, st, idxA, M);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(M)), dim3(kB), 0, st, keep, M, (uint8_t)0);
    QAIA_HIP(hipGetLastError());
    int32_t *cur = idxA, *nxt = idxB;
    for (int k = m - 1; k >= 0; --k) {
        hipLaunchKernelGGL(gather_key_kernel, dim3(grid_for(M)), dim3(kB), 0, st, obj, m, k, cur, keyA, M);
        QAIA_HIP(hipGetLastError());
        size_t t = tb;
        QAIA_CUB(hipcub::DeviceRadixSort::SortPairsDescending(temp, t, keyA, keyB, cur, nxt, (int)M, 0, 64, st));
        std::swap(cur, nxt);
    }
    // cur: sorted sample indices; nxt is free from here on
    hipLaunchKernelGGL(unique_flag_kernel, dim3(grid_for(M)), dim3(kB), 0, st, obj, m, cur, flag, M);
    hipLaunchKernelGGL(u8_to_i32_kernel, dim3(grid_for(M)), dim3(kB), 0, st, flag, nxt, M);
    QAIA_HIP(hipGetLastError());
    {
        size_t t = tb;
        QAIA_CUB(hipcub::DeviceScan::InclusiveSum(temp, t, nxt, run, (int)M, st));
        t = tb;
        QAIA_CUB(hipcub::DeviceSelect::Flagged(temp, t, cur, flag, uidx, counts + 0, M, st));
    }
    // the working list starts as the unique representatives (a copy, uidx is kept for the spread)
    int32_t *list = nxt, *other = list2;
    QAIA_HIP(hipMemcpyAsync(list, uidx, sizeof(int32_t) * (size_t)M, hipMemcpyDeviceToDevice, st));
    int64_t n = 0;
    QAIA_HIP(hipMemcpyAsync(&n, counts + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    QAIA_HIP(hipStreamSynchronize(st));
    int32_t r = 0;
    while (n > 0) {
        if (r == max_rank) {
            hipLaunchKernelGGL(rank_fill_kernel, dim3(grid_for(n)), dim3(kB), 0, st, list, n, r, rank);
            QAIA_HIP(hipGetLastError());
            break;
        }
        hipLaunchKernelGGL(chunk_nd_kernel, dim3(grid_for(n, kChunk)), dim3(kB), 0, st, obj, m, list, counts + 0,
                           n, flag);
        QAIA_HIP(hipGetLastError());
        {
            size_t t = tb;
            QAIA_CUB(hipcub::DeviceSelect::Flagged(temp, t, list, flag, sidx, counts + 1, n, st));
        }
        hipLaunchKernelGGL(global_nd_kernel, dim3(grid_for(n)), dim3(kB), 0, st, obj, m, sidx, counts + 1, keep);
        hipLaunchKernelGGL(rank_assign_kernel, dim3(grid_for(n)), dim3(kB), 0, st, list, counts + 0, keep, r, rank,
                           rem);
        QAIA_HIP(hipGetLastError());
        {
            size_t t = tb;
            QAIA_CUB(hipcub::DeviceSelect::Flagged(temp, t, list, rem, other, counts + 0, n, st));
        }
        std::swap(list, other);
        QAIA_HIP(hipMemcpyAsync(&n, counts + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        QAIA_HIP(hipStreamSynchronize(st));
        ++r;
    }
    hipLaunchKernelGGL(rank_spread_kernel, dim3(grid_for(M)), dim3(kB), 0, st, cur, run, uidx, M, rank);
    QAIA_HIP(hipGetLastError());
    return r;
}

}  // namespace qaia

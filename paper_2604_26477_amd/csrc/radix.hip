// Device primitives of the Pareto filter, the non-dominated ranks and the
// top-k selection: a stable least-significant-digit radix sort of
// (64-bit key, 32-bit value) pairs with 8-bit digits, and a stable compaction
// (the flagged items of a sequence, in order), with the inclusive count of
// flags as a by-product.
//
// Both work on tiles of 4096 items (256 threads x 16 items, item j of thread t
// at tile position j * 256 + t, so loads coalesce and "tile order" is
// (j, wave, lane)).  A stable rank inside a tile comes from wave ballots: the
// lanes of a wave holding the same digit find each other with eight ballots
// (one per digit bit), a lane's rank among them is a popcount of the lower
// lanes, and per-wave counts in LDS carry the rank across the four waves and
// the sixteen rounds of a tile.  A digit pass is three launches: per-tile
// digit counts, per-digit scans over tiles (one block per digit), and the
// scatter, which adds the scanned digit totals.
//
// Item counts and pass counts are read from device memory: a caller queues
// every launch without waiting for the host, and a launch whose pass or tile
// is not needed returns at once.
#include <climits>

#include "radix.hpp"

namespace qaia {

namespace {

constexpr int kT = 256;             // threads per block
constexpr int kJ = 16;              // items per thread
constexpr int kTile = kT * kJ;      // items per tile
constexpr int kWaves = kT / 64;
constexpr int kBins = 256;

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of this wave whose 8-bit `d` equals this lane's (among `active`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t set = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? set : ~set;
    }
    return peers;
}

__device__ __forceinline__ int64_t tiles_for(int64_t n) { return (n + kTile - 1) / kTile; }

// ------------------------------------------------------------------ sort

// hist[d * stride + tile] = number of items of `tile` whose digit is d.
__global__ __launch_bounds__(kT) void radix_hist_kernel(const uint64_t *__restrict__ keys,
                                                        const int64_t *__restrict__ d_n,
                                                        const int32_t *__restrict__ d_passes, int pass,
                                                        uint32_t *__restrict__ hist, int64_t stride) {
    if (pass >= *d_passes) return;
    const int64_t n = *d_n;
    const int64_t tile = blockIdx.x;
    if (tile >= tiles_for(n)) return;
    __shared__ uint32_t h[kBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int shift = 8 * pass;
    const int64_t base = tile * kTile;
    const int lane = threadIdx.x & 63;
#pragma unroll 4
    for (int j = 0; j < kJ; ++j) {
        const int64_t i = base + j * kT + threadIdx.x;
        const bool act = i < n;
        const uint32_t d = act ? (uint32_t)(keys[i] >> shift) & 255u : 0u;
        const uint64_t peers = match_digit(d, __ballot(act));
        if (act && (__ffsll((unsigned long long)peers) - 1) == lane) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * stride + tile] = h[threadIdx.x];
}

// Exclusive scan of one digit's row hist[d * stride + 0 .. tiles) (block d);
// the row total goes to total[d].
__global__ __launch_bounds__(kT) void radix_scan_kernel(uint32_t *__restrict__ hist, const int64_t *__restrict__ d_n,
                                                        const int32_t *__restrict__ d_passes, int pass,
                                                        int64_t stride, uint32_t *__restrict__ total) {
    if (pass >= *d_passes) return;
    const int64_t tiles = tiles_for(*d_n);
    uint32_t *row = hist + (int64_t)blockIdx.x * stride;
    __shared__ uint32_t part[kT];
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < tiles; c0 += kT * 4) {
        uint32_t v[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + (int64_t)threadIdx.x * 4 + q;
            v[q] = i < tiles ? row[i] : 0u;
            s += v[q];
        }
        part[threadIdx.x] = s;
        __syncthreads();
        for (int off = 1; off < kT; off <<= 1) {  // inclusive Hillis-Steele scan of the thread sums
            const uint32_t a = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
            __syncthreads();
            part[threadIdx.x] += a;
            __syncthreads();
        }
        uint32_t run = carry + part[threadIdx.x] - s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + (int64_t)threadIdx.x * 4 + q;
            if (i < tiles) row[i] = run;
            run += v[q];
        }
        carry += part[kT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

// Stable scatter of one digit pass: out position = (items of smaller digits)
// + (items of the same digit in earlier tiles) + (rank inside the tile).
__global__ __launch_bounds__(kT) void radix_scatter_kernel(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    int32_t *__restrict__ vout, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ total,
    const int64_t *__restrict__ d_n, const int32_t *__restrict__ d_passes, int pass, int64_t stride) {
    if (pass >= *d_passes) return;
    const int64_t n = *d_n;
    const int64_t tile = blockIdx.x;
    if (tile >= tiles_for(n)) return;
    __shared__ uint32_t base[kBins];           // global start of each digit in this tile
    __shared__ uint32_t run[kBins];            // items of each digit in earlier rounds
    __shared__ uint32_t wcnt[kWaves][kBins];   // this round's per-wave digit counts
    __shared__ uint32_t scan[kBins];
    const int tid = threadIdx.x, wave = tid >> 6;
    // exclusive scan of the digit totals
    scan[tid] = total[tid];
    __syncthreads();
    for (int off = 1; off < kBins; off <<= 1) {
        const uint32_t a = tid >= off ? scan[tid - off] : 0u;
        __syncthreads();
        scan[tid] += a;
        __syncthreads();
    }
    base[tid] = scan[tid] - total[tid] + hist[(int64_t)tid * stride + tile];
    run[tid] = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int shift = 8 * pass;
    const int64_t t0 = tile * kTile;
    for (int j = 0; j < kJ; ++j) {
        const int64_t i = t0 + j * kT + tid;
        const bool act = i < n;
        uint64_t k = 0;
        int32_t v = 0;
        if (act) {
            k = kin[i];
            v = vin[i];
        }
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint64_t peers = match_digit(d, __ballot(act));
        const uint32_t below = (uint32_t)__popcll(peers & lanes_below());
        if (act && below == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (act) {
            uint32_t pre = run[d];
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            const uint32_t pos = base[d] + pre + below;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ compaction

// cnt[tile] = number of flagged items in the tile.
template <typename TIn>
__device__ __forceinline__ bool selected(const TIn *in, const uint8_t *flag, int64_t i) {
    return flag ? flag[i] != 0 : in[i] >= 0;
}

template <typename TIn>
__global__ __launch_bounds__(kT) void select_count_kernel(const TIn *__restrict__ in, const uint8_t *__restrict__ flag,
                                                          const int64_t *__restrict__ d_n, int64_t n_host,
                                                          uint32_t *__restrict__ cnt) {
    const int64_t n = d_n ? *d_n : n_host;
    const int64_t tile = blockIdx.x;
    if (tile >= tiles_for(n)) return;
    __shared__ uint32_t wsum[kWaves];
    const int64_t t0 = tile * kTile;
    uint32_t c = 0;
#pragma unroll 4
    for (int j = 0; j < kJ; ++j) {
        const int64_t i = t0 + j * kT + threadIdx.x;
        c += (i < n && selected(in, flag, i)) ? 1u : 0u;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kWaves; ++w) s += wsum[w];
        cnt[tile] = s;
    }
}

// One block: exclusive scan of cnt[0 .. tiles) in place; *count = the total.
__global__ __launch_bounds__(1024) void select_scan_kernel(uint32_t *__restrict__ cnt, const int64_t *__restrict__ d_n,
                                                           int64_t n_host, int64_t *__restrict__ count) {
    const int64_t n = d_n ? *d_n : n_host;
    const int64_t tiles = tiles_for(n);
    __shared__ int64_t part[1024];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < tiles; c0 += 1024 * 4) {
        uint32_t v[4];
        int64_t s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + (int64_t)threadIdx.x * 4 + q;
            v[q] = i < tiles ? cnt[i] : 0u;
            s += v[q];
        }
        part[threadIdx.x] = s;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t a = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += a;
            __syncthreads();
        }
        int64_t r = carry + part[threadIdx.x] - s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + (int64_t)threadIdx.x * 4 + q;
            if (i < tiles) cnt[i] = (uint32_t)r;
            r += v[q];
        }
        carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0 && count) *count = carry;
}

// Stable scatter of the selected items (flag[i] != 0, or in[i] >= 0 without
// flags): out[rank] = in ? in[i] : i.  With
// `incl`, every item also gets incl[i] = number of flagged items in 0..i.
template <typename TIn, typename TOut>
__global__ __launch_bounds__(kT) void select_scatter_kernel(const TIn *__restrict__ in,
                                                            const uint8_t *__restrict__ flag,
                                                            const int64_t *__restrict__ d_n, int64_t n_host,
                                                            const uint32_t *__restrict__ cnt, TOut *__restrict__ out,
                                                            int32_t *__restrict__ incl) {
    const int64_t n = d_n ? *d_n : n_host;
    const int64_t tile = blockIdx.x;
    if (tile >= tiles_for(n)) return;
    __shared__ uint32_t wcnt[kWaves];
    const int tid = threadIdx.x, wave = tid >> 6;
    uint32_t run = cnt[tile];
    const int64_t t0 = tile * kTile;
    for (int j = 0; j < kJ; ++j) {
        const int64_t i = t0 + j * kT + tid;
        const bool f = i < n && selected(in, flag, i);
        const uint64_t mask = __ballot(f);
        if ((tid & 63) == 0) wcnt[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t pre = run;
        for (int w = 0; w < wave; ++w) pre += wcnt[w];
        const uint32_t r = pre + (uint32_t)__popcll(mask & lanes_below());
        if (f) out[r] = in ? (TOut)in[i] : (TOut)i;
        if (incl && i < n) incl[i] = (int32_t)(r + (f ? 1u : 0u));
        for (int w = 0; w < kWaves; ++w) run += wcnt[w];
        __syncthreads();
    }
}

}  // namespace

// ------------------------------------------------------------------ host side

int64_t radix_tiles(int64_t cap) { return std::max<int64_t>((cap + kTile - 1) / kTile, 1); }

size_t radix_hist_words(int64_t cap) { return (size_t)kBins * (size_t)radix_tiles(cap); }

void radix_pass(const uint64_t *kin, const int32_t *vin, uint64_t *kout, int32_t *vout, int64_t cap,
                const int64_t *d_n, const int32_t *d_passes, int pass, uint32_t *hist, uint32_t *total,
                hipStream_t st) {
    const int64_t tiles = radix_tiles(cap);
    QAIA_CHECK(tiles <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many items to sort");
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)tiles), dim3(kT), 0, st, kin, d_n, d_passes, pass, hist,
                       tiles);
    hipLaunchKernelGGL(radix_scan_kernel, dim3(kBins), dim3(kT), 0, st, hist, d_n, d_passes, pass, tiles, total);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)tiles), dim3(kT), 0, st, kin, vin, kout, vout, hist,
                       total, d_n, d_passes, pass, tiles);
    QAIA_HIP(hipGetLastError());
}

size_t select_cnt_words(int64_t cap) { return (size_t)radix_tiles(cap); }

template <typename TIn, typename TOut>
void select_flagged(const TIn *in, const uint8_t *flag, const int64_t *d_n, int64_t cap, TOut *out, int64_t *count,
                    uint32_t *cnt, int32_t *incl, hipStream_t st) {
    const int64_t tiles = radix_tiles(cap);
    QAIA_CHECK(tiles <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many items to select");
    QAIA_CHECK(flag != nullptr || in != nullptr, QAIA_INVALID_ARGUMENT, "selection needs flags or an input list");
    hipLaunchKernelGGL(select_count_kernel<TIn>, dim3((unsigned)tiles), dim3(kT), 0, st, in, flag, d_n, cap, cnt);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, d_n, cap, count);
    hipLaunchKernelGGL((select_scatter_kernel<TIn, TOut>), dim3((unsigned)tiles), dim3(kT), 0, st, in, flag, d_n,
                       cap, cnt, out, incl);
    QAIA_HIP(hipGetLastError());
}

template void select_flagged<int32_t, int32_t>(const int32_t *, const uint8_t *, const int64_t *, int64_t, int32_t *,
                                               int64_t *, uint32_t *, int32_t *, hipStream_t);
template void select_flagged<int32_t, int64_t>(const int32_t *, const uint8_t *, const int64_t *, int64_t, int64_t *,
                                               int64_t *, uint32_t *, int32_t *, hipStream_t);

}  // namespace qaia

// Hand-written sort and compaction primitives (radix.hip); internal to libqaia.
#pragma once

#include "internal.hpp"

namespace qaia {

// Tiles of 4096 items covering `cap` items (at least one).
int64_t radix_tiles(int64_t cap);
// uint32 words of per-tile digit counts one sort pass needs for `cap` items.
size_t radix_hist_words(int64_t cap);

// One stable 8-bit digit pass (bits 8*pass .. 8*pass+7 of the key) over
// n = *d_n <= cap items: (kin, vin) -> (kout, vout).  Does nothing when
// pass >= *d_passes.  hist: radix_hist_words(cap) words; total: 256 words.
void radix_pass(const uint64_t *kin, const int32_t *vin, uint64_t *kout, int32_t *vout, int64_t cap,
                const int64_t *d_n, const int32_t *d_passes, int pass, uint32_t *hist, uint32_t *total,
                hipStream_t st);

// uint32 words of per-tile counts a compaction of `cap` items needs.
size_t select_cnt_words(int64_t cap);

// Stable compaction: for i < n (n = *d_n, or cap when d_n is null) with
// flag[i] != 0 (or, when flag is null, in[i] >= 0), in order,
// out[k++] = in ? in[i] : i; *count = k (device, may be null).
// incl (may be null): incl[i] = number of items selected in 0..i.
template <typename TIn, typename TOut>
void select_flagged(const TIn *in, const uint8_t *flag, const int64_t *d_n, int64_t cap, TOut *out, int64_t *count,
                    uint32_t *cnt, int32_t *incl, hipStream_t st);

}  // namespace qaia

// Device-wide scan and radix-sort primitives (prims.hip).
#pragma once
#include "internal.h"

namespace huge {

// Exclusive prefix sum: out[i] = sum_{j<i} in[j] (int64), *total = sum of all
// (total may be NULL).  tmp must hold scan_tmp_elems(n) int64 values.
void scan_excl(const uint32_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st);
void scan_excl(const int32_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st);

// Stable LSD radix sort of n (key, value) pairs on key bits [0, bits).
// hist: radix_sort_hist_elems(n) uint32; offs: the same count of int64;
// scan_tmp: scan_tmp_elems(radix_sort_hist_elems(n)) int64.
// Returns true when the result is in (k1, v1), false when in (k0, v0).
int64_t radix_sort_hist_elems(int64_t n);
bool radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits, uint32_t *hist,
                      int64_t *offs, int64_t *scan_tmp, hipStream_t st);

}  // namespace huge

// Device-wide scan and radix-sort primitives (prims.hip).
#pragma once
#include "internal.h"

namespace huge {

// Exclusive prefix sum: out[i] = sum_{j<i} in[j] (int64), *total = sum of all
// (total may be NULL).  tmp must hold scan_tmp_elems(n) int64 values.
void scan_excl(const uint32_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st);
void scan_excl(const int32_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st);

// The same scan with n read from device memory when the kernels run (*n_dev,
// at most nmax <= scan_devn_max()); out[n] receives the total, and nothing is
// written when n is 0.  The launches have fixed grids, so a graph can record
// them once.  tmp must hold scan_tmp_elems(nmax) int64 values.
int64_t scan_devn_max();
void scan_excl_devn(const int32_t *in, int64_t *out, const int64_t *n_dev, int64_t nmax, int64_t *tmp,
                    hipStream_t st);

// Stable LSD radix sort of n (key, value) pairs on key bits [0, bits).
// hist: radix_sort_hist_elems(n) uint32; offs: the same count of int64;
// scan_tmp: scan_tmp_elems(radix_sort_hist_elems(n)) int64.
// Returns true when the result is in (k1, v1), false when in (k0, v0).
int64_t radix_sort_hist_elems(int64_t n);
bool radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits, uint32_t *hist,
                      int64_t *offs, int64_t *scan_tmp, hipStream_t st);

}  // namespace huge

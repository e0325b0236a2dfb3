// Table operators of bushy plans (join.hip): launch parameters and launchers.
#pragma once
#include "internal.h"

namespace huge {

enum { TAB_COUNT = 0, TAB_WRITE = 1, TAB_ROOT = 2 };  // item pass: count rows, write them, or count + set-hash

// One step over a table of width w: the verify-only row filter (edges between
// columns va[t], vb[t]), then, with add, a new column: the candidates of the
// shortest Ext list inside the symmetry-breaking window, kept when every other
// Ext list holds them, distinct from the row's vertices, in the slice and with
// the label asked.  Root steps count the rows with the set-hash of the query
// edges, given as output column pairs (ea, eb).
struct TabStep {
    int32_t w = 0;
    int32_t add = 0;
    uint32_t ext = 0;
    uint32_t lo = 0, hi = 0;  // new vertex > row[c] for c in lo, < row[c] for c in hi
    int32_t nver = 0;
    int8_t va[HUGE_KMAX] = {}, vb[HUGE_KMAX] = {};
    int32_t slice = 0;
    uint32_t slice_count = 1, slice_id = 0;
    int32_t slice_mode = 0;
    int32_t label = -1;
    int32_t ne = 0;
    int8_t ea[32] = {}, eb[32] = {};
};

// PUSH-JOIN of L (width wl) and R (width wr) on the key columns kl[i] == kr[i];
// output row = L's columns, then R's columns ro[i]; nsb symmetry-breaking
// constraints out[sa[i]] < out[sb[i]]; root: the query edges as output column
// pairs.
struct JoinSpec {
    int32_t wl = 0, wr = 0;
    int32_t nkey = 0;
    int8_t kl[HUGE_KMAX] = {}, kr[HUGE_KMAX] = {};
    int32_t nro = 0;
    int8_t ro[HUGE_KMAX] = {};
    int32_t nsb = 0;
    int8_t sa[32] = {}, sb[32] = {};
    int32_t ne = 0;
    int8_t ea[32] = {}, eb[32] = {};
};

// bound[i], pinfo[i] per input row (items, probe begin | probe column << 56)
void launch_tab_prepare(const int32_t *in, int64_t n, const TabStep &S, const GraphDev &g, uint32_t *bound,
                        uint64_t *pinfo, hipStream_t st);
// items over off (exclusive prefix of bound); acc[0] rows, [1] hash_sum, [2] hash_xor, [3] overflow bits
void launch_tab_items(const int32_t *in, int64_t n, const int64_t *off, const uint64_t *pinfo, int64_t items,
                      const TabStep &S, const GraphDev &g, int mode, int32_t *out, int64_t cap,
                      unsigned long long *acc, hipStream_t st);
// R's key hashes and row indices (for the radix sort)
void launch_join_keys(const int32_t *R, int64_t nr, const JoinSpec &J, uint32_t *keys, uint32_t *vals,
                      hipStream_t st);
// per L row: the count and first index of equal key hashes in the sorted keys
void launch_join_prepare(const int32_t *L, int64_t nl, const JoinSpec &J, const uint32_t *skeys, int64_t nr,
                         uint32_t *bound, int64_t *first, unsigned long long *acc, hipStream_t st);
// out[i] = R[svals[i]] (rows of width w): R in key-hash order
void launch_gather_rows(const int32_t *R, int64_t nr, int w, const uint32_t *svals, int32_t *out, hipStream_t st);
// items over off: left row r meets sorted right rows first[r] .. first[r] + bound[r] - 1 of Rs
void launch_join_items(const int32_t *L, int64_t nl, const int32_t *Rs, const int64_t *off, const int64_t *first,
                       int64_t items, const JoinSpec &J, int mode, int32_t *out, int64_t cap, unsigned long long *acc,
                       hipStream_t st);

}  // namespace huge

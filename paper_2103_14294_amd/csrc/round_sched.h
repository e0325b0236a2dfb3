// Algorithm 5's scheduler as one step per round, for the graph engine: the
// host loop of the level engine (run until the output queue is full or the
// input is empty, move to the successor, backtrack on empty input; the SINK
// always backtracks), with its state in device memory.  One call absorbs the
// previous action's result (a segment total from the scan, or a queue length
// from the emission counters) and stops at the first step that needs kernels,
// which it writes into the state: prepare + scan n_prep[W] rows of level W,
// or extend work items [ext_w0[W], ext_w1[W]).  Host and device code: the
// graph engine runs it in a one-thread kernel, tests run it on the CPU.
#pragma once
#include "internal.h"

namespace huge {

__host__ __device__ inline int64_t sched_min(int64_t a, int64_t b) { return a < b ? a : b; }

// qcount: the emission counters (Ctrl::qcount); max_items: largest extend action
__host__ __device__ inline void round_sched_step(GState &s, const GConst &c, unsigned long long *qcount,
                                                 int64_t max_items) {
    for (int w = 0; w <= HUGE_KMAX; ++w) {
        s.n_prep[w] = 0;
        s.n_part[w] = 0;
        s.ext_w0[w] = 0;
        s.ext_w1[w] = 0;
        for (int b = 0; b <= HUGE_TUNE_BUCKETS; ++b) s.tile_next[w][b] = 0;
    }
    if (s.done) return;
    // results of the previous round's action
    if (s.last_kind == GACT_PREPARE) {
        GLevel &l = s.lv[s.last_W];
        l.seg_total = c.off[s.last_W][l.seg_n];
        s.work[s.last_W - 1] += l.seg_total;
    } else if (s.last_kind == GACT_EMIT) {
        const int w1 = s.last_W + 1;
        const int64_t nr = (int64_t)qcount[w1];
        s.cur_bytes += (nr - s.lv[w1].nrows) * 4 * w1;
        if (s.cur_bytes > s.peak_bytes) s.peak_bytes = s.cur_bytes;
        s.lv[w1].nrows = nr;
    }
    s.last_kind = GACT_NONE;
    int W = s.W;
    for (int guard = 0; guard < 8 * HUGE_KMAX; ++guard) {
        GLevel &l = s.lv[W];
        if (!s.inner) {
            if (!(l.seg_done < l.seg_total || l.next < l.nrows)) {
                // input empty: backtrack (level 2 empty: the query is done)
                if (W == 2) {
                    s.done = 1;
                    s.W = W;
                    return;
                }
                s.cur_bytes -= l.nrows * 4 * W;
                l.nrows = l.next = l.seg_row0 = l.seg_n = l.seg_total = l.seg_done = 0;
                qcount[W] = 0;
                --W;
                continue;
            }
            s.inner = 1;
        }
        // run level W until its output queue is full or its input is empty
        bool leave = false;
        if (l.seg_done == l.seg_total) {
            if (l.next == l.nrows) {
                leave = true;
            } else {
                const int64_t cnt = sched_min(c.seg_cap[W], l.nrows - l.next);
                l.seg_row0 = l.next;
                l.seg_n = cnt;
                l.next += cnt;
                l.seg_total = l.seg_done = 0;
                s.n_prep[W] = cnt;
                s.last_kind = GACT_PREPARE;
                s.last_W = W;
                s.W = W;
                s.rounds++;
                return;
            }
        }
        if (!leave) {
            const int64_t rem = l.seg_total - l.seg_done;
            if (W == c.lastW) {  // SINK: count the rest of the segment
                const int64_t chunk = sched_min(rem, max_items);
                s.ext_w0[W] = l.seg_done;
                s.ext_w1[W] = l.seg_done + chunk;
                l.seg_done += chunk;
                s.last_kind = GACT_SINK;
                s.last_W = W;
                s.W = W;
                s.rounds++;
                return;
            }
            const int64_t fr = c.q_cap[W + 1] - s.lv[W + 1].nrows;
            if (fr <= 0 || (fr < rem && fr < c.q_cap[W + 1] / 8)) {
                leave = true;  // output queue full
            } else {
                const int64_t chunk = sched_min(sched_min(fr, rem), max_items);
                s.ext_w0[W] = l.seg_done;
                s.ext_w1[W] = l.seg_done + chunk;
                l.seg_done += chunk;
                s.last_kind = GACT_EMIT;
                s.last_W = W;
                s.W = W;
                s.rounds++;
                return;
            }
        }
        // leaving level W: the SINK hands back to its precursor, any other
        // operator moves on to its successor
        s.inner = 0;
        W = (W == c.lastW) ? (W > 2 ? W - 1 : W) : W + 1;
    }
    s.error = 1;  // no action found: stop instead of spinning
    s.done = 1;
}

}  // namespace huge

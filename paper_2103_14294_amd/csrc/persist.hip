// Persistent engine (placeholder until the work-stealing kernel lands): runs
// each plan through the level engine.
#include "internal.h"

namespace huge {

void run_persistent(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                    huge_result *outs) {
    for (int i = 0; i < np; ++i) run_levels(g, plans[i], o, &outs[i], nullptr);
}

}  // namespace huge

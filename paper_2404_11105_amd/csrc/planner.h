// planner.h — host-side pattern reduction and plan generation (internal).
#pragma once
#include <stdint.h>

#include <string>

#include "plan_ir.h"

namespace xm {

// Degree statistics of a data graph, used to weight constraints.
struct GraphStats {
    uint64_t n = 0, m = 0;
    double frac_out_ge[8] = {1, 1, 1, 1, 1, 1, 1, 1};  // share of nodes with out-degree >= t
    double frac_in_ge[8] = {1, 1, 1, 1, 1, 1, 1, 1};
};

// Returns 0, -1 (bad flags) or -2 (bad pattern) with a message in err.
int build_plan(uint32_t k, uint32_t n_arcs, const uint8_t* arcs, uint32_t flags, const GraphStats* gs,
               PlanDesc& desc, std::string& json, std::string& err);

}  // namespace xm

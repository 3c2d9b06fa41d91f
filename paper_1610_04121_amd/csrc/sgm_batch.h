// Host-side layout of a batch of stereo pairs in one device workspace.
#pragma once

#include <stddef.h>

#include <string>
#include <vector>

#include "../../include/sgm.h"
#include "sgm_plan.h"

namespace sgm {

// Parameters shared by every pair of a batch.
struct BatchParams {
    int P1, P2, cw, ch;
    bool csct;
};

// Per-pair plans and workspace offsets inside one arena, plus the offset of
// the aggregation queue counter.
struct BatchLayout {
    std::vector<Plan> plans;
    std::vector<size_t> offsets;
    size_t counter_offset = 0;
    size_t total = 0;
};

bool batch_plan(const BatchParams& bp, const sgm_item* items, int n, BatchLayout& L, const char** why);

// Message returned by sgm_last_error on this thread.
void set_last_error(const std::string& msg);

}  // namespace sgm

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
    // lanes per aggregation slice for every pair: horizontal (16 or 32) and
    // other directions (16 or 32); 0 = the per-pair default
    int lanes_h = 0, lanes_v = 0;
    // workgroups of the persistent aggregation grid (4 wavefronts each); 0 =
    // as many as fill the device (512), 1 takes the queue one item per
    // wavefront at a time on one CU (a check that no result depends on the
    // order or concurrency of the work items)
    int max_workgroups = 0;
};

// Per-pair plans and workspace offsets inside one arena.
struct BatchLayout {
    std::vector<Plan> plans;
    std::vector<size_t> offsets;
    size_t total = 0;
};

// Checks every item and lays their workspaces out back to back (each
// rounded up to 256 bytes).  false with *why set if an item is invalid.
bool batch_plan(const BatchParams& bp, const sgm_item* items, int n, BatchLayout& L, const char** why);

// The left-right threshold an item's flags carry (SGM_ITEM_LR_THRESHOLD),
// 1 when they carry none.
inline int item_lr_threshold(unsigned flags) {
    return (flags & SGM_ITEM_THRESHOLD_SET) ? (int)((flags >> 16) & 0xFFu) : 1;
}

// Bytes one item's workspace takes in an arena (a multiple of 256).
size_t item_bytes(const Plan& p);

// Descriptor tables (pinned host copy + device copy) and the aggregation
// queue counter of one launch sequence.  A staging object may be reused once
// the launches that last used it have completed.
struct BatchStaging;
BatchStaging* staging_create();  // nullptr if an allocation fails
void staging_destroy(BatchStaging* st);

// Enqueues the census, cost, aggregation, sum + WTA and post launches for n
// validated items on `stream`; item i's workspace starts at ws_base[i]
// (item_bytes(plans[i]) bytes, 256-byte aligned).  Returns an SGM_ code.
int batch_enqueue(const BatchParams& bp, const Plan* plans, uint8_t* const* ws_base, const sgm_item* items,
                  int n, BatchStaging* st, hipStream_t stream);

// Message returned by sgm_last_error on this thread.
void set_last_error(const std::string& msg);

}  // namespace sgm

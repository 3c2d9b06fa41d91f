// Shapes, workspace layout and launch entry points of one SGM pipeline.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "sgm_common.h"

namespace sgm {

// Everything a launch needs to know about one stereo pair's pipeline.
struct Plan {
    int W = 0, H = 0, D = 0;   // image size, disparity levels
    int Dp = 0;                // padded levels: 64, 128 or 256
    int P1 = 0, P2 = 0;
    int n_paths = 0;
    int cw = 9, ch = 7;        // census window
    bool csct = false;         // center-symmetric census (Eq. 1)
    bool median = false, lrcheck = false;
    bool lr_full = false;      // D_R from a second SGM with the right image as base
    bool subpixel = false;     // left disparities in 1/16 pixel
    bool adaptive = false;     // P2 of each step from the base image's intensity change
    int lr_thr = 1;
    int cmax = 0;              // largest matching cost
    bool l16 = false;          // L_r stored as u16 (else u8: Cmax + P2 <= 255)
    bool nt_store = false;     // L_r stores non-temporal: the planes and cost
                               // volume of a frame exceed the memory-side cache
    bool fused = false;        // aggregation computes costs from census words
                               // instead of reading the cost volume
    bool cc_fused = false;     // cost volume from one census + cost launch (9x7)
    bool final_pass = false;   // the last direction fused with the sum and the
                               // winner-take-all (where final_pass_active)
    bool post_in_wta = false;  // the post stage inside the WTA launch (not after
                               // the final pass)
    int lanes_h = 0, lanes_v = 0;  // lanes per aggregation slice, horizontal / other
                                   // directions (16, 32, 64; 0 = default)
};

// Device workspace of one pair.  All buffers are row-major, d fastest.
struct Workspace {
    uint8_t* cost = nullptr;   // C   u8 [H][W][Dp]
    void* lbuf = nullptr;      // L_r u8|u16 [n_paths][H][W][Dp]; with lr_full the
                               // right-base planes follow: [2 * n_paths][H][W][Dp]
    uint8_t* cost_r = nullptr; // right-base C_R u8 [H][W][Dp] (lr_full only)
    uint16_t* dl = nullptr;    // raw left disparity  u16 [H][W]
    uint16_t* dr = nullptr;    // raw right disparity u16 [H][W]
    uint64_t* census_l = nullptr;  // census words of the base image u64 [H][W]
    uint64_t* census_r = nullptr;  // census words of the match image u64 [H][W]
    int* rowcnt = nullptr;     // i32 [H]: row counters of the post stage inside
                               // the WTA launch, cleared by the census launch
};

// Fills the derived fields of a plan; returns false if invalid (message set).
bool plan_finish(Plan& p, const char** why);
// A plan from sgm_create's parameters and sgm_set_options' flags and
// threshold; false if invalid (message in sgm_last_error).
bool plan_from_options(Plan& p, int w, int h, int d, int P1, int P2, int n_paths, int cw, int ch, unsigned flags,
                       int thr);
// Message returned by sgm_last_error on this thread.
void set_last_error(const std::string& msg);
// Resource events (workspace growth, graph captures) on stderr when SGM_LOG >= 2.
void log_event(const std::string& msg);
// Every device and pinned host allocation of the library goes through these:
// hipMalloc / hipHostMalloc, unless the allocation-failure hook
// (sgm_debug_fail_alloc) says this one fails (hipErrorOutOfMemory).
hipError_t dev_malloc_bytes(void** p, size_t bytes);
hipError_t pinned_malloc_bytes(void** p, size_t bytes);
template <typename T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
    return dev_malloc_bytes(reinterpret_cast<void**>(p), bytes);
}
template <typename T>
inline hipError_t pinned_malloc(T** p, size_t bytes) {
    return pinned_malloc_bytes(reinterpret_cast<void**>(p), bytes);
}
size_t workspace_bytes(const Plan& p);
// Carves a workspace out of one device allocation of workspace_bytes(p).
Workspace workspace_carve(const Plan& p, void* base);

// Enqueue the stages (all asynchronous on `stream`).
hipError_t launch_census(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right,
                         hipStream_t stream);
// right_base: C_R(x, d) from the right image's words against the left's at
// x + d, into ws.cost_r
hipError_t launch_cost(const Plan& p, const Workspace& ws, hipStream_t stream, bool right_base = false);
// Whatever the aggregation needs before it runs: the cost volume (if
// need_cost; one census + cost launch when p.cc_fused and the window is 9x7,
// else census then cost) and the census words (if the aggregation computes
// costs itself).
hipError_t launch_matching_cost(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right,
                                bool need_cost, hipStream_t stream);
bool census_cost_fusable(const Plan& p);
// left / right: the caller's images (the base images of the adaptive P2).
// skip_last: every direction but last_direction(p), whose L_r the final
// pass computes; the other planes are then numbered 0 .. n_paths - 2.
hipError_t launch_aggregate(const Plan& p, const Workspace& ws, hipStream_t stream, const uint8_t* left = nullptr,
                            const uint8_t* right = nullptr, bool skip_last = false);
// Whether the final pass replaces the last direction's aggregation and the
// WTA launch: the tuning asks for it and the plan allows it (u8 planes, the
// cost volume, no full check, no adaptive P2, its LDS fits).
bool final_pass_active(const Plan& p);
// The final pass: after launch_aggregate(..., skip_last = true); writes the
// raw maps (or `out` when no post stage follows); s_out (debug): S u16
// [H][W][D].
hipError_t launch_final_pass(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream,
                             uint16_t* s_out = nullptr);
// Aggregation and winner-take-all the way the plan runs them (the final pass
// or aggregation + WTA): raw maps, or `out` when no post stage follows.
// post_in_wta: the post stage runs inside the WTA launch (where
// post_folded(p)) and `out` gets the final map.
hipError_t launch_aggregate_wta(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right,
                                uint16_t* out, hipStream_t stream, hipEvent_t mid_event = nullptr,
                                bool post_in_wta = false);
// Whether launch_pipeline runs the post stage inside the WTA launch: the
// tuning asks for it, a post stage exists and the final pass is not used.
bool post_folded(const Plan& p);
// whether the aggregation computes costs from census words (the tuning asks
// for it and no option needs the cost volume)
bool fused_aggregation(const Plan& p);
void default_lanes(const Plan& p, int* gh, int* gv);
hipError_t launch_wta(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream,
                      bool post_in_wta = false);
hipError_t launch_post(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream);
// The direction the final pass fuses with the sum and the winner-take-all
// (Sec. 3.3): right-to-left (direction index 1), or left-to-right (index 0)
// in the 2-path set, which has no right-to-left direction.
inline int last_direction(const Plan& p) { return p.n_paths == 2 ? 0 : 1; }

// Stages of one pipeline pass, in launch order.
enum Stage { kStageCensusCost = 0, kStageAggregate = 1, kStageWta = 2, kStagePost = 3, kNumStages = 4 };

// `events` (optional, kNumStages + 1 entries) are recorded on `stream` before
// the first stage and after each stage.
hipError_t launch_pipeline(const Plan& p, const Workspace& ws, const uint8_t* left,
                           const uint8_t* right, uint16_t* out, hipStream_t stream,
                           hipEvent_t* events = nullptr);

// Debug taps.
// The packed-u16 VALU throughput probe: blocks x 256 threads, 16 VALU
// instructions per wave per round; sink holds blocks * 256 u32.
hipError_t launch_valu_probe(int blocks, int iters, uint32_t* sink, hipStream_t stream);
// Dependent-chain latency probes (mode 1: packed u16 add + min, 2: min via
// DPP row_mirror + add, 3: permlane16 swap + min + add), one chain per lane,
// 8 links per round.
hipError_t launch_valu_latency_probe(int mode, int blocks, int iters, uint32_t* sink, hipStream_t stream);
hipError_t launch_census_only(const Plan& p, const uint8_t* img, uint64_t* out,
                              hipStream_t stream);
// S = sum of the first nplanes L_r planes (-1: n_paths), leaving out plane
// `skip` (-1: none).
hipError_t launch_sum_planes(const Plan& p, const Workspace& ws, uint16_t* s_out,
                             hipStream_t stream, int skip = -1, int nplanes = -1);
// Copies plane `plane` of L_r (or the cost volume when plane < 0) out as u16
// [H][W][D].
hipError_t launch_extract_plane(const Plan& p, const Workspace& ws, int plane, uint16_t* out,
                                hipStream_t stream);

}  // namespace sgm

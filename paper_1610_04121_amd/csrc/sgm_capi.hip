// C ABI of the SGM library (declared in include/sgm.h).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <array>
#include <new>
#include <string>
#include <vector>

#include "../../include/sgm.h"
#include "sgm_batch.h"
#include "sgm_plan.h"

namespace {
thread_local std::string g_err;

// SGM_LOG: 0 (default) quiet, 1 every error message on stderr as it is set,
// 2 also resource events (workspace growth, graph captures).
int log_level() {
    static const int level = [] {
        const char* v = std::getenv("SGM_LOG");
        return v ? std::atoi(v) : 0;
    }();
    return level;
}

// allocation-failure hook: the next g_alloc_pass allocations succeed, the
// g_alloc_fail after them fail
std::atomic<long long> g_alloc_pass{0}, g_alloc_fail{0};

bool alloc_hook_fails() {
    long long f = g_alloc_fail.load();
    if (f <= 0) return false;
    for (long long p = g_alloc_pass.load(); p > 0;)
        if (g_alloc_pass.compare_exchange_weak(p, p - 1)) return false;
    for (; f > 0;)
        if (g_alloc_fail.compare_exchange_weak(f, f - 1)) return true;
    return false;
}
}  // namespace

namespace sgm {
void set_last_error(const std::string& msg) {
    g_err = msg;
    if (log_level() >= 1 && !msg.empty()) std::fprintf(stderr, "sgm: error: %s\n", msg.c_str());
}

void log_event(const std::string& msg) {
    if (log_level() >= 2) std::fprintf(stderr, "sgm: %s\n", msg.c_str());
}

hipError_t dev_malloc_bytes(void** p, size_t bytes) {
    if (alloc_hook_fails()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t pinned_malloc_bytes(void** p, size_t bytes) {
    if (alloc_hook_fails()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}
}  // namespace sgm

namespace {

int set_err(int code, const std::string& msg) {
    sgm::set_last_error(msg);
    return code;
}

int hip_err(hipError_t e, const char* what) {
    return set_err(SGM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace sgm {

bool plan_from_options(Plan& p, int w, int h, int d, int P1, int P2, int n_paths, int cw, int ch, unsigned flags,
                       int thr) {
    p.W = w;
    p.H = h;
    p.D = d;
    p.P1 = P1;
    p.P2 = P2;
    p.n_paths = n_paths;
    p.cw = cw;
    p.ch = ch;
    p.csct = (flags & SGM_CENSUS_CSCT) != 0;
    p.median = (flags & SGM_MEDIAN3) != 0;
    p.lrcheck = (flags & SGM_LRCHECK) != 0;
    p.lr_full = (flags & SGM_LR_FULL) != 0;
    p.subpixel = (flags & SGM_SUBPIXEL) != 0;
    p.adaptive = (flags & SGM_ADAPTIVE_P2) != 0;
    p.lr_thr = thr;
    const char* why = "invalid parameters";
    if (flags & ~(unsigned)(SGM_MEDIAN3 | SGM_LRCHECK | SGM_CENSUS_CSCT | SGM_GRAPH | SGM_LR_FULL | SGM_SUBPIXEL |
                            SGM_ADAPTIVE_P2)) {
        set_err(SGM_EINVAL, "unknown flag bits");
        return false;
    }
    if (p.lr_full && !p.lrcheck) {
        set_err(SGM_EINVAL, "SGM_LR_FULL needs SGM_LRCHECK");
        return false;
    }
    if (!plan_finish(p, &why)) {
        set_err(SGM_EINVAL, why);
        return false;
    }
    return true;
}

}  // namespace sgm

struct sgm_ctx {
    sgm::Plan plan;
    sgm::Workspace ws;
    void* mem = nullptr;
    size_t mem_bytes = 0;
    int device = 0;
    // stage timing: one set of kNumStages + 1 events per profiled call
    bool profiling = false;
    int profile_every = 1;  // record events on every n-th call
    long long calls = 0;
    using EventSet = std::array<hipEvent_t, sgm::kNumStages + 1>;
    std::vector<EventSet> pending, pool;
    // graph replay (SGM_GRAPH): executable graphs keyed by the caller's
    // buffers, captured on a private stream, most recently used first
    bool use_graph = false;
    struct GraphEntry {
        const void *left, *right, *out;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t capture_stream = nullptr;
};

static constexpr size_t kMaxGraphs = 8;

static void drop_graphs(sgm_ctx* c) {
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

extern "C" {

const char* sgm_last_error(void) { return g_err.c_str(); }

void sgm_debug_fail_alloc(int after, int count) {
    g_alloc_fail.store(0);
    g_alloc_pass.store(after > 0 ? after : 0);
    g_alloc_fail.store(count > 0 ? count : 0);
}

int sgm_validate(int width, int height, int max_disp, int P1, int P2, int n_paths, int census_w,
                 int census_h, unsigned flags) {
    sgm::Plan p;
    if (!sgm::plan_from_options(p, width, height, max_disp, P1, P2, n_paths, census_w, census_h, flags, 1))
        return SGM_EINVAL;
    return SGM_OK;
}

size_t sgm_footprint_bytes(int width, int height, int max_disp, int n_paths, unsigned flags) {
    // the u8/u16 choice of L_r depends on P2; count the larger case
    sgm::Plan p;
    if (!sgm::plan_from_options(p, width, height, max_disp, 0, 0, n_paths, 9, 7, flags, 1)) return 0;
    p.l16 = true;
    return sgm::workspace_bytes(p);
}

sgm_ctx* sgm_create(int width, int height, int max_disp, int P1, int P2, int n_paths, int census_w,
                    int census_h) {
    sgm::Plan p;
    if (!sgm::plan_from_options(p, width, height, max_disp, P1, P2, n_paths, census_w, census_h, 0, 1)) return nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        hip_err(e, "hipGetDevice");
        return nullptr;
    }
    sgm_ctx* c = new (std::nothrow) sgm_ctx;
    if (!c) {
        set_err(SGM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    c->plan = p;
    c->device = dev;
    // the workspace is sized for u16 L_r so that options can change later
    sgm::Plan big = p;
    big.l16 = true;
    c->mem_bytes = sgm::workspace_bytes(big);
    e = sgm::dev_malloc(&c->mem, c->mem_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_err(SGM_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
        delete c;
        return nullptr;
    }
    c->ws = sgm::workspace_carve(p, c->mem);
    // SGM_TUNE="lanes_h,lanes_v,bits": the initial kernel shape of every new
    // context (as sgm_set_tuning); a malformed or rejected value leaves the
    // default and is reported through SGM_LOG
    if (const char* env = std::getenv("SGM_TUNE")) {
        int gh = 0, gv = 0, bits = 0;
        char tail = 0;
        if (std::sscanf(env, "%d,%d,%d%c", &gh, &gv, &bits, &tail) != 3 ||
            sgm_set_tuning(c, gh, gv, bits) != SGM_OK) {
            c->plan.lanes_h = c->plan.lanes_v = 0;
            c->plan.fused = c->plan.cc_fused = c->plan.final_pass = c->plan.post_in_wta = false;
            sgm::log_event(std::string("SGM_TUNE ignored: ") + env);
            g_err.clear();
        }
    }
    return c;
}

int sgm_set_options(sgm_ctx* c, unsigned flags, int lr_threshold) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    sgm::Plan p = c->plan;
    if (!sgm::plan_from_options(p, p.W, p.H, p.D, p.P1, p.P2, p.n_paths, p.cw, p.ch, flags, lr_threshold))
        return SGM_EINVAL;
    p.lanes_h = c->plan.lanes_h;
    p.lanes_v = c->plan.lanes_v;
    p.fused = c->plan.fused;
    p.cc_fused = c->plan.cc_fused;
    p.final_pass = c->plan.final_pass;
    p.post_in_wta = c->plan.post_in_wta;
    // the full left-right check needs a second cost volume and L_r set
    sgm::Plan big = p;
    big.l16 = true;
    const size_t need = sgm::workspace_bytes(big);
    if (need > c->mem_bytes) {
        hipError_t e = hipDeviceSynchronize();  // the old workspace may still be in use
        if (e != hipSuccess) return hip_err(e, "hipDeviceSynchronize");
        void* mem = nullptr;
        e = sgm::dev_malloc(&mem, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_err(SGM_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
        }
        (void)hipFree(c->mem);
        c->mem = mem;
        c->mem_bytes = need;
        sgm::log_event("context workspace grown to " + std::to_string(need) + " bytes");
    }
    c->plan = p;
    c->ws = sgm::workspace_carve(p, c->mem);
    c->use_graph = (flags & SGM_GRAPH) != 0;
    drop_graphs(c);
    return SGM_OK;
}

static void release_events(sgm_ctx* c) {
    for (auto* v : {&c->pending, &c->pool})
        for (auto& set : *v)
            for (hipEvent_t e : set) (void)hipEventDestroy(e);
    c->pending.clear();
    c->pool.clear();
}

int sgm_set_tuning(sgm_ctx* c, int lanes_h, int lanes_v, int fused) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    auto ok = [](int g) { return g == 0 || g == 16 || g == 32 || g == 64; };
    if (!ok(lanes_h) || !ok(lanes_v)) return set_err(SGM_EINVAL, "lanes must be 0, 16, 32 or 64");
    if (lanes_v == 64) return set_err(SGM_EINVAL, "lanes_v must be 0, 16 or 32");
    if ((lanes_h == 0) != (lanes_v == 0)) return set_err(SGM_EINVAL, "set both lane counts or neither");
    if (lanes_h < lanes_v)
        return set_err(SGM_EINVAL, "lanes_h must be at least lanes_v (shapes 16/16, 32/16, 32/32, 64/16, 64/32)");
    c->plan.lanes_h = lanes_h;
    c->plan.lanes_v = lanes_v;
    if (fused & ~(SGM_TUNE_FUSED_AGG | SGM_TUNE_FUSED_CENSUS_COST | SGM_TUNE_FINAL_PASS | SGM_TUNE_POST_IN_WTA))
        return set_err(SGM_EINVAL, "unknown tuning bits");
    c->plan.fused = (fused & SGM_TUNE_FUSED_AGG) != 0;
    c->plan.cc_fused = (fused & SGM_TUNE_FUSED_CENSUS_COST) != 0;
    c->plan.final_pass = (fused & SGM_TUNE_FINAL_PASS) != 0;
    c->plan.post_in_wta = (fused & SGM_TUNE_POST_IN_WTA) != 0;
    drop_graphs(c);
    return SGM_OK;
}

int sgm_get_tuning(sgm_ctx* c, int* lanes_h, int* lanes_v, int* fused) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    int gh = c->plan.lanes_h, gv = c->plan.lanes_v;
    if (gh <= 0 || gv <= 0) sgm::default_lanes(c->plan, &gh, &gv);
    if (lanes_h) *lanes_h = gh;
    if (lanes_v) *lanes_v = gv;
    if (fused)
        *fused = (c->plan.fused ? SGM_TUNE_FUSED_AGG : 0) | (c->plan.cc_fused ? SGM_TUNE_FUSED_CENSUS_COST : 0) |
                 (c->plan.final_pass ? SGM_TUNE_FINAL_PASS : 0) | (c->plan.post_in_wta ? SGM_TUNE_POST_IN_WTA : 0);
    return SGM_OK;
}

void sgm_destroy(sgm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    release_events(c);
    drop_graphs(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->mem) (void)hipFree(c->mem);
    delete c;
}

int sgm_profile_enable(sgm_ctx* c, int every_n) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    if (every_n < 0) return set_err(SGM_EINVAL, "every_n must be >= 0");
    c->profiling = every_n > 0;
    c->profile_every = every_n > 0 ? every_n : 1;
    c->calls = 0;
    return SGM_OK;
}

int sgm_profile_read(sgm_ctx* c, double* stage_ms, int* ncalls) {
    if (!c || !stage_ms) return set_err(SGM_EINVAL, "null argument");
    for (int i = 0; i < sgm::kNumStages; ++i) stage_ms[i] = 0.0;
    int n = 0;
    for (auto& set : c->pending) {
        hipError_t e = hipEventSynchronize(set[sgm::kNumStages]);
        if (e != hipSuccess) return hip_err(e, "hipEventSynchronize");
        for (int i = 0; i < sgm::kNumStages; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, set[i], set[i + 1]);
            if (e != hipSuccess) return hip_err(e, "hipEventElapsedTime");
            stage_ms[i] += ms;
        }
        c->pool.push_back(set);
        ++n;
    }
    c->pending.clear();
    if (ncalls) *ncalls = n;
    return SGM_OK;
}

static int check_ptrs(const void* a, const void* b, const void* out) {
    if (!a || !b || !out) return set_err(SGM_EINVAL, "null buffer pointer");
    return SGM_OK;
}

int sgm_compute(sgm_ctx* c, const uint8_t* left, const uint8_t* right, uint16_t* disp_out,
                sgm_stream_t stream) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    if (int rc = check_ptrs(left, right, disp_out)) return rc;
    if ((const void*)disp_out == (const void*)left || (const void*)disp_out == (const void*)right)
        return set_err(SGM_EINVAL, "output aliases an input");
    if (c->use_graph && !c->profiling) {  // (stage timing uses eager launches)
        // replay a graph captured for these buffers, capturing it first if needed
        size_t i = 0;
        while (i < c->graphs.size() &&
               !(c->graphs[i].left == left && c->graphs[i].right == right && c->graphs[i].out == disp_out))
            ++i;
        if (i == c->graphs.size()) {
            hipError_t e = hipSuccess;
            if (!c->capture_stream) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_err(e, "hipStreamCreate");
            e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_err(e, "hipStreamBeginCapture");
            hipError_t le = sgm::launch_pipeline(c->plan, c->ws, left, right, disp_out, c->capture_stream);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(c->capture_stream, &graph);
            if (le != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_err(le, "kernel launch during capture");
            }
            if (e != hipSuccess) return hip_err(e, "hipStreamEndCapture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_err(e, "hipGraphInstantiate");
            if (c->graphs.size() == kMaxGraphs) {
                (void)hipGraphExecDestroy(c->graphs.back().exec);
                c->graphs.pop_back();
            }
            c->graphs.insert(c->graphs.begin(), {left, right, disp_out, exec});
            sgm::log_event("pipeline graph captured (" + std::to_string(c->graphs.size()) + " cached)");
            i = 0;
        } else if (i > 0) {  // to the front, keeping the others in order
            std::rotate(c->graphs.begin(), c->graphs.begin() + i, c->graphs.begin() + i + 1);
            i = 0;
        }
        hipError_t e = hipGraphLaunch(c->graphs[i].exec, (hipStream_t)stream);
        if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
        return SGM_OK;
    }
    hipEvent_t* events = nullptr;
    if (c->profiling && (c->calls++ % c->profile_every) == 0) {
        if (c->pool.empty()) {
            sgm_ctx::EventSet set;
            for (auto& ev : set) {
                hipError_t e = hipEventCreate(&ev);
                if (e != hipSuccess) return hip_err(e, "hipEventCreate");
            }
            c->pool.push_back(set);
        }
        c->pending.push_back(c->pool.back());
        c->pool.pop_back();
        events = c->pending.back().data();
    }
    hipError_t e = sgm::launch_pipeline(c->plan, c->ws, left, right, disp_out, (hipStream_t)stream, events);
    if (e != hipSuccess) return hip_err(e, "kernel launch");
    return SGM_OK;
}

int sgm_debug_census(sgm_ctx* c, const uint8_t* img, uint64_t* census_out, sgm_stream_t stream) {
    if (!c || !img || !census_out) return set_err(SGM_EINVAL, "null argument");
    hipError_t e = sgm::launch_census_only(c->plan, img, census_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_err(e, "census launch");
    return SGM_OK;
}

int sgm_debug_sums(sgm_ctx* c, const uint8_t* left, const uint8_t* right, uint16_t* s_out,
                   sgm_stream_t stream) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    if (int rc = check_ptrs(left, right, s_out)) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = sgm::launch_matching_cost(c->plan, c->ws, left, right, !sgm::fused_aggregation(c->plan), s);
    if (e == hipSuccess) e = sgm::launch_aggregate(c->plan, c->ws, s, left, right);
    if (e == hipSuccess) e = sgm::launch_sum_planes(c->plan, c->ws, s_out, s);
    if (e != hipSuccess) return hip_err(e, "kernel launch");
    return SGM_OK;
}

int sgm_debug_phase_sums(sgm_ctx* c, const uint8_t* left, const uint8_t* right, int phase, uint16_t* s_out,
                         sgm_stream_t stream) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    if (int rc = check_ptrs(left, right, s_out)) return rc;
    if (phase < 0 || phase > 1) return set_err(SGM_EINVAL, "phase must be 0 or 1");
    // the sums of the schedule the context runs: with the final pass, phase
    // 0 from the planes of the first launch and phase 1 as the final pass
    // forms them (its raw maps go to the workspace)
    sgm::Plan p = c->plan;
    p.median = true;
    const bool fp = sgm::final_pass_active(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = sgm::launch_matching_cost(p, c->ws, left, right, !sgm::fused_aggregation(p), s);
    if (e == hipSuccess) e = sgm::launch_aggregate(p, c->ws, s, left, right, fp);
    if (e == hipSuccess) {
        if (fp)
            e = phase == 0 ? sgm::launch_sum_planes(p, c->ws, s_out, s, -1, p.n_paths - 1)
                           : sgm::launch_final_pass(p, c->ws, nullptr, s, s_out);
        else
            e = sgm::launch_sum_planes(p, c->ws, s_out, s, phase == 0 ? sgm::last_direction(p) : -1);
    }
    if (e != hipSuccess) return hip_err(e, "kernel launch");
    return SGM_OK;
}

int sgm_debug_stage(sgm_ctx* c, const uint8_t* left, const uint8_t* right, int which, uint16_t* out,
                    sgm_stream_t stream) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    if (int rc = check_ptrs(left, right, out)) return rc;
    const int nplanes = c->plan.n_paths * (c->plan.lr_full ? 2 : 1);
    if (which < (c->plan.lr_full ? -2 : -1) || which >= nplanes) return set_err(SGM_EINVAL, "stage index out of range");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e =
        sgm::launch_matching_cost(c->plan, c->ws, left, right, which < 0 || !sgm::fused_aggregation(c->plan), s);
    if (e == hipSuccess && which >= 0) e = sgm::launch_aggregate(c->plan, c->ws, s, left, right);
    if (e == hipSuccess) e = sgm::launch_extract_plane(c->plan, c->ws, which, out, s);
    if (e != hipSuccess) return hip_err(e, "kernel launch");
    return SGM_OK;
}

int sgm_debug_raw_disparity(sgm_ctx* c, const uint8_t* left, const uint8_t* right, uint16_t* dl_out,
                            uint16_t* dr_out, sgm_stream_t stream) {
    if (!c) return set_err(SGM_EINVAL, "null context");
    if (int rc = check_ptrs(left, right, dl_out)) return rc;
    if (!dr_out) return set_err(SGM_EINVAL, "null buffer pointer");
    sgm::Plan p = c->plan;
    p.lrcheck = true;   // produce the right view too
    p.median = false;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = sgm::launch_matching_cost(p, c->ws, left, right, !sgm::fused_aggregation(p), s);
    if (e == hipSuccess) e = sgm::launch_aggregate_wta(p, c->ws, left, right, nullptr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dl_out, c->ws.dl, (size_t)p.W * p.H * 2, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dr_out, c->ws.dr, (size_t)p.W * p.H * 2, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(e, "kernel launch");
    return SGM_OK;
}

int sgm_debug_valu_probe(int mode, int blocks, int iters, uint32_t* sink, sgm_stream_t stream) {
    if (mode < 0 || mode > 3) return set_err(SGM_EINVAL, "mode must be 0 .. 3");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1) return set_err(SGM_EINVAL, "blocks in [1, 2^20], iters >= 1");
    if (!sink) return set_err(SGM_EINVAL, "null buffer pointer");
    hipError_t e = mode == 0 ? sgm::launch_valu_probe(blocks, iters, sink, (hipStream_t)stream)
                             : sgm::launch_valu_latency_probe(mode, blocks, iters, sink, (hipStream_t)stream);
    if (e != hipSuccess) return hip_err(e, "kernel launch");
    return SGM_OK;
}

int sgm_path_walk(int width, int height, int rx, int ry, int slice, int max_steps, int* xs, int* ys,
                  uint8_t* restart) {
    if (width < 1 || height < 1 || rx < -1 || rx > 1 || ry < -1 || ry > 1 || (rx == 0 && ry == 0))
        return set_err(SGM_EINVAL, "bad walk arguments");
    const sgm::Dir d{rx, ry};
    if (slice < 0 || slice >= sgm::slice_count(width, height, d)) return set_err(SGM_EINVAL, "slice out of range");
    const int steps = sgm::slice_steps(width, height, d);
    sgm::Walk w = sgm::walk_start(width, height, d, slice);
    int n = 0;
    for (int k = 0; k < steps && n < max_steps; ++k) {
        if (k) sgm::walk_next(width, w, d);
        if (xs) xs[n] = w.x;
        if (ys) ys[n] = w.y;
        if (restart) restart[n] = w.restart ? 1 : 0;
        ++n;
    }
    return n;
}

}  // extern "C"

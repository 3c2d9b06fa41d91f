// Batched SGM: many stereo pairs of different sizes, disparity ranges and
// path counts in one launch per stage.
//
// Census, cost, WTA and post launches flatten every pair's blocks into one
// grid; a block finds its pair by binary search over the pairs' first-block
// offsets.  The aggregation is a persistent kernel: its workgroups take
// quads of work items (pair, direction, group of slices; one item per
// wavefront) from a queue in device memory, longest slices first, through a
// vector atomic counter that the census launch resets (no memset, so the
// launches can also be graph-captured).  Items are independent within the
// aggregation: the wavefronts of a workgroup meet at a barrier between
// quads, no workgroup ever waits for another, and every workgroup leaves the
// loop when the queue is empty.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sgm.h"
#include "sgm_batch.h"
#include "sgm_device.h"
#include "sgm_plan.h"

namespace sgm {

namespace {

using namespace dev;

// One pair as the batched kernels see it.
struct BatchItem {
    const uint8_t* left;
    const uint8_t* right;
    uint16_t* out;
    uint64_t* census_l;
    uint64_t* census_r;
    uint8_t* cost;
    uint8_t* cost_r;  // right-base costs (lr_full), else nullptr
    void* lbuf;       // L_r planes; with lr_full the right-base planes follow
    uint16_t* dl;
    uint16_t* dr;
    int W, H, D, Dp, P, cmax, l16, median, lrcheck, thr, csct, gh, gv, subpixel, lr_full, adaptive;
    int census_blk0, cost_blk0, wta_blk0, post_blk0;  // first block in each launch
};

// One aggregation work item: S = 64 / G slices of one direction of one pair;
// rb = 1 for a direction of the right-base SGM (full left-right check);
// item = -1 marks an empty place of a quad.
struct WorkItem {
    int item, plane, rx, ry, first, steps, rb;
};

// Work items go out four at a time, one per wavefront of a workgroup (a
// quad).  Opposite directions over the same pixels share a quad (A, A, B,
// B): the axis-aligned ones over the same two slice groups, the diagonals
// over the groups that cover (most of) the same pixels.  Both walks over a
// pixel's costs then run on one CU and its L2, and the second read can hit
// there, as in the single-pair aggregation launch.
constexpr int kQuad = 4;

// Index of the pair whose block range [blk0, next blk0) holds block b.
template <int BatchItem::*FIRST>
__device__ inline int find_item(const BatchItem* items, int n, int b) {
    int lo = 0, hi = n;  // items[lo].*FIRST <= b < items[hi].*FIRST
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid].*FIRST <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void census_batch_kernel(const BatchItem* items, int n, int generic, int rx,
                                                           int ry, unsigned* queue_counter) {
    const int b = blockIdx.x;
    if (b == 0 && threadIdx.x == 0) *queue_counter = 0u;  // the aggregation launch follows
    const int i = find_item<&BatchItem::census_blk0>(items, n, b);
    const BatchItem& it = items[i];
    const int local = b - it.census_blk0;
    CensusArgs a{{it.left, it.right}, {it.census_l, it.census_r}, it.W, it.H, it.csct};
    if (!generic) {
        const int nx = (it.W + kCenTX - 1) / kCenTX, ny = (it.H + kCenTY - 1) / kCenTY;
        const int z = local / (nx * ny), rem = local - z * nx * ny;
        census97_block(a, rem % nx, rem / nx, z);
    } else {
        const int nx = (it.W + 15) / 16, ny = (it.H + 15) / 16;
        const int z = local / (nx * ny), rem = local - z * nx * ny;
        census_generic_block(a, rx, ry, rem % nx, rem / nx, z);
    }
}

// Blocks 0 .. nx * H - 1 of a pair make its cost volume; with the full
// left-right check, the next nx * H make the right-base costs.
template <bool RB>
__device__ inline void cost_batch_block(const BatchItem& it, int bx, int y, uint64_t* smem) {
    const CostArgs a = RB ? CostArgs{it.census_r, it.census_l, it.cost_r, it.W, it.H, it.D, it.Dp, it.cmax}
                          : CostArgs{it.census_l, it.census_r, it.cost, it.W, it.H, it.D, it.Dp, it.cmax};
    if (it.Dp == 64)
        cost_block<RB, 64>(a, bx, y, smem);
    else if (it.Dp == 128)
        cost_block<RB, 128>(a, bx, y, smem);
    else
        cost_block<RB, 256>(a, bx, y, smem);
}

__global__ __launch_bounds__(kCostThreads) void cost_batch_kernel(const BatchItem* items, int n) {
    extern __shared__ __align__(16) uint64_t cost_smem[];
    const int b = blockIdx.x;
    const BatchItem& it = items[find_item<&BatchItem::cost_blk0>(items, n, b)];
    int local = b - it.cost_blk0;
    const int nx = (it.W + kCostTX - 1) / kCostTX;
    if (local < nx * it.H) {
        cost_batch_block<false>(it, local % nx, local / nx, cost_smem);
    } else {
        local -= nx * it.H;
        cost_batch_block<true>(it, local % nx, local / nx, cost_smem);
    }
}

// NT: non-temporal L_r stores (the batch's planes exceed the memory-side
// cache); ADAPT: adaptive P2 (the block's penalty table is in s.p2lut).
template <typename LT, int Dp, bool NT, bool ADAPT>
__device__ __attribute__((always_inline)) inline void aggregate_item(const SliceArgs& s, int kind, int g, int first,
                                                                     int lane) {
    if (kind == kHoriz) {
        if (g == 32)
            aggregate_wave<32, Dp / 32, LT, kHoriz, false, ADAPT, NT>(s, first, lane);
        else
            aggregate_wave<16, Dp / 16, LT, kHoriz, false, ADAPT, NT>(s, first, lane);
    } else if (kind == kVert) {
        if (g == 32)
            aggregate_wave<32, Dp / 32, LT, kVert, false, ADAPT, NT>(s, first, lane);
        else
            aggregate_wave<16, Dp / 16, LT, kVert, false, ADAPT, NT>(s, first, lane);
    } else {
        if (g == 32)
            aggregate_wave<32, Dp / 32, LT, kDiag, false, ADAPT, NT>(s, first, lane);
        else
            aggregate_wave<16, Dp / 16, LT, kDiag, false, ADAPT, NT>(s, first, lane);
    }
}

// g: the work item's lanes per slice (its pair's horizontal or other group
// width, by the direction's kind)
template <typename LT, bool NT, bool ADAPT>
__device__ __attribute__((always_inline)) inline void aggregate_item_dp(const SliceArgs& s, int Dp, int kind, int g,
                                                                        int first, int lane) {
    if (Dp == 64)
        aggregate_item<LT, 64, NT, ADAPT>(s, kind, g, first, lane);
    else if (Dp == 128)
        aggregate_item<LT, 128, NT, ADAPT>(s, kind, g, first, lane);
    else
        aggregate_item<LT, 256, NT, ADAPT>(s, kind, g, first, lane);
}

// ANY_ADAPT: some pair of the batch uses the adaptive P2 (a second
// instantiation, so batches without one keep the smaller kernel).  A
// workgroup takes one quad of work items at a time, wavefront k its item k;
// the quad's items have the same length, so its wavefronts finish together.
template <bool NT, bool ANY_ADAPT>
__global__ __launch_bounds__(256) void aggregate_batch_kernel(const BatchItem* items, const WorkItem* work,
                                                              int nquads, unsigned* queue_counter, int P1, int P2) {
    __shared__ uint16_t p2lut[ANY_ADAPT ? 256 : 1];
    __shared__ unsigned quad;
    if constexpr (ANY_ADAPT)  // P1, P2 belong to the batch: one table per block
        fill_p2_lut(p2lut, P1, P2);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (;;) {
        // the barrier also ends every wavefront's read of the previous quad
        // index (and, on the first pass, the penalty table's fill)
        __syncthreads();
        if (threadIdx.x == 0) quad = atomicAdd(queue_counter, 1u);
        __syncthreads();
        const unsigned q = __builtin_amdgcn_readfirstlane(quad);
        if (q >= (unsigned)nquads) break;
        const WorkItem w = work[(size_t)q * kQuad + wave];
        if (w.item < 0) continue;
        const BatchItem& it = items[w.item];
        const uint32_t plane = (uint32_t)it.W * (uint32_t)it.H * (uint32_t)it.Dp;
        void* lplane = it.l16 ? (void*)(reinterpret_cast<uint16_t*>(it.lbuf) + (size_t)plane * w.plane)
                              : (void*)(reinterpret_cast<uint8_t*>(it.lbuf) + (size_t)plane * w.plane);
        // a right-base direction reads the right-base costs; the adaptive P2
        // follows its SGM's base image
        SliceArgs s{w.rb ? it.cost_r : it.cost, it.census_l, it.census_r, lplane, plane, it.W, it.H, it.D, P1, P2,
                    it.cmax, w.rx, w.ry};
        s.img = w.rb ? it.right : it.left;
        s.p2lut = ANY_ADAPT ? p2lut : nullptr;
        const int kind = w.ry == 0 ? kHoriz : (w.rx == 0 ? kVert : kDiag);
        const int g = kind == kHoriz ? it.gh : it.gv;
        if (ANY_ADAPT && it.adaptive) {
            if (it.l16)
                aggregate_item_dp<uint16_t, NT, ANY_ADAPT>(s, it.Dp, kind, g, w.first, lane);
            else
                aggregate_item_dp<uint8_t, NT, ANY_ADAPT>(s, it.Dp, kind, g, w.first, lane);
        } else {
            if (it.l16)
                aggregate_item_dp<uint16_t, NT, false>(s, it.Dp, kind, g, w.first, lane);
            else
                aggregate_item_dp<uint8_t, NT, false>(s, it.Dp, kind, g, w.first, lane);
        }
    }
}

// Blocks 0 .. H - 1 of a pair are its rows; with the full left-right check
// blocks H .. 2H - 1 are the rows of the right-base SGM, whose winners are
// D_R.
template <bool NT>
__global__ __launch_bounds__(1024) void wta_batch_kernel(const BatchItem* items, int n) {
    extern __shared__ uint32_t wta_smem[];
    const int b = blockIdx.x;
    const BatchItem& it = items[find_item<&BatchItem::wta_blk0>(items, n, b)];
    const bool post = it.median || it.lrcheck;
    const size_t plane = (size_t)it.W * it.H * it.Dp;
    int y = b - it.wta_blk0;
    WtaArgs a{it.lbuf, plane, post ? it.dl : it.out, (it.lrcheck && !it.lr_full) ? it.dr : nullptr,
              it.W, it.H, it.D, it.Dp, it.P, it.subpixel};
    if (y >= it.H) {  // right-base rows: planes P .. 2P - 1, winners into D_R
        y -= it.H;
        a.lbuf = static_cast<const uint8_t*>(it.lbuf) + plane * it.P * (it.l16 ? 2 : 1);
        a.dl = it.dr;
        a.dr = nullptr;
        a.subpixel = 0;
    }
    if (it.l16)
        wta_row<uint16_t, NT>(a, y, wta_smem);
    else
        wta_row<uint8_t, NT>(a, y, wta_smem);
}

__global__ __launch_bounds__(256) void post_batch_kernel(const BatchItem* items, int n) {
    extern __shared__ uint16_t post_smem[];
    const int b = blockIdx.x;
    const BatchItem& it = items[find_item<&BatchItem::post_blk0>(items, n, b)];
    PostArgs a{it.dl, it.dr, it.out, it.W, it.H, it.median, it.lrcheck, it.thr, it.subpixel};
    post_row(a, b - it.post_blk0, post_smem);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
bool batch_plan(const BatchParams& bp, const sgm_item* items, int n, BatchLayout& L, const char** why) {
    L.plans.clear();
    L.offsets.clear();
    L.total = 0;
    if (n < 0 || (n > 0 && !items)) {
        *why = "bad item array";
        return false;
    }
    for (int i = 0; i < n; ++i) {
        const sgm_item& it = items[i];
        Plan p;
        p.W = it.w;
        p.H = it.h;
        p.D = it.max_disp;
        p.P1 = bp.P1;
        p.P2 = bp.P2;
        p.n_paths = it.n_paths;
        p.cw = bp.cw;
        p.ch = bp.ch;
        p.csct = bp.csct || (it.flags & SGM_CENSUS_CSCT) != 0;
        p.median = (it.flags & SGM_MEDIAN3) != 0;
        p.lrcheck = (it.flags & SGM_LRCHECK) != 0;
        p.subpixel = (it.flags & SGM_SUBPIXEL) != 0;
        p.lr_full = (it.flags & SGM_LR_FULL) != 0;
        p.adaptive = (it.flags & SGM_ADAPTIVE_P2) != 0;
        p.lr_thr = item_lr_threshold(it.flags);
        if (it.flags & ~(unsigned)(SGM_MEDIAN3 | SGM_LRCHECK | SGM_SUBPIXEL | SGM_LR_FULL | SGM_ADAPTIVE_P2 |
                                   SGM_CENSUS_CSCT | SGM_ITEM_THRESHOLD_SET | 0x00FF0000u)) {
            *why = "item flags may only hold SGM_MEDIAN3, SGM_LRCHECK, SGM_SUBPIXEL, SGM_LR_FULL, SGM_ADAPTIVE_P2, "
                   "SGM_CENSUS_CSCT and SGM_ITEM_LR_THRESHOLD(t)";
            return false;
        }
        if (p.lr_full && !p.lrcheck) {
            *why = "SGM_LR_FULL needs SGM_LRCHECK";
            return false;
        }
        if (!plan_finish(p, why)) return false;
        L.offsets.push_back(L.total);
        L.total += item_bytes(p);
        L.plans.push_back(p);
    }
    return true;
}

size_t item_bytes(const Plan& p) { return align256(workspace_bytes(p)); }

struct BatchStaging {
    BatchItem* d_items = nullptr;
    WorkItem* d_work = nullptr;
    size_t items_cap = 0, work_cap = 0;
    BatchItem* h_items = nullptr;  // pinned
    WorkItem* h_work = nullptr;
    unsigned* counter = nullptr;   // aggregation queue head (device)
    hipEvent_t staged = nullptr;   // the last copy out of the pinned tables
    bool staged_pending = false;
};

BatchStaging* staging_create() {
    BatchStaging* st = new (std::nothrow) BatchStaging;
    if (!st) return nullptr;
    if (sgm::dev_malloc((void**)&st->counter, 256) != hipSuccess ||
        hipEventCreateWithFlags(&st->staged, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        staging_destroy(st);
        return nullptr;
    }
    return st;
}

void staging_destroy(BatchStaging* st) {
    if (!st) return;
    if (st->staged_pending) (void)hipEventSynchronize(st->staged);
    if (st->d_items) (void)hipFree(st->d_items);
    if (st->d_work) (void)hipFree(st->d_work);
    if (st->h_items) (void)hipHostFree(st->h_items);
    if (st->h_work) (void)hipHostFree(st->h_work);
    if (st->counter) (void)hipFree(st->counter);
    if (st->staged) (void)hipEventDestroy(st->staged);
    delete st;
}

namespace {

int berr(int code, const std::string& m) {
    set_last_error(m);
    return code;
}

int bhip(hipError_t e, const char* what) { return berr(SGM_EHIP, std::string(what) + ": " + hipGetErrorString(e)); }

// Grows the tables; waits first for the last copy out of the pinned ones.
int grow_staging(BatchStaging* b, size_t nitems, size_t nwork) {
    if (b->staged_pending) {
        hipError_t e = hipEventSynchronize(b->staged);
        if (e != hipSuccess) return bhip(e, "hipEventSynchronize");
        b->staged_pending = false;
    }
    if (nitems > b->items_cap) {
        size_t cap = std::max(nitems, 2 * b->items_cap);
        if (b->h_items) (void)hipHostFree(b->h_items);
        if (b->d_items) (void)hipFree(b->d_items);
        b->h_items = nullptr;
        b->d_items = nullptr;
        b->items_cap = 0;
        if (sgm::pinned_malloc((void**)&b->h_items, cap * sizeof(BatchItem)) != hipSuccess ||
            sgm::dev_malloc((void**)&b->d_items, cap * sizeof(BatchItem)) != hipSuccess) {
            (void)hipGetLastError();
            return berr(SGM_ENOMEM, "batch descriptor allocation failed");
        }
        b->items_cap = cap;
    }
    if (nwork > b->work_cap) {
        size_t cap = std::max(nwork, 2 * b->work_cap);
        if (b->h_work) (void)hipHostFree(b->h_work);
        if (b->d_work) (void)hipFree(b->d_work);
        b->h_work = nullptr;
        b->d_work = nullptr;
        b->work_cap = 0;
        if (sgm::pinned_malloc((void**)&b->h_work, cap * sizeof(WorkItem)) != hipSuccess ||
            sgm::dev_malloc((void**)&b->d_work, cap * sizeof(WorkItem)) != hipSuccess) {
            (void)hipGetLastError();
            return berr(SGM_ENOMEM, "batch work-queue allocation failed");
        }
        b->work_cap = cap;
    }
    return SGM_OK;
}

}  // namespace

// Everything one batch's launches take, built on the host: the descriptor
// and work tables and the launch shapes.
struct BatchLaunch {
    std::vector<BatchItem> desc;
    std::vector<WorkItem> work;
    size_t census_blocks = 0, cost_blocks = 0, wta_blocks = 0, post_blocks = 0;
    size_t cost_smem = 0, wta_smem = 0, post_smem = 0;
    bool generic = false, any_adapt = false, nt = false;
    int blocks = 0;  // persistent aggregation workgroups
};

int batch_build(const BatchParams& bp, const Plan* plans, uint8_t* const* ws_base, const sgm_item* items, int n,
                BatchLaunch& B) {
    // work items: every direction's slices of every pair, S per wavefront,
    // in quads (kQuad items, one workgroup each)
    std::vector<WorkItem>& work = B.work;
    std::vector<std::array<WorkItem, kQuad>> quads;
    std::vector<WorkItem> singles;  // items without an opposite partner
    size_t census_blocks = 0, cost_blocks = 0, wta_blocks = 0, post_blocks = 0;
    std::vector<BatchItem>& desc = B.desc;
    desc.assign(n, BatchItem{});
    work.clear();
    const bool generic = !(bp.cw == 9 && bp.ch == 7);
    size_t cost_smem = 0, wta_smem = 0, post_smem = 0;
    bool any_adapt = false;
    for (int i = 0; i < n; ++i) {
        const Plan& p = plans[i];
        const Workspace ws = workspace_carve(p, ws_base[i]);
        int gh, gv;
        default_lanes(p, &gh, &gv);
        // the batch kernel has 32- and 16-lane groups; the runner's tuning,
        // when set, applies to every pair
        gh = bp.lanes_h ? bp.lanes_h : (gh == 32 ? 32 : 16);
        gv = bp.lanes_v ? bp.lanes_v : 16;
        BatchItem& d = desc[i];
        d.left = items[i].left;
        d.right = items[i].right;
        d.out = items[i].out;
        d.census_l = ws.census_l;
        d.census_r = ws.census_r;
        d.cost = ws.cost;
        d.cost_r = ws.cost_r;
        d.lbuf = ws.lbuf;
        d.dl = ws.dl;
        d.dr = ws.dr;
        d.W = p.W;
        d.H = p.H;
        d.D = p.D;
        d.Dp = p.Dp;
        d.P = p.n_paths;
        d.cmax = p.cmax;
        d.l16 = p.l16 ? 1 : 0;
        d.median = p.median ? 1 : 0;
        d.lrcheck = p.lrcheck ? 1 : 0;
        d.thr = p.lr_thr;
        d.csct = p.csct ? 1 : 0;
        d.gh = gh;
        d.gv = gv;
        d.subpixel = p.subpixel ? 1 : 0;
        d.lr_full = p.lr_full ? 1 : 0;
        d.adaptive = p.adaptive ? 1 : 0;
        any_adapt = any_adapt || p.adaptive;
        const int nsgm = p.lr_full ? 2 : 1;
        d.census_blk0 = (int)census_blocks;
        census_blocks += generic ? (size_t)2 * ((p.W + 15) / 16) * ((p.H + 15) / 16)
                                 : (size_t)2 * ((p.W + kCenTX - 1) / kCenTX) * ((p.H + kCenTY - 1) / kCenTY);
        d.cost_blk0 = (int)cost_blocks;
        cost_blocks += (size_t)nsgm * ((p.W + kCostTX - 1) / kCostTX) * p.H;
        d.wta_blk0 = (int)wta_blocks;
        wta_blocks += (size_t)nsgm * p.H;
        d.post_blk0 = (int)post_blocks;
        if (p.median || p.lrcheck) post_blocks += p.H;
        const int nright = kCostTX + p.D - 1;
        cost_smem = std::max(cost_smem, 8 * (size_t)((kCostTX + nright + 1) & ~1) + (size_t)kCostTX * (p.Dp + 16));
        if (p.lrcheck) {
            wta_smem = std::max(wta_smem, 4 * (size_t)(p.W + kWtaGuard));
            post_smem = std::max(post_smem, 2 * (size_t)p.W);
        }
        for (int sg = 0; sg < nsgm; ++sg)
            for (int r = 0; r < p.n_paths; ++r) {
                const Dir dir = direction(p.n_paths, r);
                const int S = 64 / (dir.ry == 0 ? gh : gv);
                const int nsl = slice_count(p.W, p.H, dir), steps = slice_steps(p.W, p.H, dir);
                auto unit = [&](int rr, const Dir& dd, int f) {
                    return WorkItem{i, sg * p.n_paths + rr, dd.rx, dd.ry, f, steps, sg};
                };
                // Quads of directions ra and rb (opposite, equal slice counts
                // and lengths): rb's groups in the order of key_b (the first
                // slice of ra over the same pixels) meet ra's groups in
                // order, two and two; an odd count leaves one of each
                auto pair_up = [&](int ra, int rb, auto key_b) {
                    const Dir da = direction(p.n_paths, ra), db = direction(p.n_paths, rb);
                    std::vector<int> fb;
                    for (int f = 0; f < nsl; f += S) fb.push_back(f);
                    std::stable_sort(fb.begin(), fb.end(), [&](int u, int v) { return key_b(u) < key_b(v); });
                    size_t g = 0;
                    for (; g + 1 < fb.size(); g += 2)
                        quads.push_back({unit(ra, da, (int)g * S), unit(ra, da, (int)(g + 1) * S), unit(rb, db, fb[g]),
                                         unit(rb, db, fb[g + 1])});
                    if (g < fb.size()) {
                        singles.push_back(unit(ra, da, (int)g * S));
                        singles.push_back(unit(rb, db, fb[g]));
                    }
                };
                // with 4 or 8 paths, directions 0/1 (+-x) and 2/3 (+-y) are
                // opposite pairs over the same slices
                if (p.n_paths >= 4 && r < 4) {
                    if ((r & 1) == 0) pair_up(r, r + 1, [](int f) { return f; });
                    continue;
                }
                // with 8 paths, 4 (1, 1) / 7 (-1, -1) and 5 (-1, 1) / 6 (1, -1)
                // are opposite diagonals.  Under the wrap schedule the slice
                // from column c of the top row covers x = c +- y (mod W);
                // the opposite one from column c' of the bottom row covers
                // x = c' -+ (H - 1 - y), the same pixels when c' = c +- (H - 1)
                if (p.n_paths == 8) {
                    const int W = p.W, k = (p.H - 1) % p.W;
                    if (r == 4) pair_up(4, 7, [=](int f) { return (f - k + W) % W; });
                    if (r == 5) pair_up(5, 6, [=](int f) { return (f + k) % W; });
                    continue;
                }
                for (int f = 0; f < nsl; f += S) singles.push_back(unit(r, dir, f));
            }
    }
    // the unpaired items, longest first, fill quads of their own
    std::stable_sort(singles.begin(), singles.end(),
                     [](const WorkItem& a, const WorkItem& c) { return a.steps > c.steps; });
    for (size_t k = 0; k < singles.size(); k += kQuad) {
        std::array<WorkItem, kQuad> qd;
        for (int j = 0; j < kQuad; ++j)
            qd[j] = k + j < singles.size() ? singles[k + j] : WorkItem{-1, 0, 0, 0, 0, 0, 0};
        quads.push_back(qd);
    }
    if (census_blocks > 0x7FFFFFFF || cost_blocks > 0x7FFFFFFF || quads.size() > 0x1FFFFFFF)
        return berr(SGM_EINVAL, "batch too large");
    // longest slices first (largest-processing-time-first order); a quad's
    // first item is one of its longest
    std::stable_sort(quads.begin(), quads.end(),
                     [](const std::array<WorkItem, kQuad>& a, const std::array<WorkItem, kQuad>& c) {
                         return a[0].steps > c[0].steps;
                     });
    work.clear();
    for (const auto& qd : quads) work.insert(work.end(), qd.begin(), qd.end());

    // persistent grid: at most two wavefronts per SIMD (256 CUs x 4 SIMDs)
    B.blocks = std::min((int)quads.size(), bp.max_workgroups > 0 ? std::min(bp.max_workgroups, 512) : 512);
    // the planes and cost volumes of the whole batch against the memory-side
    // cache: the store policy of the single-pair path (Plan::nt_store)
    long long fbytes = 0;
    for (const BatchItem& d : desc)
        fbytes += (long long)d.W * d.H * d.Dp * (d.P * (d.l16 ? 2 : 1) + 1) * (d.lr_full ? 2 : 1);
    B.nt = fbytes > kMallBytes;
    B.generic = generic;
    B.any_adapt = any_adapt;
    B.census_blocks = census_blocks;
    B.cost_blocks = cost_blocks;
    B.wta_blocks = wta_blocks;
    B.post_blocks = post_blocks;
    B.cost_smem = cost_smem;
    B.wta_smem = wta_smem;
    B.post_smem = post_smem;
    return SGM_OK;
}

hipError_t batch_launch(const BatchParams& bp, const BatchLaunch& B, const BatchItem* d_items, const WorkItem* d_work,
                        unsigned* counter, hipStream_t s) {
    const int n = (int)B.desc.size();
    hipLaunchKernelGGL(census_batch_kernel, dim3((unsigned)B.census_blocks), dim3(256), 0, s, d_items, n,
                       B.generic ? 1 : 0, (bp.cw - 1) / 2, (bp.ch - 1) / 2, counter);
    hipLaunchKernelGGL(cost_batch_kernel, dim3((unsigned)B.cost_blocks), dim3(kCostThreads), B.cost_smem, s, d_items,
                       n);
    const int nquads = (int)(B.work.size() / kQuad);
    auto agg = B.nt ? (B.any_adapt ? aggregate_batch_kernel<true, true> : aggregate_batch_kernel<true, false>)
                    : (B.any_adapt ? aggregate_batch_kernel<false, true> : aggregate_batch_kernel<false, false>);
    hipLaunchKernelGGL(agg, dim3((unsigned)B.blocks), dim3(256), 0, s, d_items, d_work, nquads, counter, bp.P1,
                       bp.P2);
    hipLaunchKernelGGL(B.nt ? wta_batch_kernel<true> : wta_batch_kernel<false>, dim3((unsigned)B.wta_blocks),
                       dim3(1024), B.wta_smem, s, d_items, n);
    if (B.post_blocks > 0) {
        // pairs without a post stage own empty block ranges; the search for
        // the last pair whose range starts at or before a block skips them
        hipLaunchKernelGGL(post_batch_kernel, dim3((unsigned)B.post_blocks), dim3(256), B.post_smem, s, d_items, n);
    }
    return hipGetLastError();
}

int batch_enqueue(const BatchParams& bp, const Plan* plans, uint8_t* const* ws_base, const sgm_item* items, int n,
                  BatchStaging* st, hipStream_t s) {
    if (n <= 0) return SGM_OK;
    BatchLaunch B;
    if (int rc = batch_build(bp, plans, ws_base, items, n, B)) return rc;
    if (int rc = grow_staging(st, B.desc.size(), B.work.size())) return rc;
    memcpy(st->h_items, B.desc.data(), B.desc.size() * sizeof(BatchItem));
    memcpy(st->h_work, B.work.data(), B.work.size() * sizeof(WorkItem));
    hipError_t e =
        hipMemcpyAsync(st->d_items, st->h_items, B.desc.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(st->d_work, st->h_work, B.work.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(st->staged, s);
    if (e != hipSuccess) return bhip(e, "descriptor copy");
    st->staged_pending = true;
    e = batch_launch(bp, B, st->d_items, st->d_work, st->counter, s);
    if (e != hipSuccess) return bhip(e, "batch kernel launch");
    return SGM_OK;
}

}  // namespace sgm

// A batch's launch sequence captured in a graph (sgm_batch_set_graph): the
// kernels read descriptor and work tables and a queue counter that belong to
// the graph.  The work table depends only on the items' shapes and options
// (the signature); the descriptors also hold the caller's and the arena's
// pointers, so they are copied again, ahead of the replay on the same stream,
// whenever they differ from the last copy.
struct BatchGraph {
    std::vector<long long> sig;
    sgm::BatchItem* d_items = nullptr;
    sgm::WorkItem* d_work = nullptr;
    unsigned* counter = nullptr;
    sgm::BatchItem* h_items = nullptr;  // pinned source of the descriptor copies
    hipEvent_t copied = nullptr;        // the last copy out of h_items
    bool copy_pending = false;
    std::vector<sgm::BatchItem> last;   // descriptors in d_items
    hipGraphExec_t exec = nullptr;
};

static void graph_free(BatchGraph* g) {
    if (!g) return;
    if (g->copy_pending) (void)hipEventSynchronize(g->copied);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->d_items) (void)hipFree(g->d_items);
    if (g->d_work) (void)hipFree(g->d_work);
    if (g->counter) (void)hipFree(g->counter);
    if (g->h_items) (void)hipHostFree(g->h_items);
    if (g->copied) (void)hipEventDestroy(g->copied);
    delete g;
}

struct sgm_batch {
    sgm::BatchParams bp;
    int device = 0;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    sgm::BatchStaging* st = nullptr;
    bool use_graph = false;
    std::vector<BatchGraph*> graphs;  // most recently used first
    hipStream_t capture_stream = nullptr;
};

static constexpr size_t kMaxBatchGraphs = 8;

static void drop_batch_graphs(sgm_batch* b) {
    for (BatchGraph* g : b->graphs) graph_free(g);
    b->graphs.clear();
}

namespace {

int api_err(int code, const std::string& m) {
    sgm::set_last_error(m);
    return code;
}

int api_hip(hipError_t e, const char* what) {
    return api_err(SGM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// What a captured graph depends on besides pointers: the runner's kernel
// shape and every item's size, range, path count and options.
std::vector<long long> batch_signature(const sgm::BatchParams& bp, const sgm_item* items, int n) {
    std::vector<long long> sig{n, bp.lanes_h, bp.lanes_v, bp.max_workgroups};
    sig.reserve(4 + 5 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const sgm_item& it = items[i];
        sig.insert(sig.end(), {it.w, it.h, it.max_disp, it.n_paths, (long long)it.flags});
    }
    return sig;
}

// Builds a graph entry for this batch: its tables, the work table's copy
// (on `s`, so that it precedes the first replay) and the captured launches.
int graph_create(sgm_batch* b, const sgm::BatchLaunch& B, std::vector<long long> sig, hipStream_t s,
                 BatchGraph** out) {
    using namespace sgm;
    BatchGraph* g = new (std::nothrow) BatchGraph;
    if (!g) return api_err(SGM_ENOMEM, "host allocation failed");
    g->sig = std::move(sig);
    const size_t nd = B.desc.size(), nw = B.work.size();
    if (sgm::dev_malloc((void**)&g->d_items, nd * sizeof(BatchItem)) != hipSuccess ||
        sgm::dev_malloc((void**)&g->d_work, nw * sizeof(WorkItem)) != hipSuccess ||
        sgm::dev_malloc((void**)&g->counter, 256) != hipSuccess ||
        sgm::pinned_malloc((void**)&g->h_items, std::max(nd * sizeof(BatchItem), nw * sizeof(WorkItem))) !=
            hipSuccess ||
        hipEventCreateWithFlags(&g->copied, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        graph_free(g);
        return api_err(SGM_ENOMEM, "batch graph allocation failed");
    }
    // the work table once, through the pinned buffer, waiting for the copy
    // before the buffer holds descriptors
    memcpy(g->h_items, B.work.data(), nw * sizeof(WorkItem));
    hipError_t e = hipMemcpyAsync(g->d_work, g->h_items, nw * sizeof(WorkItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && !b->capture_stream) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        graph_free(g);
        return api_hip(e, "batch graph set-up");
    }
    e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        graph_free(g);
        return api_hip(e, "hipStreamBeginCapture");
    }
    hipError_t le = batch_launch(b->bp, B, g->d_items, g->d_work, g->counter, b->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &graph);
    if (le == hipSuccess && e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (le != hipSuccess || e != hipSuccess) {
        graph_free(g);
        return api_hip(le != hipSuccess ? le : e, "batch graph capture");
    }
    *out = g;
    sgm::log_event("batch graph captured: " + std::to_string(nd) + " items, " + std::to_string(nw) + " work items");
    return SGM_OK;
}

// sgm_batch_compute with graphs on: finds (or captures) the graph of this
// batch's signature, copies the descriptors if they changed, replays it.
int batch_replay(sgm_batch* b, const sgm::BatchLayout& L, uint8_t* const* bases, const sgm_item* items, int n,
                 hipStream_t s) {
    using namespace sgm;
    BatchLaunch B;
    if (int rc = batch_build(b->bp, L.plans.data(), bases, items, n, B)) return rc;
    std::vector<long long> sig = batch_signature(b->bp, items, n);
    size_t i = 0;
    while (i < b->graphs.size() && b->graphs[i]->sig != sig) ++i;
    if (i == b->graphs.size()) {
        BatchGraph* g = nullptr;
        if (int rc = graph_create(b, B, std::move(sig), s, &g)) return rc;
        if (b->graphs.size() == kMaxBatchGraphs) {
            // its last replay and copy were enqueued on a stream the caller
            // may still run: wait for the device before freeing its tables
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) {
                graph_free(g);
                return api_hip(e, "hipDeviceSynchronize");
            }
            graph_free(b->graphs.back());
            b->graphs.pop_back();
        }
        b->graphs.insert(b->graphs.begin(), g);
    } else if (i > 0) {  // to the front, keeping the others in order
        std::rotate(b->graphs.begin(), b->graphs.begin() + i, b->graphs.begin() + i + 1);
    }
    BatchGraph* g = b->graphs[0];
    const size_t bytes = B.desc.size() * sizeof(BatchItem);
    if (g->last.size() != B.desc.size() || memcmp(g->last.data(), B.desc.data(), bytes) != 0) {
        if (g->copy_pending) {
            hipError_t e = hipEventSynchronize(g->copied);
            if (e != hipSuccess) return api_hip(e, "hipEventSynchronize");
            g->copy_pending = false;
        }
        memcpy(g->h_items, B.desc.data(), bytes);
        hipError_t e = hipMemcpyAsync(g->d_items, g->h_items, bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(g->copied, s);
        if (e != hipSuccess) return api_hip(e, "descriptor copy");
        g->copy_pending = true;
        g->last = B.desc;
    }
    hipError_t e = hipGraphLaunch(g->exec, s);
    if (e != hipSuccess) return api_hip(e, "hipGraphLaunch");
    return SGM_OK;
}

}  // namespace

extern "C" {

sgm_batch* sgm_batch_create(int P1, int P2, int census_w, int census_h) {
    sgm::Plan probe;  // validate the batch-wide parameters on a 1x1 pair
    probe.W = probe.H = probe.D = 1;
    probe.P1 = P1;
    probe.P2 = P2;
    probe.n_paths = 2;
    probe.cw = census_w;
    probe.ch = census_h;
    const char* why = "invalid parameters";
    if (!sgm::plan_finish(probe, &why)) {
        api_err(SGM_EINVAL, why);
        return nullptr;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        api_hip(e, "hipGetDevice");
        return nullptr;
    }
    sgm_batch* b = new (std::nothrow) sgm_batch;
    if (!b) {
        api_err(SGM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    b->bp = sgm::BatchParams{P1, P2, census_w, census_h, false};
    b->device = dev;
    b->st = sgm::staging_create();
    if (!b->st) {
        api_err(SGM_ENOMEM, "batch staging allocation failed");
        delete b;
        return nullptr;
    }
    return b;
}

int sgm_batch_set_tuning(sgm_batch* b, int lanes_h, int lanes_v) {
    if (!b) return api_err(SGM_EINVAL, "null batch");
    auto ok = [](int g) { return g == 0 || g == 16 || g == 32; };
    if (!ok(lanes_h) || !ok(lanes_v)) return api_err(SGM_EINVAL, "batch lanes must be 0, 16 or 32");
    b->bp.lanes_h = lanes_h;
    b->bp.lanes_v = lanes_v;
    return SGM_OK;
}

int sgm_batch_set_grid(sgm_batch* b, int max_workgroups) {
    if (!b) return api_err(SGM_EINVAL, "null batch");
    if (max_workgroups < 0) return api_err(SGM_EINVAL, "max_workgroups must be >= 0");
    b->bp.max_workgroups = max_workgroups;
    return SGM_OK;
}

int sgm_batch_set_graph(sgm_batch* b, int enable) {
    if (!b) return api_err(SGM_EINVAL, "null batch");
    if (enable != 0 && enable != 1) return api_err(SGM_EINVAL, "enable must be 0 or 1");
    b->use_graph = enable != 0;
    if (!b->use_graph) {
        hipError_t e = hipDeviceSynchronize();  // replays may still read the graphs' tables
        if (e != hipSuccess) return api_hip(e, "hipDeviceSynchronize");
        drop_batch_graphs(b);
    }
    return SGM_OK;
}

size_t sgm_batch_footprint(sgm_batch* b, const sgm_item* items, int n) {
    if (!b) return 0;
    sgm::BatchLayout L;
    const char* why = "";
    if (!sgm::batch_plan(b->bp, items, n, L, &why)) return 0;
    return L.total;
}

int sgm_batch_compute(sgm_batch* b, const sgm_item* items, int n, sgm_stream_t stream) {
    using namespace sgm;
    if (!b) return api_err(SGM_EINVAL, "null batch");
    if (n == 0) return SGM_OK;
    BatchLayout L;
    const char* why = "invalid item";
    if (!batch_plan(b->bp, items, n, L, &why)) return api_err(SGM_EINVAL, why);
    for (int i = 0; i < n; ++i) {
        if (!items[i].left || !items[i].right || !items[i].out) return api_err(SGM_EINVAL, "null buffer pointer");
        if ((const void*)items[i].out == (const void*)items[i].left ||
            (const void*)items[i].out == (const void*)items[i].right)
            return api_err(SGM_EINVAL, "output aliases an input");
    }
    hipStream_t s = (hipStream_t)stream;

    // workspace: grows (after the device is idle) to the largest batch seen
    if (L.total > b->arena_bytes) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return api_hip(e, "hipDeviceSynchronize");
        if (b->arena) (void)hipFree(b->arena);
        b->arena = nullptr;
        b->arena_bytes = 0;
        e = sgm::dev_malloc(&b->arena, L.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return api_err(SGM_ENOMEM, std::string("batch workspace allocation failed: ") + hipGetErrorString(e));
        }
        b->arena_bytes = L.total;
        sgm::log_event("batch workspace grown to " + std::to_string(L.total) + " bytes");
    }
    std::vector<uint8_t*> bases(n);
    for (int i = 0; i < n; ++i) bases[i] = static_cast<uint8_t*>(b->arena) + L.offsets[i];
    if (!b->use_graph) return batch_enqueue(b->bp, L.plans.data(), bases.data(), items, n, b->st, s);
    return batch_replay(b, L, bases.data(), items, n, s);
}

void sgm_batch_destroy(sgm_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    drop_batch_graphs(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->arena) (void)hipFree(b->arena);
    sgm::staging_destroy(b->st);
    delete b;
}

int sgm_compute_batch(const sgm_item* items, int n, int P1, int P2, int census_w, int census_h,
                      sgm_stream_t stream) {
    sgm_batch* b = sgm_batch_create(P1, P2, census_w, census_h);
    if (!b) return SGM_EINVAL;
    int rc = sgm_batch_compute(b, items, n, stream);
    if (rc == SGM_OK) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) rc = api_hip(e, "hipStreamSynchronize");
    }
    sgm_batch_destroy(b);
    return rc;
}

}  // extern "C"

// Single-pair SGM kernels for gfx950 and their host-side launchers.  The
// stage bodies live in sgm_device.h; each kernel here maps its grid onto one
// stereo pair.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "sgm_device.h"
#include "sgm_plan.h"

namespace sgm {

namespace {

using namespace dev;

__global__ __launch_bounds__(256) void census97_kernel(CensusArgs a) { census97_block(a, blockIdx.x, blockIdx.y, blockIdx.z); }

__global__ __launch_bounds__(256) void census_generic_kernel(CensusArgs a, int rx, int ry) {
    census_generic_block(a, rx, ry, blockIdx.x, blockIdx.y, blockIdx.z);
}

__global__ __launch_bounds__(256) void census_cost_kernel(CensusCostArgs a) {
    extern __shared__ __align__(16) uint8_t cc_smem[];
    census_cost_block(a, blockIdx.x, blockIdx.y, cc_smem);
}

template <bool RB, int DP>
__global__ __launch_bounds__(kCostThreads) void cost_kernel(CostArgs a) {
    extern __shared__ __align__(16) uint64_t cost_smem[];
    cost_block<RB, DP>(a, blockIdx.x, blockIdx.y, cost_smem);
}

// Direction table of one pair's aggregation launch: the directions of one
// SGM, or of two (left-base and right-base, for the full left-right check).
constexpr int kMaxLaunchDirs = 2 * kMaxDirs;
struct AggArgs {
    SliceArgs base;          // shared fields; rx, ry, cost, lplane set per direction
    void* lbuf;              // all L_r planes
    int ndirs, total;
    int start[kMaxLaunchDirs + 1];  // first wave of each direction
    int rx[kMaxLaunchDirs], ry[kMaxLaunchDirs], plane_index[kMaxLaunchDirs];
    const uint8_t* cost[kMaxLaunchDirs];  // the cost volume each direction reads
    const uint8_t* img[kMaxLaunchDirs];   // its SGM's base image (adaptive P2)
    // paired[k]: directions k and k + 1 are opposite, axis-aligned and have
    // the same wave count; their waves interleave (see aggregate_kernel)
    int paired[kMaxLaunchDirs];
};

// One launch covers every direction.  Horizontal slices (the longest when
// W > H) may use a different group width GH than the others (GV), so that
// the longest dependency chains get the fewest instructions per step.
template <int GH, int GV, int Dp, typename LT, bool FUSED, bool ADAPT, bool NT>
__global__ __launch_bounds__(256) void aggregate_kernel(AggArgs a) {
    __shared__ uint16_t p2lut[ADAPT ? 256 : 1];
    if constexpr (ADAPT) {  // every wave of the block takes part before any leaves
        fill_p2_lut(p2lut, a.base.P1, a.base.P2);
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (wave >= a.total) return;
    int r = 0;
    while (r + 1 < a.ndirs && wave >= a.start[r + 1]) ++r;
    int local = wave - a.start[r];
    // The 2n waves of a pair of opposite directions over the same n slice
    // groups interleave two by two (A, A, B, B per workgroup), so both
    // directions' waves over the same slices share a CU and its L2: the
    // second read of a slice's costs can hit where the two walks pass close
    // in time.  A bijection between the pair's waves and (direction, slice
    // group); an odd n ends with one wave of each.
    const int r0 = (r > 0 && a.paired[r - 1]) ? r - 1 : r;
    if (a.paired[r0]) {
        const int n = a.start[r0 + 1] - a.start[r0];
        const int j = wave - a.start[r0];
        const int g = j >> 2, w4 = j & 3;
        if (4 * g + 4 <= 2 * n) {
            r = r0 + (w4 >> 1);
            local = 2 * g + (w4 & 1);
        } else {
            r = r0 + (w4 & 1);
            local = 2 * g;
        }
    }
    SliceArgs s = a.base;
    s.rx = a.rx[r];
    s.ry = a.ry[r];
    s.cost = a.cost[r];
    s.img = a.img[r];
    s.p2lut = ADAPT ? p2lut : nullptr;
    s.lplane = reinterpret_cast<LT*>(a.lbuf) + (size_t)s.plane * a.plane_index[r];
    if (s.ry == 0) {
        aggregate_wave<GH, Dp / GH, LT, kHoriz, FUSED, ADAPT, NT>(s, local * (64 / GH), lane);
    } else if (s.rx == 0) {
        aggregate_wave<GV, Dp / GV, LT, kVert, FUSED, ADAPT, NT>(s, local * (64 / GV), lane);
    } else {
        aggregate_wave<GV, Dp / GV, LT, kDiag, FUSED, ADAPT, NT>(s, local * (64 / GV), lane);
    }
}

template <typename LT, bool NT, bool FOLD>
__global__ __launch_bounds__(1024) void wta_kernel(WtaArgs a) {
    extern __shared__ uint32_t wta_smem[];
    wta_row<LT, NT, FOLD>(a, blockIdx.x, wta_smem);
}

// Winner-take-all of two SGMs in one launch (full left-right check): rows
// 0 .. H-1 of the left-base sums give D_L, blocks H .. 2H-1 the rows of the
// right-base sums, D_R.
template <typename LT, bool NT, bool FOLD>
__global__ __launch_bounds__(1024) void wta_pair_kernel(WtaArgs l, WtaArgs r) {
    extern __shared__ uint32_t wta_smem[];
    const int y = blockIdx.x;
    if (y < l.H)
        wta_row<LT, NT, FOLD>(l, y, wta_smem);
    else
        wta_row<LT, NT, FOLD>(r, y - l.H, wta_smem);
}

// The final pass (see final_pass_block): NPL = n_paths - 1 stored planes;
// NT: non-temporal plane loads.
template <int Dp, int NPL, bool NT>
__global__ __launch_bounds__(kFinalThreads) void final_pass_kernel(FinalArgs f) {
    extern __shared__ __align__(16) uint8_t fp_smem[];
    final_pass_block<Dp, NPL, NT>(f, blockIdx.x, fp_smem);
}

__global__ __launch_bounds__(256) void post_kernel(PostArgs a) {
    extern __shared__ uint16_t post_smem[];
    post_row(a, blockIdx.x, post_smem);
}

// Debug tap: S = sum of planes, u16 [H][W][D].
// Plane `skip` (-1: none) is left out.
template <typename LT>
__global__ void sum_planes_kernel(const void* lbuf, size_t plane, uint16_t* s, int W, int H, int D,
                                  int Dp, int nplanes, int skip) {
    const size_t n = (size_t)W * H * D;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / D, d = i - p * D;
        uint32_t acc = 0;
        for (int k = 0; k < nplanes; ++k)
            if (k != skip) acc += reinterpret_cast<const LT*>(lbuf)[plane * k + p * Dp + d];
        s[i] = (uint16_t)acc;
    }
}

// Debug tap: one L_r plane (or the cost volume) as u16 [H][W][D].
template <typename LT>
__global__ void extract_plane_kernel(const LT* src, uint16_t* out, int W, int H, int D, int Dp) {
    const size_t n = (size_t)W * H * D;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / D, d = i - p * D;
        out[i] = (uint16_t)src[p * Dp + d];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
bool plan_finish(Plan& p, const char** why) {
    auto fail = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (p.W < 1 || p.H < 1) return fail("width and height must be >= 1");
    if (p.W > kMaxWidth) return fail("width must be <= 16000");
    if (p.D < 1 || p.D > kMaxDisp) return fail("max_disp must be in [1, 256]");
    if (!(p.n_paths == 2 || p.n_paths == 4 || p.n_paths == 8)) return fail("n_paths must be 2, 4 or 8");
    if (p.cw < 1 || p.ch < 1 || !(p.cw & 1) || !(p.ch & 1)) return fail("census window sides must be odd and >= 1");
    if (p.cw > 31 || p.ch > 15) return fail("census window must be at most 31 wide and 15 tall");
    if (!p.csct && p.cw * p.ch > 64) return fail("full census window must have <= 64 pixels");
    if (p.csct && (p.cw * p.ch - 1) / 2 > 64) return fail("CSCT window must have <= 64 pairs");
    if (p.P1 < 0 || p.P2 < 0) return fail("P1 and P2 must be >= 0");
    if (p.P1 > 65535) return fail("P1 must be <= 65535");
    p.cmax = p.csct ? (p.cw * p.ch - 1) / 2 : p.cw * p.ch - 1;
    // the largest penalty of one step bounds L_r <= Cmax + penalty: P2, or
    // with adaptive P2 (max(P1, P2 / (1 + g)) per step) the larger of P1, P2
    const long long pmax = p.adaptive ? std::max(p.P1, p.P2) : p.P2;
    if ((long long)p.n_paths * (p.cmax + pmax) > 65535)
        return fail(p.adaptive ? "n_paths * (Cmax + max(P1, P2)) must be <= 65535 (16-bit summed costs, adaptive P2)"
                               : "n_paths * (Cmax + P2) must be <= 65535 (16-bit summed costs)");
    if (p.lr_thr < 0) return fail("lr threshold must be >= 0");
    p.Dp = padded_disp(p.D);
    p.l16 = p.cmax + pmax > 255;
    // Normal stores leave a frame's L_r planes in the 256 MiB memory-side
    // cache for the WTA to read back.  When the planes and the cost volume
    // do not fit, the dirty planes would be written back while the WTA reads,
    // so they are stored non-temporally instead.
    {
        const long long cells = (long long)p.W * p.H * p.Dp;
        const long long nsgm = p.lr_full ? 2 : 1;
        const long long bytes = nsgm * cells * (p.n_paths * (p.l16 ? 2 : 1) + 1);
        p.nt_store = bytes > kMallBytes;
    }
    // one L_r plane (u16) must stay below 2 GiB: kernels address planes with
    // 32-bit byte offsets
    if ((long long)p.W * p.H * p.Dp > (1LL << 30)) return fail("width * height * padded disparities must be <= 2^30");
    return true;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t workspace_bytes(const Plan& p) {
    const size_t npx = (size_t)p.W * p.H;
    const size_t cells = npx * p.Dp;
    const int nsgm = p.lr_full ? 2 : 1;
    return align256(cells) + align256(cells * nsgm * p.n_paths * (p.l16 ? 2 : 1)) + 2 * align256(npx * 2) +
           2 * align256(8 * (npx + kCensusGuard)) + align256(4 * (size_t)p.H) + (p.lr_full ? align256(cells) : 0);
}

Workspace workspace_carve(const Plan& p, void* base) {
    const size_t npx = (size_t)p.W * p.H;
    const size_t cells = npx * p.Dp;
    uint8_t* b = static_cast<uint8_t*>(base);
    Workspace ws;
    ws.cost = b;
    b += align256(cells);
    ws.lbuf = b;
    b += align256(cells * (p.lr_full ? 2 : 1) * p.n_paths * (p.l16 ? 2 : 1));
    ws.dl = reinterpret_cast<uint16_t*>(b);
    b += align256(npx * 2);
    ws.dr = reinterpret_cast<uint16_t*>(b);
    b += align256(npx * 2);
    ws.census_l = reinterpret_cast<uint64_t*>(b) + kCensusGuard;
    b += align256(8 * (npx + kCensusGuard));
    ws.census_r = reinterpret_cast<uint64_t*>(b) + kCensusGuard;
    b += align256(8 * (npx + kCensusGuard));
    ws.rowcnt = reinterpret_cast<int*>(b);
    b += align256(4 * (size_t)p.H);
    if (p.lr_full) ws.cost_r = b;
    return ws;
}

static hipError_t launch_census_pair(const Plan& p, const uint8_t* left, const uint8_t* right, uint64_t* cl,
                                     uint64_t* cr, int nimg, hipStream_t stream, int* zero = nullptr) {
    CensusArgs a{{left, right}, {cl, cr}, p.W, p.H, p.csct ? 1 : 0, zero, zero ? p.H : 0};
    if (p.cw == 9 && p.ch == 7) {
        dim3 grid((p.W + kCenTX - 1) / kCenTX, (p.H + kCenTY - 1) / kCenTY, nimg);
        hipLaunchKernelGGL(census97_kernel, grid, dim3(256), 0, stream, a);
    } else {
        dim3 grid((p.W + 15) / 16, (p.H + 15) / 16, nimg);
        hipLaunchKernelGGL(census_generic_kernel, grid, dim3(256), 0, stream, a, (p.cw - 1) / 2, (p.ch - 1) / 2);
    }
    return hipGetLastError();
}

hipError_t launch_census(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right,
                         hipStream_t stream) {
    return launch_census_pair(p, left, right, ws.census_l, ws.census_r, 2, stream, ws.rowcnt);
}

bool census_cost_fusable(const Plan& p) { return p.cc_fused && p.cw == 9 && p.ch == 7; }

hipError_t launch_matching_cost(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right,
                                bool need_cost, hipStream_t stream) {
    if (p.lr_full) {  // census words, then both cost volumes
        hipError_t e = launch_census(p, ws, left, right, stream);
        if (e == hipSuccess) e = launch_cost(p, ws, stream, false);
        if (e == hipSuccess) e = launch_cost(p, ws, stream, true);
        return e;
    }
    const bool fusable = census_cost_fusable(p);
    hipError_t e = hipSuccess;
    if (need_cost && fusable) {
        const CcLayout L = cc_layout(p.D, p.Dp);
        CensusCostArgs a{left, right, ws.cost, p.W, p.H, p.D, p.Dp, p.cmax, p.csct ? 1 : 0, ws.rowcnt, p.H};
        hipLaunchKernelGGL(census_cost_kernel, dim3((p.W + kCcTX - 1) / kCcTX, p.H), dim3(256), L.bytes, stream, a);
        e = hipGetLastError();
    }
    // census words in global memory: for the fused aggregation, and for the
    // cost kernel of windows other than 9x7
    if (e == hipSuccess && (fused_aggregation(p) || (need_cost && !fusable)))
        e = launch_census(p, ws, left, right, stream);
    if (e == hipSuccess && need_cost && !fusable) e = launch_cost(p, ws, stream);
    return e;
}

hipError_t launch_cost(const Plan& p, const Workspace& ws, hipStream_t stream, bool right_base) {
    const int nright = kCostTX + p.D - 1;
    const size_t smem = 8 * (size_t)((kCostTX + nright + 1) & ~1) + (size_t)kCostTX * (p.Dp + 16);
    dim3 grid((p.W + kCostTX - 1) / kCostTX, p.H);
    if (right_base && !ws.cost_r) return hipErrorInvalidValue;
    const CostArgs a = right_base ? CostArgs{ws.census_r, ws.census_l, ws.cost_r, p.W, p.H, p.D, p.Dp, p.cmax}
                                  : CostArgs{ws.census_l, ws.census_r, ws.cost, p.W, p.H, p.D, p.Dp, p.cmax};
    auto k = right_base ? (p.Dp == 64 ? cost_kernel<true, 64> : p.Dp == 128 ? cost_kernel<true, 128> : cost_kernel<true, 256>)
                        : (p.Dp == 64 ? cost_kernel<false, 64> : p.Dp == 128 ? cost_kernel<false, 128> : cost_kernel<false, 256>);
    hipLaunchKernelGGL(k, grid, dim3(kCostThreads), smem, stream, a);
    return hipGetLastError();
}

static void fill_agg_args(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right, int SH,
                          int SV, AggArgs& a, bool skip_last) {
    a.base = SliceArgs{ws.cost, ws.census_l, ws.census_r, nullptr, (uint32_t)((size_t)p.W * p.H * p.Dp),
                       p.W, p.H, p.D, p.P1, p.P2, p.cmax, 0, 0};
    a.lbuf = ws.lbuf;
    // directions of the left-base SGM (planes 0 .. P-1) and, for the full
    // left-right check, of the right-base SGM (planes P .. 2P-1)
    const int nsgm = p.lr_full ? 2 : 1;
    const int all = nsgm * p.n_paths;
    const int last = skip_last ? last_direction(p) : -1;
    a.ndirs = all - (skip_last ? 1 : 0);
    // longest slices first, so that they start first
    int order[kMaxLaunchDirs], n = 0;
    const bool horiz_first = p.W >= p.H;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < all; ++i) {
            if (i == last) continue;
            const bool horiz = direction(p.n_paths, i % p.n_paths).ry == 0;
            if ((horiz == horiz_first) == (pass == 0)) order[n++] = i;
        }
    int acc = 0;
    for (int k = 0; k < a.ndirs; ++k) {
        const Dir d = direction(p.n_paths, order[k] % p.n_paths);
        const int S = d.ry == 0 ? SH : SV;
        a.rx[k] = d.rx;
        a.ry[k] = d.ry;
        // without the last direction the stored planes close up
        a.plane_index[k] = order[k] - (last >= 0 && order[k] > last ? 1 : 0);
        a.cost[k] = order[k] < p.n_paths ? ws.cost : ws.cost_r;
        a.img[k] = order[k] < p.n_paths ? left : right;
        a.start[k] = acc;
        acc += (slice_count(p.W, p.H, d) + S - 1) / S;
    }
    a.start[a.ndirs] = acc;
    a.total = acc;
    for (int k = 0; k < a.ndirs; ++k) {
        a.paired[k] = 0;
        if (k + 1 < a.ndirs && !(k > 0 && a.paired[k - 1]) && a.rx[k] == -a.rx[k + 1] && a.ry[k] == -a.ry[k + 1] &&
            (a.rx[k] == 0 || a.ry[k] == 0) && order[k] / p.n_paths == order[k + 1] / p.n_paths &&
            a.start[k + 1] - a.start[k] == a.start[k + 2] - a.start[k + 1])
            a.paired[k] = 1;
    }
}

// Images of the two SGMs (base left / base right) for the adaptive P2.
struct Images {
    const uint8_t *left, *right;
    bool skip_last;  // leave out the direction the final pass fuses
};

template <int GH, int GV, int Dp, typename LT, bool FUSED, bool ADAPT, bool NT>
static hipError_t launch_agg_t(const Plan& p, const Workspace& ws, Images im, hipStream_t stream) {
    AggArgs a;
    fill_agg_args(p, ws, im.left, im.right, 64 / GH, 64 / GV, a, im.skip_last);
    hipLaunchKernelGGL((aggregate_kernel<GH, GV, Dp, LT, FUSED, ADAPT, NT>), dim3((a.total + 3) / 4), dim3(256), 0,
                       stream, a);
    return hipGetLastError();
}

template <int Dp, typename LT, bool FUSED, bool ADAPT, bool NT>
static hipError_t launch_agg_dp(const Plan& p, const Workspace& ws, Images im, int gh, int gv, hipStream_t stream) {
    switch (gh * 100 + gv) {
        case 1616: return launch_agg_t<16, 16, Dp, LT, FUSED, ADAPT, NT>(p, ws, im, stream);
        case 3216: return launch_agg_t<32, 16, Dp, LT, FUSED, ADAPT, NT>(p, ws, im, stream);
        case 3232: return launch_agg_t<32, 32, Dp, LT, FUSED, ADAPT, NT>(p, ws, im, stream);
        default: break;
    }
    if constexpr (Dp >= 128) {  // 64 lanes need at least 2 levels per lane
        if (gh == 64 && gv == 16) return launch_agg_t<64, 16, Dp, LT, FUSED, ADAPT, NT>(p, ws, im, stream);
        if (gh == 64 && gv == 32) return launch_agg_t<64, 32, Dp, LT, FUSED, ADAPT, NT>(p, ws, im, stream);
    }
    return hipErrorInvalidValue;
}

template <typename LT, bool FUSED, bool ADAPT, bool NT>
static hipError_t launch_agg_lt(const Plan& p, const Workspace& ws, Images im, int gh, int gv, hipStream_t stream) {
    if (p.Dp == 64) {
        // Dp = 64 has only 4 levels per lane at G = 16 and 2 at G = 32
        return launch_agg_dp<64, LT, FUSED, ADAPT, NT>(p, ws, im, gh == 64 ? 32 : gh, gv == 64 ? 32 : gv, stream);
    }
    if (p.Dp == 128) return launch_agg_dp<128, LT, FUSED, ADAPT, NT>(p, ws, im, gh, gv, stream);
    return launch_agg_dp<256, LT, FUSED, ADAPT, NT>(p, ws, im, gh, gv, stream);
}

// Group widths: horizontal slices are the longest chains on wide images,
// so they get more lanes (fewer instructions per step); the rest use 16.
void default_lanes(const Plan& p, int* gh, int* gv) {
    *gh = p.W > p.H ? 32 : 16;
    *gv = 16;
}

bool fused_aggregation(const Plan& p) { return p.fused && !p.lr_full && !p.adaptive; }

hipError_t launch_aggregate(const Plan& p, const Workspace& ws, hipStream_t stream, const uint8_t* left,
                            const uint8_t* right, bool skip_last) {
    int gh = p.lanes_h, gv = p.lanes_v;
    if (gh <= 0 || gv <= 0) default_lanes(p, &gh, &gv);
    const Images im{left, right, skip_last};
    if (p.adaptive) {
        if (!left || (p.lr_full && !right)) return hipErrorInvalidValue;
        return p.l16 ? launch_agg_lt<uint16_t, false, true, false>(p, ws, im, gh, gv, stream)
                     : launch_agg_lt<uint8_t, false, true, false>(p, ws, im, gh, gv, stream);
    }
    if (fused_aggregation(p))
        return p.l16 ? launch_agg_lt<uint16_t, true, false, false>(p, ws, im, gh, gv, stream)
                     : launch_agg_lt<uint8_t, true, false, false>(p, ws, im, gh, gv, stream);
    // the store policy is an instruction operand: a second instantiation of
    // the plain (stored-cost, constant-P2) kernels
    if (p.nt_store)
        return p.l16 ? launch_agg_lt<uint16_t, false, false, true>(p, ws, im, gh, gv, stream)
                     : launch_agg_lt<uint8_t, false, false, true>(p, ws, im, gh, gv, stream);
    return p.l16 ? launch_agg_lt<uint16_t, false, false, false>(p, ws, im, gh, gv, stream)
                 : launch_agg_lt<uint8_t, false, false, false>(p, ws, im, gh, gv, stream);
}

bool final_pass_active(const Plan& p) {
    if (!p.final_pass || p.l16 || p.lr_full || p.adaptive || fused_aggregation(p)) return false;
    return final_smem_bytes(p.Dp, p.W, p.lrcheck) <= 64 * 1024;
}

template <int Dp, int NPL>
static hipError_t launch_final_t(const Plan& p, const FinalArgs& f, hipStream_t stream) {
    using L = FinalLayout<Dp>;
    const size_t smem = final_smem_bytes(Dp, p.W, p.lrcheck);
    auto k = p.nt_store ? final_pass_kernel<Dp, NPL, true> : final_pass_kernel<Dp, NPL, false>;
    hipLaunchKernelGGL(k, dim3((p.H + L::R - 1) / L::R), dim3(kFinalThreads), smem, stream, f);
    return hipGetLastError();
}

template <int Dp>
static hipError_t launch_final_d(const Plan& p, const FinalArgs& f, hipStream_t stream) {
    switch (p.n_paths) {
        case 2: return launch_final_t<Dp, 1>(p, f, stream);
        case 4: return launch_final_t<Dp, 3>(p, f, stream);
        default: return launch_final_t<Dp, 7>(p, f, stream);
    }
}

hipError_t launch_final_pass(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream, uint16_t* s_out) {
    if (!final_pass_active(p)) return hipErrorInvalidValue;
    const Dir d = direction(p.n_paths, last_direction(p));
    const bool post = p.median || p.lrcheck;
    const size_t plane = (size_t)p.W * p.H * p.Dp;
    FinalArgs f;
    f.agg = SliceArgs{ws.cost, ws.census_l, ws.census_r, nullptr, (uint32_t)plane, p.W, p.H, p.D, p.P1, p.P2,
                      p.cmax, d.rx, d.ry};
    f.planes = static_cast<const uint8_t*>(ws.lbuf);
    f.plane = plane;
    f.wta = WtaArgs{nullptr, plane, post ? ws.dl : out, p.lrcheck ? ws.dr : nullptr, p.W, p.H, p.D, p.Dp,
                    p.n_paths - 1, p.subpixel ? 1 : 0};
    f.s_out = s_out;
    if (p.Dp == 64) return launch_final_d<64>(p, f, stream);
    if (p.Dp == 128) return launch_final_d<128>(p, f, stream);
    return launch_final_d<256>(p, f, stream);
}

bool post_folded(const Plan& p) { return p.post_in_wta && (p.median || p.lrcheck) && !final_pass_active(p); }

hipError_t launch_aggregate_wta(const Plan& p, const Workspace& ws, const uint8_t* left, const uint8_t* right,
                                uint16_t* out, hipStream_t stream, hipEvent_t mid_event, bool post_in_wta) {
    const bool fp = final_pass_active(p);
    hipError_t e = launch_aggregate(p, ws, stream, left, right, fp);
    if (e == hipSuccess && mid_event) e = hipEventRecord(mid_event, stream);
    if (e == hipSuccess) e = fp ? launch_final_pass(p, ws, out, stream) : launch_wta(p, ws, out, stream, post_in_wta);
    return e;
}

// Whether the L_r planes were stored non-temporally, so the WTA streams them
// the same way: the plain aggregation kernels follow p.nt_store; the
// adaptive-P2 and census-computing ones always store them normally.
static bool planes_nt(const Plan& p) { return p.nt_store && !p.adaptive && !fused_aggregation(p); }

static PostArgs post_args(const Plan& p, const Workspace& ws, uint16_t* out) {
    return PostArgs{ws.dl, ws.dr, out, p.W, p.H, p.median ? 1 : 0, p.lrcheck ? 1 : 0, p.lr_thr, p.subpixel ? 1 : 0};
}

hipError_t launch_wta(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream, bool post_in_wta) {
    const bool nt = planes_nt(p);
    const bool post = p.median || p.lrcheck;
    const bool fold = post_in_wta && post;
    if (fold && !ws.rowcnt) return hipErrorInvalidValue;
    if (p.lr_full) {
        const size_t plane = (size_t)p.W * p.H * p.Dp;
        const void* rbuf = static_cast<const uint8_t*>(ws.lbuf) + plane * p.n_paths * (p.l16 ? 2 : 1);
        WtaArgs l{ws.lbuf, plane, ws.dl, nullptr, p.W, p.H, p.D, p.Dp, p.n_paths, p.subpixel ? 1 : 0};
        WtaArgs r{rbuf, plane, ws.dr, nullptr, p.W, p.H, p.D, p.Dp, p.n_paths};
        size_t smem = 0;
        if (fold) {  // D_L and D_R rows come from separate blocks
            for (WtaArgs* w : {&l, &r}) {
                w->rowcnt = ws.rowcnt;
                w->contrib = 2;
                w->post = post_args(p, ws, out);
            }
            smem = 2 * (size_t)p.W;  // the post stage's D_R medians
        }
        auto k = fold ? (p.l16 ? (nt ? wta_pair_kernel<uint16_t, true, true> : wta_pair_kernel<uint16_t, false, true>)
                               : (nt ? wta_pair_kernel<uint8_t, true, true> : wta_pair_kernel<uint8_t, false, true>))
                      : (p.l16 ? (nt ? wta_pair_kernel<uint16_t, true, false> : wta_pair_kernel<uint16_t, false, false>)
                               : (nt ? wta_pair_kernel<uint8_t, true, false> : wta_pair_kernel<uint8_t, false, false>));
        hipLaunchKernelGGL(k, dim3(2 * p.H), dim3(1024), smem, stream, l, r);
        return hipGetLastError();
    }
    WtaArgs a{ws.lbuf, (size_t)p.W * p.H * p.Dp, post ? ws.dl : out, p.lrcheck ? ws.dr : nullptr,
              p.W, p.H, p.D, p.Dp, p.n_paths, p.subpixel ? 1 : 0};
    if (fold) {
        a.rowcnt = ws.rowcnt;
        a.post = post_args(p, ws, out);
    }
    // the right-view keys; with the post stage inside, its D_R medians reuse them
    const size_t smem = p.lrcheck ? 4 * (size_t)(p.W + kWtaGuard) : 0;
    // the planes are read the way they were stored: non-temporally when they
    // exceed the memory-side cache and the aggregation stored them so
    auto k = fold ? (p.l16 ? (nt ? wta_kernel<uint16_t, true, true> : wta_kernel<uint16_t, false, true>)
                           : (nt ? wta_kernel<uint8_t, true, true> : wta_kernel<uint8_t, false, true>))
                  : (p.l16 ? (nt ? wta_kernel<uint16_t, true, false> : wta_kernel<uint16_t, false, false>)
                           : (nt ? wta_kernel<uint8_t, true, false> : wta_kernel<uint8_t, false, false>));
    hipLaunchKernelGGL(k, dim3(p.H), dim3(1024), smem, stream, a);
    return hipGetLastError();
}

hipError_t launch_post(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream) {
    if (!p.median && !p.lrcheck) return hipSuccess;  // the WTA wrote `out`
    const PostArgs a = post_args(p, ws, out);
    hipLaunchKernelGGL(post_kernel, dim3(p.H), dim3(256), p.lrcheck ? 2 * (size_t)p.W : 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_pipeline(const Plan& p, const Workspace& ws, const uint8_t* left,
                           const uint8_t* right, uint16_t* out, hipStream_t stream, hipEvent_t* events) {
    hipError_t e = hipSuccess;
    auto mark = [&](int i) {
        if (events && e == hipSuccess) e = hipEventRecord(events[i], stream);
    };
    mark(0);
    if (e == hipSuccess) e = launch_matching_cost(p, ws, left, right, !fused_aggregation(p), stream);
    mark(1);
    const bool fold = post_folded(p);
    if (e == hipSuccess)
        e = launch_aggregate_wta(p, ws, left, right, out, stream, events ? events[2] : nullptr, fold);
    mark(3);
    if (e == hipSuccess && !fold) e = launch_post(p, ws, out, stream);
    mark(4);
    return e;
}

hipError_t launch_census_only(const Plan& p, const uint8_t* img, uint64_t* out, hipStream_t stream) {
    return launch_census_pair(p, img, img, out, out, 1, stream);
}

hipError_t launch_sum_planes(const Plan& p, const Workspace& ws, uint16_t* s_out, hipStream_t stream, int skip,
                             int nplanes) {
    const size_t plane = (size_t)p.W * p.H * p.Dp;
    if (nplanes < 0) nplanes = p.n_paths;
    if (p.l16)
        hipLaunchKernelGGL(sum_planes_kernel<uint16_t>, dim3(1024), dim3(256), 0, stream, ws.lbuf, plane, s_out,
                           p.W, p.H, p.D, p.Dp, nplanes, skip);
    else
        hipLaunchKernelGGL(sum_planes_kernel<uint8_t>, dim3(1024), dim3(256), 0, stream, ws.lbuf, plane, s_out,
                           p.W, p.H, p.D, p.Dp, nplanes, skip);
    return hipGetLastError();
}

hipError_t launch_extract_plane(const Plan& p, const Workspace& ws, int plane, uint16_t* out,
                                hipStream_t stream) {
    const size_t cells = (size_t)p.W * p.H * p.Dp;
    if (plane < 0)  // -1: the cost volume, -2: the right-base cost volume
        hipLaunchKernelGGL(extract_plane_kernel<uint8_t>, dim3(1024), dim3(256), 0, stream,
                           plane == -2 ? ws.cost_r : ws.cost, out, p.W, p.H, p.D, p.Dp);
    else if (p.l16)
        hipLaunchKernelGGL(extract_plane_kernel<uint16_t>, dim3(1024), dim3(256), 0, stream,
                           reinterpret_cast<const uint16_t*>(ws.lbuf) + cells * plane, out, p.W, p.H, p.D, p.Dp);
    else
        hipLaunchKernelGGL(extract_plane_kernel<uint8_t>, dim3(1024), dim3(256), 0, stream,
                           reinterpret_cast<const uint8_t*>(ws.lbuf) + cells * plane, out, p.W, p.H, p.D, p.Dp);
    return hipGetLastError();
}

}  // namespace sgm

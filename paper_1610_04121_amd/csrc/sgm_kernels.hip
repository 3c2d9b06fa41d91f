// SGM pipeline kernels for gfx950 (CDNA4, 64-wide wavefronts).
//
// Stages (Sec. 2 of arXiv 1610.04121):
//   census_cost_kernel  census of both images (Eq. 1 / full window) staged in
//                       LDS, then the Hamming cost volume C (Eq. 2), u8;
//   aggregate_kernel    Eq. 3 along every path direction, one wavefront per
//                       slice, all directions in one launch;
//   wta_kernel          S = sum_r L_r and winner-take-all (Eq. 4) for the
//                       left view, plus the right-view disparity;
//   post_kernel         3x3 median and left-right consistency check.
#include <hip/hip_runtime.h>

#include "sgm_plan.h"

namespace sgm {

namespace {

constexpr int kCostTX = 256;           // base pixels per census/cost block
constexpr uint32_t kBig = 1u << 30;    // "no such neighbour" in Eq. 3's minimum

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------------------
// Census (Sec. 3.1).  `tile` holds image rows y-ry..y+ry (clamped to the
// image) with pitch `pitch`; column c of the tile is image column xs + c,
// clamped.  (cx, ry) is the centre pixel in tile coordinates.
// ---------------------------------------------------------------------------
__device__ inline uint64_t census_full(const uint8_t* tile, int pitch, int cx, int rx, int ry) {
    const int cw = 2 * rx + 1;
    const int centre = tile[ry * pitch + cx];
    uint64_t word = 0;
    for (int j = -ry; j <= ry; ++j) {
        const uint8_t* row = tile + (ry + j) * pitch + cx;
        for (int i = -rx; i <= rx; ++i) {
            const uint64_t bit = row[i] >= centre ? 1u : 0u;
            word |= bit << ((j + ry) * cw + (i + rx));
        }
    }
    return word;
}

// Center-symmetric census, Eq. 1: pairs (x+i, y+j) vs (x-i, y-j) for
// i = 1..rx, j = -ry..ry, then (x, y+j) vs (x, y-j) for j = 1..ry.
__device__ inline uint64_t census_csct(const uint8_t* tile, int pitch, int cx, int rx, int ry) {
    uint64_t word = 0;
    int k = 0;
    for (int i = 1; i <= rx; ++i)
        for (int j = -ry; j <= ry; ++j, ++k) {
            const uint64_t bit =
                tile[(ry + j) * pitch + cx + i] >= tile[(ry - j) * pitch + cx - i] ? 1u : 0u;
            word |= bit << k;
        }
    for (int j = 1; j <= ry; ++j, ++k) {
        const uint64_t bit = tile[(ry + j) * pitch + cx] >= tile[(ry - j) * pitch + cx] ? 1u : 0u;
        word |= bit << k;
    }
    return word;
}

struct CostArgs {
    const uint8_t* left;
    const uint8_t* right;
    uint8_t* cost;
    int W, H, D, Dp, rx, ry, cmax, csct;
};

// One block per (row y, run of kCostTX base pixels).  The right census is
// needed from x0 - (D-1) on, because C(x, d) reads the match image at x - d.
__global__ __launch_bounds__(256) void census_cost_kernel(CostArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * kCostTX;
    const int nright = kCostTX + a.D - 1;
    const int xs = x0 - (a.D - 1) - a.rx;
    const int ncol = nright + 2 * a.rx;
    const int nrow = 2 * a.ry + 1;
    uint64_t* cl = reinterpret_cast<uint64_t*>(smem);
    uint64_t* cr = cl + kCostTX;
    uint8_t* tl = reinterpret_cast<uint8_t*>(cr + nright);
    uint8_t* tr = tl + nrow * ncol;

    for (int i = threadIdx.x; i < nrow * ncol; i += blockDim.x) {
        const int j = i / ncol, c = i - j * ncol;
        const size_t src = (size_t)clampi(y + j - a.ry, 0, a.H - 1) * a.W + clampi(xs + c, 0, a.W - 1);
        tl[i] = a.left[src];
        tr[i] = a.right[src];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kCostTX + nright; i += blockDim.x) {
        const bool is_left = i < kCostTX;
        const int k = is_left ? i : i - kCostTX;
        // tile column of the census centre
        const int cx = is_left ? (x0 + k) - xs : (x0 - (a.D - 1) + k) - xs;
        const uint8_t* t = is_left ? tl : tr;
        const uint64_t w = a.csct ? census_csct(t, ncol, cx, a.rx, a.ry) : census_full(t, ncol, cx, a.rx, a.ry);
        (is_left ? cl : cr)[k] = w;
    }
    __syncthreads();
    const int nq = a.Dp >> 2;  // 4 disparities per thread and store
    for (int i = threadIdx.x; i < kCostTX * nq; i += blockDim.x) {
        const int px = i / nq, q = i - px * nq;
        const int x = x0 + px;
        if (x >= a.W) break;
        const uint64_t base = cl[px];
        uint32_t word = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int d = 4 * q + j;
            uint32_t c;
            if (d >= a.D)
                c = 0;
            else if (x - d < 0)
                c = a.cmax;  // no candidate in the match image
            else
                c = __popcll(base ^ cr[px - d + a.D - 1]);
            word |= c << (8 * j);
        }
        *reinterpret_cast<uint32_t*>(a.cost + ((size_t)y * a.W + x) * a.Dp + 4 * q) = word;
    }
}

// Census only (debug tap): one thread per pixel straight from global memory.
__global__ __launch_bounds__(256) void census_only_kernel(const uint8_t* img, uint64_t* out, int W,
                                                          int H, int rx, int ry, int csct) {
    const int x = blockIdx.x * 16 + (threadIdx.x & 15);
    const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= W || y >= H) return;
    const int cw = 2 * rx + 1;
    const int centre = img[(size_t)y * W + x];
    uint64_t word = 0;
    if (!csct) {
        for (int j = -ry; j <= ry; ++j)
            for (int i = -rx; i <= rx; ++i) {
                const int v = img[(size_t)clampi(y + j, 0, H - 1) * W + clampi(x + i, 0, W - 1)];
                word |= (uint64_t)(v >= centre ? 1u : 0u) << ((j + ry) * cw + (i + rx));
            }
    } else {
        int k = 0;
        auto at = [&](int i, int j) {
            return (int)img[(size_t)clampi(y + j, 0, H - 1) * W + clampi(x + i, 0, W - 1)];
        };
        for (int i = 1; i <= rx; ++i)
            for (int j = -ry; j <= ry; ++j, ++k) word |= (uint64_t)(at(i, j) >= at(-i, -j) ? 1u : 0u) << k;
        for (int j = 1; j <= ry; ++j, ++k) word |= (uint64_t)(at(0, j) >= at(0, -j) ? 1u : 0u) << k;
    }
    out[(size_t)y * W + x] = word;
}

// ---------------------------------------------------------------------------
// Aggregation (Eq. 3).
//
// A wavefront owns one slice (a scanline of one direction) and walks it
// step by step; the recurrence forbids parallelism along the path (Sec. 3.2)
// so the parallelism is slices x disparities x directions.  Lane l holds
// disparities l*CPL .. l*CPL+CPL-1 of L_r(p - r, .) in registers.  Per step:
//   lp      = L + P1                     (the d+-1 candidates of Eq. 3)
//   R(d)    = min(L(d), lp(d-1), lp(d+1), m + P2)
//   L'(d)   = C(p, d) + R(d) - m         (m = min_k L(p - r, k))
//   m'      = min_d L'(d)                (wavefront min-reduction)
// The d-1 / d+1 values of a lane's first / last cell come from the
// neighbouring lanes through DPP row-crossing shifts; lanes without a
// neighbour read kBig, which never wins the minimum.  A restart (path start)
// sets L = 0 and m = 0, which makes L' = C exactly.  Padded levels d >= D add
// kBig to their cost, so they stay >= kBig and never win or leak.
// ---------------------------------------------------------------------------
struct AggArgs {
    const uint8_t* cost;
    void* lbuf;
    size_t plane;  // elements per L_r plane = H * W * Dp
    int W, H, D, Dp, P1, P2;
    int ndirs, total;
    int start[kMaxDirs + 1];  // first wave of each direction
    int rx[kMaxDirs], ry[kMaxDirs], plane_index[kMaxDirs];
};

// DPP controls (GFX9 encoding).
constexpr int kDppQuadPerm1032 = 0xB1;
constexpr int kDppQuadPerm2301 = 0x4E;
constexpr int kDppWaveShl1 = 0x130;  // lane i reads lane i+1
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i-1
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// Lane i receives lane i-1's (from_lower) or lane i+1's (from_upper) value;
// the lane without a source receives 0, which the caller ORs with kBig.
__device__ inline uint32_t from_lower_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppWaveShr1, 0xF, 0xF, true);
}
__device__ inline uint32_t from_upper_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppWaveShl1, 0xF, 0xF, true);
}

// Minimum over the 64 lanes as a wave-uniform (scalar) value: a butterfly
// inside each row of 16 lanes (DPP quad permutes and mirrors, folded into
// v_min_u32_dpp), then row broadcasts carry row 0's minimum into row 1 and
// row 2's into row 3, and rows 0-1's into rows 2-3; lane 63 ends with the
// minimum of all 64 lanes.  Lanes outside a broadcast's row mask keep their
// value (min(v, v) = v).
__device__ inline uint32_t wave_min(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppQuadPerm1032, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppQuadPerm2301, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowHalfMirror, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowMirror, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, kDppRowBcast15, 0xA, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, kDppRowBcast31, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

template <int CPL> struct RawCost;
template <> struct RawCost<1> { using T = uint8_t; };
template <> struct RawCost<2> { using T = uint16_t; };
template <> struct RawCost<4> { using T = uint32_t; };

template <int CPL>
__device__ inline void unpack_costs(uint32_t v, uint32_t (&c)[CPL]) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) c[i] = (v >> (8 * i)) & 0xFF;
}

template <int CPL, typename LT>
__device__ inline void store_l(LT* p, const uint32_t (&l)[CPL]) {
    if constexpr (sizeof(LT) == 1) {
        if constexpr (CPL == 1) {
            *p = (uint8_t)l[0];
        } else if constexpr (CPL == 2) {
            *reinterpret_cast<uint16_t*>(p) = (uint16_t)((l[0] & 0xFF) | (l[1] << 8));
        } else {
            *reinterpret_cast<uint32_t*>(p) =
                (l[0] & 0xFF) | ((l[1] & 0xFF) << 8) | ((l[2] & 0xFF) << 16) | (l[3] << 24);
        }
    } else {
        if constexpr (CPL == 1) {
            *p = (uint16_t)l[0];
        } else if constexpr (CPL == 2) {
            *reinterpret_cast<uint32_t*>(p) = (l[0] & 0xFFFF) | (l[1] << 16);
        } else {
            uint2 v;
            v.x = (l[0] & 0xFFFF) | (l[1] << 16);
            v.y = (l[2] & 0xFFFF) | (l[3] << 16);
            *reinterpret_cast<uint2*>(p) = v;
        }
    }
}

// Walks one slice by pixel offset (y * W + x).  Horizontal and vertical
// slices never restart after their first pixel; diagonal ones restart where
// they wrap around a side border (see walk_next).
enum { kHoriz = 0, kVert = 1, kDiag = 2 };

template <int KIND>
struct Walker {
    int x, po, rx, step, W;  // step = ry * W + rx
    bool restart;
    __device__ inline void next() {
        po += step;
        restart = false;
        if constexpr (KIND == kDiag) {
            // branch-free wrap: x < 0 -> +W, x >= W -> -W
            x += rx;
            const int under = x >> 31;
            const int over = (W - 1 - x) >> 31;
            const int wrap = (under & W) - (over & W);
            x += wrap;
            po += wrap;
            restart = (under | over) != 0;
        }
    }
};

// Cost loads run kPrefetch steps ahead of the recurrence so that their
// latency overlaps the dependent min-plus chain of the steps in between.
constexpr int kPrefetch = 16;

template <int CPL, typename LT, bool PAD, int KIND>
__device__ inline void aggregate_slice(const uint8_t* __restrict__ cost, LT* __restrict__ out, int lane, int D,
                                       uint32_t P1, uint32_t P2, Walker<KIND> w, int steps) {
    constexpr int kLog2Dp = CPL == 1 ? 6 : (CPL == 2 ? 7 : 8);
    using Raw = typename RawCost<CPL>::T;
    const unsigned lofs = lane * CPL;
    auto load = [&](int po) -> uint32_t {
        const uint8_t* p = cost + ((size_t)(unsigned)po << kLog2Dp);
        return *reinterpret_cast<const Raw*>(p + lofs);
    };
    // lanes without a d-1 / d+1 neighbour see kBig
    const uint32_t edge_lo = lane == 0 ? kBig : 0u;
    const uint32_t edge_hi = lane == 63 ? kBig : 0u;

    uint32_t pad[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) pad[c] = (PAD && lofs + c >= D) ? kBig : 0u;

    uint32_t L[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) L[c] = 0;
    uint32_t m = 0;
    // one step of Eq. 3 at the walker's pixel, then advance the walker
    auto step = [&](uint32_t raw) {
        if (w.restart) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) L[c] = 0;
            m = 0;
        }
        uint32_t cst[CPL];
        unpack_costs<CPL>(raw, cst);
        uint32_t lp[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) lp[c] = L[c] + P1;
        const uint32_t in_lo = from_lower_lane(lp[CPL - 1]) | edge_lo;
        const uint32_t in_hi = from_upper_lane(lp[0]) | edge_hi;
        const uint32_t mp2 = m + P2;
        uint32_t lmin = ~0u;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const uint32_t lo = c == 0 ? in_lo : lp[c - 1];
            const uint32_t hi = c == CPL - 1 ? in_hi : lp[c + 1];
            const uint32_t R = min(min(L[c], lo), min(hi, mp2));
            L[c] = R + (cst[c] | pad[c]) - m;
            lmin = min(lmin, L[c]);
        }
        m = wave_min(lmin);
        LT* o = out + ((size_t)(unsigned)w.po << kLog2Dp);
        store_l<CPL, LT>(o + lofs, L);
        w.next();
    };

    // ring[j] holds the raw costs of the step congruent to j modulo
    // kPrefetch.  The walker `ahead` leads by kPrefetch - 1 steps and stops at
    // the slice's last pixel, so every load is unconditional and in bounds
    // (loads past the end re-read the last pixel and are never consumed).
    uint32_t ring[kPrefetch];
    Walker<KIND> ahead = w;
    int ahead_k = 0;  // step index of `ahead`
    auto advance_ahead = [&]() {
        if (ahead_k + 1 < steps) {
            ahead.next();
            ++ahead_k;
        }
    };
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
        if (j) advance_ahead();
        ring[j] = load(ahead.po);
    }
    int k = 0;
    for (; k + kPrefetch <= steps; k += kPrefetch) {
#pragma unroll
        for (int j = 0; j < kPrefetch; ++j) {
            const uint32_t raw = ring[j];
            advance_ahead();
            ring[j] = load(ahead.po);
            step(raw);
        }
    }
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j)
        if (k + j < steps) step(ring[j]);
}

template <int CPL, typename LT, bool PAD>
__global__ __launch_bounds__(256) void aggregate_kernel(AggArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (wave >= a.total) return;
    int r = 0;
    while (r + 1 < a.ndirs && wave >= a.start[r + 1]) ++r;
    const Dir dir{a.rx[r], a.ry[r]};
    const int steps = slice_steps(a.W, a.H, dir);
    const Walk w0 = walk_start(a.W, a.H, dir, wave - a.start[r]);
    LT* out = reinterpret_cast<LT*>(a.lbuf) + a.plane * a.plane_index[r];
    const int po = w0.y * a.W + w0.x;
    const int step = dir.ry * a.W + dir.rx;
    if (dir.ry == 0)
        aggregate_slice<CPL, LT, PAD, kHoriz>(a.cost, out, lane, a.D, a.P1, a.P2,
                                               Walker<kHoriz>{w0.x, po, dir.rx, step, a.W, true}, steps);
    else if (dir.rx == 0)
        aggregate_slice<CPL, LT, PAD, kVert>(a.cost, out, lane, a.D, a.P1, a.P2,
                                              Walker<kVert>{w0.x, po, dir.rx, step, a.W, true}, steps);
    else
        aggregate_slice<CPL, LT, PAD, kDiag>(a.cost, out, lane, a.D, a.P1, a.P2,
                                              Walker<kDiag>{w0.x, po, dir.rx, step, a.W, true}, steps);
}

// ---------------------------------------------------------------------------
// Sum over directions and winner-take-all (Eq. 4), one block per row.
// Thread (x, g) sums 16 disparities 16g..16g+15 over all planes.  The left
// disparity is the smallest key (S << 9 | d) over the pixel's threads.  The
// right view: pixel x at disparity d is right pixel x - d, so every (x, d)
// offers its key to column x - d through an LDS atomic minimum; the column's
// winner is argmin_d S(x + d, d) with ties to the smallest d.
// ---------------------------------------------------------------------------
struct WtaArgs {
    const void* lbuf;
    size_t plane;
    uint16_t* dl;  // left disparity (raw, or the final output)
    uint16_t* dr;  // right disparity or nullptr
    int W, H, D, Dp, nplanes;
};

template <typename LT>
__device__ inline void load16(const LT* p, uint32_t (&v)[16]) {
    if constexpr (sizeof(LT) == 1) {
        const uint4 q = *reinterpret_cast<const uint4*>(p);
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = (w[i >> 2] >> (8 * (i & 3))) & 0xFF;
    } else {
        const uint4 q0 = reinterpret_cast<const uint4*>(p)[0];
        const uint4 q1 = reinterpret_cast<const uint4*>(p)[1];
        const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = (w[i >> 1] >> (16 * (i & 1))) & 0xFFFF;
    }
}

template <typename LT>
__global__ __launch_bounds__(1024) void wta_kernel(WtaArgs a) {
    extern __shared__ uint32_t keyR[];
    const int y = blockIdx.x;
    const bool right = a.dr != nullptr;
    if (right)
        for (int i = threadIdx.x; i < a.W; i += blockDim.x) keyR[i] = ~0u;
    __syncthreads();
    const int G = a.Dp >> 4;  // threads per pixel: 4, 8 or 16 (divides 64)
    const LT* base = reinterpret_cast<const LT*>(a.lbuf);
    for (int i = threadIdx.x; i < a.W * G; i += blockDim.x) {
        const int x = i / G, g = i - x * G;
        const size_t off = ((size_t)y * a.W + x) * a.Dp + 16 * g;
        uint32_t s[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) s[j] = 0;
        for (int p = 0; p < a.nplanes; ++p) {
            uint32_t v[16];
            load16<LT>(base + a.plane * p + off, v);
#pragma unroll
            for (int j = 0; j < 16; ++j) s[j] += v[j];
        }
        uint32_t best = ~0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int d = 16 * g + j;
            if (d < a.D) {
                const uint32_t key = (s[j] << 9) | (uint32_t)d;
                best = min(best, key);
                if (right && x - d >= 0) atomicMin(&keyR[x - d], key);
            }
        }
        for (int o = 1; o < G; o <<= 1) best = min(best, (uint32_t)__shfl_xor((int)best, o));
        if (g == 0) a.dl[(size_t)y * a.W + x] = (uint16_t)(best & 0x1FF);
    }
    if (right) {
        __syncthreads();
        for (int i = threadIdx.x; i < a.W; i += blockDim.x)
            a.dr[(size_t)y * a.W + i] = (uint16_t)(keyR[i] & 0x1FF);
    }
}

// ---------------------------------------------------------------------------
// 3x3 median (clamp-to-edge) of both maps, then the left-right check.
// The median of 9 is the median of (max of row minima, median of row
// medians, min of row maxima) once each row of 3 is sorted.
// ---------------------------------------------------------------------------
__device__ inline void sort3(uint32_t& a, uint32_t& b, uint32_t& c) {
    uint32_t t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
}

__device__ inline uint32_t med3(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}

__device__ inline uint32_t median9(const uint16_t* img, int W, int H, int x, int y) {
    uint32_t v[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint16_t* row = img + (size_t)clampi(y + j - 1, 0, H - 1) * W;
#pragma unroll
        for (int i = 0; i < 3; ++i) v[j][i] = row[clampi(x + i - 1, 0, W - 1)];
        sort3(v[j][0], v[j][1], v[j][2]);
    }
    const uint32_t lo = max(v[0][0], max(v[1][0], v[2][0]));
    const uint32_t mid = med3(v[0][1], v[1][1], v[2][1]);
    const uint32_t hi = min(v[0][2], min(v[1][2], v[2][2]));
    return med3(lo, mid, hi);
}

struct PostArgs {
    const uint16_t* dl;
    const uint16_t* dr;
    uint16_t* out;
    int W, H, median, lrcheck, thr;
};

__global__ __launch_bounds__(256) void post_kernel(PostArgs a) {
    extern __shared__ uint16_t rview[];
    const int y = blockIdx.x;
    if (a.lrcheck) {
        for (int x = threadIdx.x; x < a.W; x += blockDim.x)
            rview[x] = a.median ? (uint16_t)median9(a.dr, a.W, a.H, x, y) : a.dr[(size_t)y * a.W + x];
        __syncthreads();
    }
    for (int x = threadIdx.x; x < a.W; x += blockDim.x) {
        const int d = a.median ? (int)median9(a.dl, a.W, a.H, x, y) : (int)a.dl[(size_t)y * a.W + x];
        int o = d;
        if (a.lrcheck) {
            o = kInvalid;
            if (x - d >= 0) {
                const int e = rview[x - d];
                if (abs(d - e) <= a.thr) o = d;
            }
        }
        a.out[(size_t)y * a.W + x] = (uint16_t)o;
    }
}

// Debug tap: S = sum of planes, u16 [H][W][D].
template <typename LT>
__global__ void sum_planes_kernel(const void* lbuf, size_t plane, uint16_t* s, int W, int H, int D,
                                  int Dp, int nplanes) {
    const size_t n = (size_t)W * H * D;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / D, d = i - p * D;
        uint32_t acc = 0;
        for (int k = 0; k < nplanes; ++k) acc += reinterpret_cast<const LT*>(lbuf)[plane * k + p * Dp + d];
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
    if (p.W > kMaxWidth) return fail("width must be <= 16384");
    if (p.D < 1 || p.D > kMaxDisp) return fail("max_disp must be in [1, 256]");
    if (!(p.n_paths == 2 || p.n_paths == 4 || p.n_paths == 8)) return fail("n_paths must be 2, 4 or 8");
    if (p.cw < 1 || p.ch < 1 || !(p.cw & 1) || !(p.ch & 1)) return fail("census window sides must be odd and >= 1");
    if (p.cw > 31 || p.ch > 15) return fail("census window must be at most 31 wide and 15 tall");
    if (!p.csct && p.cw * p.ch > 64) return fail("full census window must have <= 64 pixels");
    if (p.csct && (p.cw * p.ch - 1) / 2 > 64) return fail("CSCT window must have <= 64 pairs");
    if (p.P1 < 0 || p.P2 < 0) return fail("P1 and P2 must be >= 0");
    if (p.P1 > 65535) return fail("P1 must be <= 65535");
    p.cmax = p.csct ? (p.cw * p.ch - 1) / 2 : p.cw * p.ch - 1;
    if ((long long)p.n_paths * (p.cmax + (long long)p.P2) > 65535)
        return fail("n_paths * (Cmax + P2) must be <= 65535 (16-bit summed costs)");
    if (p.lr_thr < 0) return fail("lr threshold must be >= 0");
    p.cpl = cells_per_lane(p.D);
    p.Dp = padded_disp(p.D);
    p.l16 = p.cmax + p.P2 > 255;
    return true;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t workspace_bytes(const Plan& p) {
    const size_t npx = (size_t)p.W * p.H;
    const size_t cells = npx * p.Dp;
    return align256(cells) + align256(cells * p.n_paths * (p.l16 ? 2 : 1)) + 2 * align256(npx * 2);
}

Workspace workspace_carve(const Plan& p, void* base) {
    const size_t npx = (size_t)p.W * p.H;
    const size_t cells = npx * p.Dp;
    uint8_t* b = static_cast<uint8_t*>(base);
    Workspace ws;
    ws.cost = b;
    b += align256(cells);
    ws.lbuf = b;
    b += align256(cells * p.n_paths * (p.l16 ? 2 : 1));
    ws.dl = reinterpret_cast<uint16_t*>(b);
    b += align256(npx * 2);
    ws.dr = reinterpret_cast<uint16_t*>(b);
    return ws;
}

hipError_t launch_census_cost(const Plan& p, const Workspace& ws, const uint8_t* left,
                              const uint8_t* right, hipStream_t stream) {
    CostArgs a{left, right, ws.cost, p.W, p.H, p.D, p.Dp, (p.cw - 1) / 2, (p.ch - 1) / 2, p.cmax, p.csct ? 1 : 0};
    const int nright = kCostTX + p.D - 1;
    const int ncol = nright + 2 * a.rx;
    const size_t smem = 8 * (size_t)(kCostTX + nright) + 2 * (size_t)(2 * a.ry + 1) * ncol;
    dim3 grid((p.W + kCostTX - 1) / kCostTX, p.H);
    hipLaunchKernelGGL(census_cost_kernel, grid, dim3(256), smem, stream, a);
    return hipGetLastError();
}

static void fill_agg_args(const Plan& p, const Workspace& ws, AggArgs& a) {
    a.cost = ws.cost;
    a.lbuf = ws.lbuf;
    a.plane = (size_t)p.W * p.H * p.Dp;
    a.W = p.W;
    a.H = p.H;
    a.D = p.D;
    a.Dp = p.Dp;
    a.P1 = p.P1;
    a.P2 = p.P2;
    a.ndirs = p.n_paths;
    // longest slices first, so that they start first
    int order[kMaxDirs], n = 0;
    const bool horiz_first = p.W >= p.H;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < p.n_paths; ++i) {
            const bool horiz = direction(p.n_paths, i).ry == 0;
            if ((horiz == horiz_first) == (pass == 0)) order[n++] = i;
        }
    int acc = 0;
    for (int k = 0; k < p.n_paths; ++k) {
        const Dir d = direction(p.n_paths, order[k]);
        a.rx[k] = d.rx;
        a.ry[k] = d.ry;
        a.plane_index[k] = order[k];
        a.start[k] = acc;
        acc += slice_count(p.W, p.H, d);
    }
    a.start[p.n_paths] = acc;
    a.total = acc;
}

template <int CPL, typename LT>
static void launch_agg_t(const AggArgs& a, bool pad, hipStream_t stream) {
    dim3 grid((a.total + 3) / 4);
    if (pad)
        hipLaunchKernelGGL((aggregate_kernel<CPL, LT, true>), grid, dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((aggregate_kernel<CPL, LT, false>), grid, dim3(256), 0, stream, a);
}

hipError_t launch_aggregate(const Plan& p, const Workspace& ws, hipStream_t stream) {
    AggArgs a;
    fill_agg_args(p, ws, a);
    const bool pad = p.D != p.Dp;
    switch (p.cpl * 2 + (p.l16 ? 1 : 0)) {
        case 2: launch_agg_t<1, uint8_t>(a, pad, stream); break;
        case 3: launch_agg_t<1, uint16_t>(a, pad, stream); break;
        case 4: launch_agg_t<2, uint8_t>(a, pad, stream); break;
        case 5: launch_agg_t<2, uint16_t>(a, pad, stream); break;
        case 8: launch_agg_t<4, uint8_t>(a, pad, stream); break;
        default: launch_agg_t<4, uint16_t>(a, pad, stream); break;
    }
    return hipGetLastError();
}

hipError_t launch_wta(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream) {
    const bool post = p.median || p.lrcheck;
    WtaArgs a{ws.lbuf, (size_t)p.W * p.H * p.Dp, post ? ws.dl : out, p.lrcheck ? ws.dr : nullptr,
              p.W, p.H, p.D, p.Dp, p.n_paths};
    const size_t smem = p.lrcheck ? 4 * (size_t)p.W : 0;
    if (p.l16)
        hipLaunchKernelGGL(wta_kernel<uint16_t>, dim3(p.H), dim3(1024), smem, stream, a);
    else
        hipLaunchKernelGGL(wta_kernel<uint8_t>, dim3(p.H), dim3(1024), smem, stream, a);
    return hipGetLastError();
}

hipError_t launch_post(const Plan& p, const Workspace& ws, uint16_t* out, hipStream_t stream) {
    if (!p.median && !p.lrcheck) return hipSuccess;  // the WTA wrote `out`
    PostArgs a{ws.dl, ws.dr, out, p.W, p.H, p.median ? 1 : 0, p.lrcheck ? 1 : 0, p.lr_thr};
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
    if (e == hipSuccess) e = launch_census_cost(p, ws, left, right, stream);
    mark(1);
    if (e == hipSuccess) e = launch_aggregate(p, ws, stream);
    mark(2);
    if (e == hipSuccess) e = launch_wta(p, ws, out, stream);
    mark(3);
    if (e == hipSuccess) e = launch_post(p, ws, out, stream);
    mark(4);
    return e;
}

hipError_t launch_census_only(const Plan& p, const uint8_t* img, uint64_t* out, hipStream_t stream) {
    dim3 grid((p.W + 15) / 16, (p.H + 15) / 16);
    hipLaunchKernelGGL(census_only_kernel, grid, dim3(256), 0, stream, img, out, p.W, p.H, (p.cw - 1) / 2,
                       (p.ch - 1) / 2, p.csct ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_sum_planes(const Plan& p, const Workspace& ws, uint16_t* s_out, hipStream_t stream) {
    const size_t plane = (size_t)p.W * p.H * p.Dp;
    if (p.l16)
        hipLaunchKernelGGL(sum_planes_kernel<uint16_t>, dim3(1024), dim3(256), 0, stream, ws.lbuf, plane, s_out,
                           p.W, p.H, p.D, p.Dp, p.n_paths);
    else
        hipLaunchKernelGGL(sum_planes_kernel<uint8_t>, dim3(1024), dim3(256), 0, stream, ws.lbuf, plane, s_out,
                           p.W, p.H, p.D, p.Dp, p.n_paths);
    return hipGetLastError();
}

hipError_t launch_extract_plane(const Plan& p, const Workspace& ws, int plane, uint16_t* out,
                                hipStream_t stream) {
    const size_t cells = (size_t)p.W * p.H * p.Dp;
    if (plane < 0)
        hipLaunchKernelGGL(extract_plane_kernel<uint8_t>, dim3(1024), dim3(256), 0, stream, ws.cost, out, p.W, p.H,
                           p.D, p.Dp);
    else if (p.l16)
        hipLaunchKernelGGL(extract_plane_kernel<uint16_t>, dim3(1024), dim3(256), 0, stream,
                           reinterpret_cast<const uint16_t*>(ws.lbuf) + cells * plane, out, p.W, p.H, p.D, p.Dp);
    else
        hipLaunchKernelGGL(extract_plane_kernel<uint8_t>, dim3(1024), dim3(256), 0, stream,
                           reinterpret_cast<const uint8_t*>(ws.lbuf) + cells * plane, out, p.W, p.H, p.D, p.Dp);
    return hipGetLastError();
}

}  // namespace sgm

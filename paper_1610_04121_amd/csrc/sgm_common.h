// Host/device definitions shared by the SGM kernels and the C ABI.
//
// Terminology follows the paper (arXiv 1610.04121): C is the matching cost
// (Eq. 2), L_r the aggregated cost of path direction r (Eq. 3), S the sum
// over directions (Eq. 4).  D is the number of disparity levels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgm {

constexpr int kMaxDirs = 8;
constexpr int kMaxDisp = 256;
constexpr long long kMallBytes = 256ll << 20;  // MI355X memory-side (Infinity) cache
constexpr int kMaxWidth = 16000;  // the WTA keeps 4 * (W + 256) bytes of keys in LDS (< 64 KiB)
constexpr uint32_t kInvalid = 0xFFFF;
// words of addressable space in front of each census buffer in the workspace
constexpr int kCensusGuard = 256;

// Path directions (rx, ry): 2 paths = left-to-right and top-to-bottom
// (Sec. 4); 4 = the axial ones; 8 = axial plus diagonal.
struct Dir {
    int rx, ry;
};

__host__ __device__ inline Dir direction(int n_paths, int i) {
    const int axial[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
    if (n_paths == 2) i = (i == 0) ? 0 : 2;
    return Dir{axial[i][0], axial[i][1]};
}

// Aggregation work is cut into slices that run one wavefront each.
// Horizontal directions have one slice per row (W steps); every other
// direction has one slice per column (H steps).  A diagonal slice moves one
// row per step and wraps from one side border to the other when x leaves the
// image, restarting the path there (the wrap-around schedule of Sec. 3.2), so
// every slice has the same length and each pixel lies on exactly one slice.
__host__ __device__ inline int slice_count(int W, int H, Dir r) { return r.ry == 0 ? H : W; }
__host__ __device__ inline int slice_steps(int W, int H, Dir r) { return r.ry == 0 ? W : H; }

struct Walk {
    int x, y;
    bool restart;
};

__host__ __device__ inline Walk walk_start(int W, int H, Dir r, int slice) {
    if (r.ry == 0) return Walk{r.rx > 0 ? 0 : W - 1, slice, true};
    return Walk{slice, r.ry > 0 ? 0 : H - 1, true};
}

__host__ __device__ inline void walk_next(int W, Walk& w, Dir r) {
    w.restart = false;
    w.y += r.ry;
    w.x += r.rx;
    if (w.x < 0) {
        w.x += W;
        w.restart = true;
    } else if (w.x >= W) {
        w.x -= W;
        w.restart = true;
    }
}

// Disparity levels are padded to Dp in {64, 128, 256}, so that a group of
// 16, 32 or 64 lanes holds an even number of levels per lane.
inline int padded_disp(int D) { return D <= 64 ? 64 : (D <= 128 ? 128 : 256); }

}  // namespace sgm

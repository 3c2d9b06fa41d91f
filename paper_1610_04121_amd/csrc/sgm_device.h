// Device code of the SGM pipeline for gfx950 (CDNA4, 64-wide wavefronts),
// shared by the single-pair kernels and the batched kernels.  Each stage is
// a device function that takes its block coordinates explicitly.
//
// Stages (Sec. 2 of arXiv 1610.04121):
//   census97_block / census_generic_block  census words (Eq. 1 / full window)
//   cost_block      Hamming cost volume C (Eq. 2), u8
//   aggregate_wave  Eq. 3 along one direction, one group of lanes per slice
//   wta_row         S = sum_r L_r and winner-take-all (Eq. 4), right view
//   post_row        3x3 median and left-right consistency check
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "sgm_common.h"

namespace sgm {
namespace dev {



__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// 16-byte store at byte offset `ofs` of [base, base + bytes) through a
// range-checked buffer resource, with device scope (sc1): measured faster
// than plain stores for the cost volume, whose wavefronts store contiguous
// runs (whole lines).
__device__ inline void store16_sc1(void* base, uint32_t bytes, uint32_t ofs, uint4 v) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b128((unsigned __attribute__((ext_vector_type(4)))){v.x, v.y, v.z, v.w}, r, ofs,
                                           0, 16);
}

// ---------------------------------------------------------------------------
// Census kernel: 9x7 windows (full or center-symmetric), register blocked.
// A block covers 64 x 16 pixels of one image (blockIdx.z); each thread makes
// 4 consecutive census words of one row.  The block stages a (16 + 6) x 72
// tile (clamp-to-edge), and each thread reads its 12 x 7 window patch as
// 3 aligned dwords per row.  The comparisons s(u, v) = [u >= v] of the 4
// pixels run byte-parallel in one dword (census_words4).
// ---------------------------------------------------------------------------
constexpr int kCenTX = 64, kCenTY = 16;

struct CensusArgs {
    const uint8_t* img[2];
    uint64_t* out[2];
    int W, H, csct;
    // block (0, 0, 0) clears zero[0 .. nzero) for the frame's later launches
    // (the row counters of the post stage inside the WTA launch)
    int* zero = nullptr;
    int nzero = 0;
};

__device__ inline void census_clear(const CensusArgs& a, int bx, int by, int z) {
    if (a.zero && (bx | by | z) == 0)
        for (int i = threadIdx.x; i < a.nzero; i += blockDim.x) a.zero[i] = 0;
}

// Byte-parallel comparison: bit 7 of byte b of the result is [u_b >= v_b]
// for unsigned bytes (the other bits are don't-care).  vlo = v & 0x7F7F7F7F.
// (u | 0x80) - (v & 0x7F) per byte lies in [1, 255], so no borrow crosses a
// byte, and its bit 7 compares the low 7 bits; the top bits decide whenever
// they differ.
__device__ inline uint32_t ge_bytes(uint32_t u, uint32_t v, uint32_t vlo) {
    const uint32_t d = (u | 0x80808080u) - vlo;
    return (u & ~v) | (~(u ^ v) & d);
}

// Moves each byte of acc down one bit and puts bit 7 of the byte of g on top.
__device__ inline uint32_t push_bits(uint32_t acc, uint32_t g) {
    return ((acc >> 1) & 0x7F7F7F7Fu) | (g & 0x80808080u);
}

// o[p] byte b = a[b] byte p (4x4 byte transpose).
__device__ inline void transpose_bytes4(const uint32_t (&a)[4], uint32_t (&o)[4]) {
    const uint32_t t01l = __builtin_amdgcn_perm(a[1], a[0], 0x05010400u);
    const uint32_t t01h = __builtin_amdgcn_perm(a[1], a[0], 0x07030602u);
    const uint32_t t23l = __builtin_amdgcn_perm(a[3], a[2], 0x05010400u);
    const uint32_t t23h = __builtin_amdgcn_perm(a[3], a[2], 0x07030602u);
    o[0] = __builtin_amdgcn_perm(t23l, t01l, 0x05040100u);
    o[1] = __builtin_amdgcn_perm(t23l, t01l, 0x07060302u);
    o[2] = __builtin_amdgcn_perm(t23h, t01h, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(t23h, t01h, 0x07060302u);
}

// Census words (9x7 window, full or center-symmetric) of 4 consecutive
// pixels of one row, from a byte tile with row pitch TW (a multiple of 4).
// Pixel p (0..3) has its window on tile rows r0 .. r0+6 and columns
// c0+p .. c0+p+8 (centre at row r0+3, column c0+p+4); c0 is a multiple of 4,
// so each window row is read as 3 aligned dwords.
//
// The 4 pixels' samples at one window offset are 4 consecutive bytes of a
// tile row, so one dword holds them and ge_bytes compares all four.  Byte b
// of the census word (bits 8b .. 8b+7) is gathered for the 4 pixels in the
// 4 bytes of acc[b], one push_bits per bit; a byte transpose then turns the
// per-bit-byte registers into per-pixel words.
__device__ inline void census_words4(const uint8_t* tile, int TW, int r0, int c0, bool csct, uint64_t words[4]) {
    constexpr int RY = 3, CW = 9;
    uint32_t dw[2 * RY + 1][3];
#pragma unroll
    for (int j = 0; j < 2 * RY + 1; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) dw[j][k] = *reinterpret_cast<const uint32_t*>(&tile[(r0 + j) * TW + c0 + 4 * k]);
    // bytes b .. b+3 of window row j (b in 0..8): column offset b - 4 of the 4 pixels
    auto at = [&](int j, int b) -> uint32_t {
        const int q = b >> 2, s = b & 3;
        return s == 0 ? dw[j][q] : __builtin_amdgcn_alignbit(dw[j][q + 1], dw[j][q], 8 * s);
    };
    uint32_t acc[8];
    if (!csct) {
        // bit k = (j, i) of the window: k = j * 9 + i, j in 0..6, i in 0..8
        const uint32_t c = at(RY, 4), clo = c & 0x7F7F7F7Fu;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint32_t a = 0;
            const int nb = b < 7 ? 8 : (2 * RY + 1) * CW - 56;  // 7 bits in the top byte
#pragma unroll
            for (int t = 0; t < nb; ++t) {
                const int k = 8 * b + t;
                a = push_bits(a, ge_bytes(at(k / CW, k % CW), c, clo));
            }
            acc[b] = nb == 8 ? a : (a >> (8 - nb)) & (0xFFu >> (8 - nb)) * 0x01010101u;
        }
    } else {
        // pairs in order k = 0..30: i = 1..4 with j = -3..3, then (0, j), j = 1..3
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t a = 0;
            const int nb = b < 3 ? 8 : 7;
#pragma unroll
            for (int t = 0; t < nb; ++t) {
                const int k = 8 * b + t;
                int i, j;
                if (k < 28) {
                    i = 1 + k / 7;
                    j = k % 7 - 3;
                } else {
                    i = 0;
                    j = k - 27;
                }
                const uint32_t u = at(RY + j, 4 + i), v = at(RY - j, 4 - i);
                a = push_bits(a, ge_bytes(u, v, v & 0x7F7F7F7Fu));
            }
            acc[b] = nb == 8 ? a : (a >> 1) & 0x7F7F7F7Fu;
        }
#pragma unroll
        for (int b = 4; b < 8; ++b) acc[b] = 0;
    }
    uint32_t lo[4], hi[4];
    transpose_bytes4({acc[0], acc[1], acc[2], acc[3]}, lo);
    transpose_bytes4({acc[4], acc[5], acc[6], acc[7]}, hi);
#pragma unroll
    for (int p = 0; p < 4; ++p) words[p] = ((uint64_t)hi[p] << 32) | lo[p];
}

__device__ inline void census97_block(const CensusArgs& a, int bx, int by, int z) {
    census_clear(a, bx, by, z);
    constexpr int RY = 3;
    constexpr int TW = kCenTX + 8, TH = kCenTY + 2 * RY;
    __shared__ __align__(16) uint8_t tile[TH * TW];

    const uint8_t* img = a.img[z];
    const int x0 = bx * kCenTX, y0 = by * kCenTY;
    // all loads first, then the LDS stores (the block has 256 threads)
    constexpr int kIt = (TH * TW + 255) / 256;
    uint32_t v[kIt];
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int r = i / TW, c = i - r * TW;
        const int yy = clampi(y0 - RY + r, 0, a.H - 1), xx = clampi(x0 - 4 + c, 0, a.W - 1);
        v[k] = i < TH * TW ? img[(size_t)yy * a.W + xx] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kIt; ++k)
        if (threadIdx.x + 256 * k < TH * TW) tile[threadIdx.x + 256 * k] = (uint8_t)v[k];
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int y = y0 + ty;
    uint64_t words[4];
    census_words4(tile, TW, ty, 4 * tx, a.csct != 0, words);
    const int x = x0 + 4 * tx;
    if (y < a.H) {
        uint64_t* o = a.out[z] + (size_t)y * a.W + x;
        if (x + 3 < a.W && ((a.W & 1) == 0)) {
            // plain (write-back) stores: a thread's two 16-byte stores fill
            // the two halves of its 32 bytes, which the L2 merges; with
            // device scope each half would be written through on its own
            reinterpret_cast<ulonglong2*>(o)[0] = make_ulonglong2(words[0], words[1]);
            reinterpret_cast<ulonglong2*>(o)[1] = make_ulonglong2(words[2], words[3]);
        } else {
#pragma unroll
            for (int p = 0; p < 4; ++p)
                if (x + p < a.W) o[p] = words[p];
        }
    }
}

// Any other window: one thread per pixel, straight from global memory.
__device__ inline void census_generic_block(const CensusArgs& a, int rx, int ry, int bx, int by, int z) {
    census_clear(a, bx, by, z);
    const int x = bx * 16 + (threadIdx.x & 15);
    const int y = by * 16 + (threadIdx.x >> 4);

    if (x >= a.W || y >= a.H) return;
    const uint8_t* img = a.img[z];
    auto at = [&](int i, int j) {
        return (int)img[(size_t)clampi(y + j, 0, a.H - 1) * a.W + clampi(x + i, 0, a.W - 1)];
    };
    const int cw = 2 * rx + 1;
    uint64_t word = 0;
    if (!a.csct) {
        const int c = at(0, 0);
        for (int j = -ry; j <= ry; ++j)
            for (int i = -rx; i <= rx; ++i)
                word |= (uint64_t)(at(i, j) >= c ? 1u : 0u) << ((j + ry) * cw + (i + rx));
    } else {
        int k = 0;
        for (int i = 1; i <= rx; ++i)
            for (int j = -ry; j <= ry; ++j, ++k) word |= (uint64_t)(at(i, j) >= at(-i, -j) ? 1u : 0u) << k;
        for (int j = 1; j <= ry; ++j, ++k) word |= (uint64_t)(at(0, j) >= at(0, -j) ? 1u : 0u) << k;
    }
    a.out[z][(size_t)y * a.W + x] = word;
}

// ---------------------------------------------------------------------------
// Matching cost (Eq. 2).  One block per (row y, run of 64 base pixels).  The
// census words of the run and of the match run from x0 - (D-1) on are staged
// in LDS.  Lane l of every wavefront is pixel x0 + l, so the match words a
// wavefront reads for one disparity are consecutive (no bank conflicts) and
// their addresses differ by constants (immediate offsets).  Each wavefront
// computes runs of 16 disparities, writes them to an LDS tile [64][Dp + 16]
// (the padding spreads rows over banks), and the block then copies the tile
// to the cost volume with contiguous 16-byte stores.
// ---------------------------------------------------------------------------
constexpr int kCostTX = 64;
constexpr int kCostThreads = 256;  // block size of every launch of cost_block

struct CostArgs {
    const uint64_t* cl;
    const uint64_t* cr;
    uint8_t* cost;
    int W, H, D, Dp, cmax;
};

// RB = false: base words cl = left view, match words cr = right view at x - d
// (Eq. 2).  RB = true: base = right view, match = left view at x + d (the
// right-base costs of the full left-right check).  DP = a.Dp (64, 128 or
// 256) as a constant, so the chunk and copy loops unroll and the tile pitch
// is an immediate.
template <bool RB, int DP>
__device__ inline void cost_block(const CostArgs& a, int bx, int y, uint64_t* cw_smem) {
    static_assert(DP == 64 || DP == 128 || DP == 256, "padded disparity range");
    const int x0 = bx * kCostTX;
    const int D = a.D;
    constexpr int Dp = DP;
    const int nright = kCostTX + D - 1;
    constexpr int tpitch = Dp + 16;  // bytes per tile row
    uint64_t* cl = cw_smem;
    // cr[i] = match word of column xm0 + i
    uint64_t* cr = cl + kCostTX;
    const int xm0 = RB ? x0 : x0 - (D - 1);
    // the tile starts on a 16-byte boundary (an even number of words)
    uint8_t* tile = reinterpret_cast<uint8_t*>(cl + ((kCostTX + nright + 1) & ~1));
    const uint64_t* gl = a.cl + (size_t)y * a.W;
    const uint64_t* gr = a.cr + (size_t)y * a.W;
    // Every global load is issued before the first LDS store, so the loads'
    // latencies overlap instead of adding up.  The block has kCostThreads
    // threads: one base word each for the first 64, and the match words
    // (nright <= kCostTX + 255 < 2 * kCostThreads) in two rounds.
    {
        const int t = threadIdx.x;
        uint64_t vl = 0, vr[2] = {0, 0};
        const bool hl = t < kCostTX && x0 + t < a.W;
        if (hl) vl = gl[x0 + t];
        bool hr[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = t + kCostThreads * k, xr = xm0 + i;
            hr[k] = i < nright && xr >= 0 && xr < a.W;
            if (hr[k]) vr[k] = gr[xr];
        }
        if (hl) cl[t] = vl;
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (hr[k]) cr[t + kCostThreads * k] = vr[k];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = x0 + lane;
    const uint64_t base = cl[lane];
    constexpr int nchunks = Dp >> 4;
    constexpr int nwaves = kCostThreads / 64;
#pragma unroll
    for (int it = 0; it < nchunks / nwaves; ++it) {
        const int ch = wave + nwaves * it;
        const int d0 = 16 * ch;
        // match word of disparity d0 + j: cr[lane + D - 1 - d0 - j] (left
        // base), cr[lane + d0 + j] (right base)
        auto word = [&](int j) -> uint64_t { return RB ? cr[lane + d0 + j] : cr[lane + D - 1 - d0 - j]; };
        // all 16 disparities inside the image for every lane of the run
        const bool inside = RB ? (x0 + kCostTX - 1 + d0 + 15 < a.W) : (x0 >= d0 + 15);
        uint32_t w[4];
        if (inside && d0 + 16 <= D) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t wd = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) wd |= (uint32_t)__popcll(base ^ word(4 * q + j)) << (8 * j);
                w[q] = wd;
            }
        } else if (d0 + 16 <= D) {
            // a run at the image border: every lane's LDS word exists, so
            // every lane takes the popcount and a select puts Cmax where the
            // match pixel is outside the image (no per-lane branch)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t wd = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int d = d0 + 4 * q + j;
                    const uint32_t pc = (uint32_t)__popcll(base ^ word(4 * q + j));
                    const bool out = RB ? x + d >= a.W : x - d < 0;
                    wd |= (out ? (uint32_t)a.cmax : pc) << (8 * j);
                }
                w[q] = wd;
            }
        } else {  // the chunk holding D - 1 and the padded levels
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t wd = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int d = d0 + 4 * q + j;
                    uint32_t c = 0;  // padded levels d >= D
                    if (d < D) {
                        const uint32_t pc = (uint32_t)__popcll(base ^ word(4 * q + j));
                        const bool out = RB ? x + d >= a.W : x - d < 0;
                        c = out ? (uint32_t)a.cmax : pc;
                    }
                    wd |= c << (8 * j);
                }
                w[q] = wd;
            }
        }
        *reinterpret_cast<uint4*>(tile + lane * tpitch + d0) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    __syncthreads();
    const int npx = min(kCostTX, a.W - x0);
    uint8_t* dst = a.cost + ((size_t)y * a.W + x0) * Dp;
    // kCostTX * nchunks 16-byte pieces, nchunks / nwaves per thread: all LDS
    // reads first, then the stores
    constexpr int nper = kCostTX * nchunks / kCostThreads;
    uint4 v[nper];
#pragma unroll
    for (int j = 0; j < nper; ++j) {
        const int c = threadIdx.x + kCostThreads * j;
        v[j] = *reinterpret_cast<const uint4*>(tile + (c / nchunks) * tpitch + 16 * (c % nchunks));
    }
#pragma unroll
    for (int j = 0; j < nper; ++j) {
        const int c = threadIdx.x + kCostThreads * j;
        if (c < npx * nchunks) store16_sc1(dst, (uint32_t)(npx * Dp), 16u * (uint32_t)c, v[j]);
    }
}

// ---------------------------------------------------------------------------
// Census + matching cost in one pass (9x7 windows).  One block per (row y,
// segment of kCcRuns runs of 64 base pixels).  The block stages the 7 image
// rows around y of both views in LDS (clamp-to-edge): the base view over the
// segment, the match view over the segment plus the D - 1 columns to its
// left.  It computes every census word it needs exactly once into LDS, then
// for each run of 64 pixels builds the costs in an LDS tile [64][Dp + 16]
// (two tiles, alternating, so one run's copy-out overlaps the next run's
// popcounts) and writes the run's slice of the cost volume with contiguous
// 16-byte stores.  No census word goes through global memory.
// ---------------------------------------------------------------------------
constexpr int kCcRuns = 4;
constexpr int kCcTX = 64 * kCcRuns;

struct CensusCostArgs {
    const uint8_t* left;
    const uint8_t* right;
    uint8_t* cost;
    int W, H, D, Dp, cmax, csct;
    int* zero = nullptr;  // as CensusArgs::zero
    int nzero = 0;
};

// Byte sizes of the LDS regions of census_cost_block.
struct CcLayout {
    int twl, twr;     // tile row pitches (bytes), base / match view
    int nr;           // match census words: kCcTX + D - 1, rounded up to 4
    int words_off;    // byte offset of the census words (base, then match)
    int tiles_off;    // byte offset of the two cost tiles
    int tpitch;       // bytes per cost-tile row
    int bytes;        // total
};

__host__ __device__ inline CcLayout cc_layout(int D, int Dp) {
    CcLayout L;
    L.twl = kCcTX + 8;
    L.nr = (kCcTX + D - 1 + 3) & ~3;
    L.twr = L.nr + 8;
    L.words_off = (7 * (L.twl + L.twr) + 15) & ~15;
    L.tiles_off = L.words_off + 8 * (kCcTX + L.nr);
    L.tpitch = Dp + 16;
    L.bytes = L.tiles_off + 2 * 64 * L.tpitch;
    return L;
}

__device__ inline void census_cost_block(const CensusCostArgs& a, int bx, int y, uint8_t* smem) {
    if (a.zero && (bx | y) == 0)
        for (int i = threadIdx.x; i < a.nzero; i += blockDim.x) a.zero[i] = 0;
    constexpr int RY = 3;
    const int D = a.D, Dp = a.Dp;
    const CcLayout L = cc_layout(D, Dp);
    const int x0 = bx * kCcTX;
    const int xs = x0 - (D - 1);  // first match column
    uint8_t* tl = smem;           // base view tile: 7 rows, columns x0 - 4 ..
    uint8_t* tr = smem + 7 * L.twl;  // match view tile: 7 rows, columns xs - 4 ..
    uint64_t* cl = reinterpret_cast<uint64_t*>(smem + L.words_off);  // cl[i]: column x0 + i
    uint64_t* cr = cl + kCcTX;                                        // cr[i]: column xs + i
    uint8_t* tiles = smem + L.tiles_off;

    // Stage the 7 image rows of both views.  Every load is issued before the
    // first LDS store, so the loads' latencies overlap instead of adding up
    // (the block has 256 threads; a base row has kCcTX + 8 <= 512 bytes, a
    // match row at most 520 <= 768).
    {
        const int t = threadIdx.x;
        uint32_t vl[7][2], vr[7][3];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            const size_t row = (size_t)clampi(y - RY + r, 0, a.H - 1) * a.W;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int c = t + 256 * k;
                vl[r][k] = c < L.twl ? a.left[row + clampi(x0 - 4 + c, 0, a.W - 1)] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int c = t + 256 * k;
                vr[r][k] = c < L.twr ? a.right[row + clampi(xs - 4 + c, 0, a.W - 1)] : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < 7; ++r) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (t + 256 * k < L.twl) tl[r * L.twl + t + 256 * k] = (uint8_t)vl[r][k];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (t + 256 * k < L.twr) tr[r * L.twr + t + 256 * k] = (uint8_t)vr[r][k];
        }
    }
    __syncthreads();
    {
        const int nl4 = kCcTX / 4, nr4 = L.nr / 4;
        for (int t = threadIdx.x; t < nl4 + nr4; t += blockDim.x) {
            uint64_t w[4];
            if (t < nl4) {
                census_words4(tl, L.twl, 0, 4 * t, a.csct != 0, w);
#pragma unroll
                for (int p = 0; p < 4; ++p) cl[4 * t + p] = w[p];
            } else {
                const int u = t - nl4;
                census_words4(tr, L.twr, 0, 4 * u, a.csct != 0, w);
#pragma unroll
                for (int p = 0; p < 4; ++p) cr[4 * u + p] = w[p];
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int nchunks = Dp >> 4;
    for (int run = 0; run < kCcRuns; ++run) {
        const int xr0 = x0 + 64 * run;
        if (xr0 >= a.W) break;  // the same for the whole block
        uint8_t* tile = tiles + (run & 1) * 64 * L.tpitch;
        const int x = xr0 + lane;
        const uint64_t base = cl[64 * run + lane];
        for (int ch = wave; ch < nchunks; ch += nwaves) {
            const int d0 = 16 * ch;
            // match word of disparity d0 + j is cr[64 run + lane + D - 1 - d0 - j]
            const uint64_t* m = cr + (64 * run + lane + D - 1 - d0 - 15);
            uint32_t w[4];
            if (xr0 >= d0 + 15 && d0 + 16 <= D) {  // all 16 disparities valid for every lane
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t word = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) word |= (uint32_t)__popcll(base ^ m[15 - (4 * q + j)]) << (8 * j);
                    w[q] = word;
                }
            } else if (d0 + 16 <= D) {  // at the border: popcount on every lane, then a select
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t word = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t pc = (uint32_t)__popcll(base ^ m[15 - (4 * q + j)]);
                        word |= (x - (d0 + 4 * q + j) < 0 ? (uint32_t)a.cmax : pc) << (8 * j);
                    }
                    w[q] = word;
                }
            } else {  // the chunk holding D - 1 and the padded levels
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t word = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int d = d0 + 4 * q + j;
                        uint32_t c = 0;  // padded levels d >= D
                        if (d < D) {
                            const uint32_t pc = (uint32_t)__popcll(base ^ m[15 - (4 * q + j)]);
                            c = x - d < 0 ? (uint32_t)a.cmax : pc;
                        }
                        word |= c << (8 * j);
                    }
                    w[q] = word;
                }
            }
            *reinterpret_cast<uint4*>(tile + lane * L.tpitch + d0) = make_uint4(w[0], w[1], w[2], w[3]);
        }
        __syncthreads();
        const int npx = min(64, a.W - xr0);
        const int lg = Dp == 64 ? 2 : (Dp == 128 ? 3 : 4);  // log2(nchunks)
        uint8_t* dst = a.cost + ((size_t)y * a.W + xr0) * Dp;
        for (int c = threadIdx.x; c < npx * nchunks; c += blockDim.x) {
            const int px = c >> lg, k = c & (nchunks - 1);
            store16_sc1(dst, (uint32_t)(npx * Dp), 16u * (uint32_t)c,
                        *reinterpret_cast<const uint4*>(tile + px * L.tpitch + 16 * k));
        }
    }
}

// ---------------------------------------------------------------------------
// Aggregation (Eq. 3).
//
// The recurrence forbids parallelism along a path (Sec. 3.2), so the work is
// spread over slices x disparities x directions.  A group of G lanes (G in
// {16, 32, 64}) owns one slice and walks it step by step; a wavefront holds
// S = 64 / G slices of the same direction.  Lane q of a group holds the
// disparities q*CPL .. q*CPL + CPL - 1 (CPL = Dp / G) of L_r(p - r, .) as
// CPL/2 packed u16 pairs in a "split" layout: pair k holds disparities
// q*CPL + k (low half) and q*CPL + k + CPL/2 (high half), so the d-1 / d+1
// neighbours of pair k are pairs k-1 / k+1 of the same lane, except at the
// lane's two ends, which take one DPP lane shift and one v_alignbit each.
// Per step, in saturating u16 arithmetic:
//   lp    = L + P1                          (the d+-1 candidates of Eq. 3)
//   R(d)  = min(L(d), lp(d-1), lp(d+1), m + P2)
//   L'(d) = R(d) - m + C(p, d)              (m = min_k L(p - r, k))
//   m'    = min_d L'(d)                     (group min-reduction)
// 0xFFFF stands for "no such disparity": the d-1 of d = 0, the d+1 of
// d = D-1 and padded levels d >= D (their cost is 0xFFFF, so they stay
// 0xFFFF).  Real values are at most Cmax + 2*P2 < 0xFFFF (validated), so
// saturation never changes a result.  A path start sets L = 0 and m = 0,
// which makes L' = C exactly.
// ---------------------------------------------------------------------------
// Everything one wavefront needs to aggregate slices of one direction.
struct SliceArgs {
    const uint8_t* cost;       // C u8 [H][W][Dp] (cost-volume variant)
    const uint64_t* census_l;  // census words (fused variant)
    const uint64_t* census_r;
    void* lplane;              // this direction's L_r plane [H][W][Dp]
    uint32_t plane;            // elements per plane = H * W * Dp
    int W, H, D, P1, P2, cmax, rx, ry;
    const uint8_t* img = nullptr;      // base image u8 [H][W] (adaptive P2)
    const uint16_t* p2lut = nullptr;   // LDS: adaptive P2 of each intensity change 0..255
};

// Adaptive P2 of one step: max(P1, floor(P2 / (1 + g))) for an intensity
// change g in [0, 255].  A block tabulates it once in LDS (fill_p2_lut) and
// the recurrence looks values up.
__device__ inline uint32_t adaptive_p2(uint32_t P1, uint32_t P2, uint32_t g) {
    const uint32_t q = P2 / (1u + g);
    return q > P1 ? q : P1;
}

// Fills lut[0..255] with adaptive_p2 (all threads of the block take part;
// the caller synchronizes before use).
__device__ inline void fill_p2_lut(uint16_t* lut, int P1, int P2) {
    for (int g = threadIdx.x; g < 256; g += blockDim.x) lut[g] = (uint16_t)adaptive_p2((uint32_t)P1, (uint32_t)P2, (uint32_t)g);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ inline u16x2 as2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t as1(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline u16x2 vmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ inline u16x2 vadds(u16x2 a, u16x2 b) { return __builtin_elementwise_add_sat(a, b); }

// Minimum of three packed u16 pairs in one v_pk_minimum3_f16.  Exact for
// halves below 0x7C00: those bit patterns are the non-negative finite f16
// values (zero, subnormals, normals), whose order is the order of the
// patterns read as unsigned integers, and a minimum returns one of its
// inputs unchanged.  f16 subnormals are not flushed in these kernels (the
// f16/f64 denormal mode keeps them), so small integers compare correctly.
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
__device__ inline u16x2 vmin3h(u16x2 a, u16x2 b, u16x2 c) {
    const h16x2 m = __builtin_elementwise_minimum(__builtin_elementwise_minimum(__builtin_bit_cast(h16x2, a),
                                                                                __builtin_bit_cast(h16x2, b)),
                                                  __builtin_bit_cast(h16x2, c));
    return __builtin_bit_cast(u16x2, m);
}

// DPP controls (GFX9 encoding).
constexpr int kDppQuadPerm1032 = 0xB1;
constexpr int kDppQuadPerm2301 = 0x4E;
constexpr int kDppRowShl1 = 0x101;   // lane i reads lane i+1 within a row of 16
constexpr int kDppRowShr1 = 0x111;   // lane i reads lane i-1 within a row of 16
constexpr int kDppWaveShl1 = 0x130;  // lane i reads lane i+1
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i-1
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowHalfMirror = 0x141;

// Lane q of a group receives lane q-1's (from_lower) or q+1's (from_upper)
// value; a lane without a source receives 0 (bound_ctrl), and group edges are
// overwritten by the caller's OR mask.
template <int G>
__device__ inline uint32_t from_lower(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, G == 16 ? kDppRowShr1 : kDppWaveShr1, 0xF, 0xF, true);
}
template <int G>
__device__ inline uint32_t from_upper(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, G == 16 ? kDppRowShl1 : kDppWaveShl1, 0xF, 0xF, true);
}

// Minimum over each group of G lanes; every lane of the group receives it.
// The butterfly inside a row of 16 uses DPP (folded into v_min_u32_dpp);
// groups spanning 2 or 4 rows combine rows with the gfx950 permlane swaps.
template <int G>
__device__ inline uint32_t group_min(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppQuadPerm1032, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppQuadPerm2301, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowHalfMirror, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowMirror, 0xF, 0xF, true));
    if constexpr (G >= 32) {
        const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = min((uint32_t)sw[0], (uint32_t)sw[1]);
    }
    if constexpr (G == 64) {
        const auto sw = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        v = min((uint32_t)sw[0], (uint32_t)sw[1]);
    }
    return v;
}

// Raw cost bytes of one lane for one step: CPL bytes.
template <int CPL> struct Raw;
template <> struct Raw<2> { using T = uint16_t; };
template <> struct Raw<4> { using T = uint32_t; };
template <> struct Raw<8> { using T = uint2; };
template <> struct Raw<16> { using T = uint4; };

// Unpacks a lane's cost bytes b_0..b_{CPL-1} into pairs (b_k, b_{k+CPL/2})
// with one v_perm per pair.  sel[k] is the per-lane byte selector; it selects
// 0xFF bytes for padded levels, which makes their cost 0xFFFF.
template <int CPL>
__device__ inline void unpack_costs(const typename Raw<CPL>::T& r, const uint32_t (&sel)[CPL / 2],
                                    u16x2 (&c)[CPL / 2]) {
    if constexpr (CPL == 2) {
        c[0] = as2(__builtin_amdgcn_perm(0u, (uint32_t)r, sel[0]));
    } else if constexpr (CPL == 4) {
        c[0] = as2(__builtin_amdgcn_perm(r, r, sel[0]));
        c[1] = as2(__builtin_amdgcn_perm(r, r, sel[1]));
    } else if constexpr (CPL == 8) {
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = as2(__builtin_amdgcn_perm(r.y, r.x, sel[k]));
    } else {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = as2(__builtin_amdgcn_perm(w[2 + k / 4], w[k / 4], sel[k]));
    }
}

// Selector of pair k for a lane whose first disparity is d0: low half b_k,
// high half b_{k+CPL/2} (bytes of the v_perm source pair), and the padding
// value `pad` (a 16-bit v_perm selector) for d >= D.
template <int CPL>
__device__ inline uint32_t unpack_selector(int k, int d0, int D, uint32_t pad) {
    constexpr int NP = CPL / 2;
    uint32_t lo, hi;
    if constexpr (CPL == 2) {
        lo = 0;
        hi = 1;
    } else if constexpr (CPL == 4) {
        lo = k;
        hi = k + 2;
    } else {
        lo = k % 4;
        hi = 4 + k % 4;
    }
    const uint32_t slo = (d0 + k < D) ? (lo | 0x0C00u) : pad;
    const uint32_t shi = (d0 + k + NP < D) ? (hi | 0x0C00u) : pad;
    return slo | (shi << 16);
}

enum { kHoriz = 0, kVert = 1, kDiag = 2 };

// Raw-buffer resource for a byte range (gfx9-family descriptor word 3).  Every
// access below passes its whole byte offset in the VGPR operand, so the
// hardware range check covers it: loads past `bytes` return 0 and stores past
// it are dropped.
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

template <int CPL>
__device__ inline typename Raw<CPL>::T buffer_load_raw(__amdgpu_buffer_rsrc_t r, uint32_t ofs) {
    if constexpr (CPL == 2) {
        return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, ofs, 0, 0);
    } else if constexpr (CPL == 4) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, ofs, 0, 0);
    } else if constexpr (CPL == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, ofs, 0, 0);
        return make_uint2(v[0], v[1]);
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, ofs, 0, 0);
        return make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// AUX is the cache-policy operand of the store (gfx950: 2 = non-temporal,
// 16 = device scope, sc1).
template <int AUX>
__device__ inline void buffer_store(__amdgpu_buffer_rsrc_t r, uint32_t ofs, uint16_t v) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, ofs, 0, AUX);
}
template <int AUX>
__device__ inline void buffer_store(__amdgpu_buffer_rsrc_t r, uint32_t ofs, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, ofs, 0, AUX);
}
template <int AUX>
__device__ inline void buffer_store(__amdgpu_buffer_rsrc_t r, uint32_t ofs, uint2 v) {
    __builtin_amdgcn_raw_buffer_store_b64((unsigned __attribute__((ext_vector_type(2)))){v.x, v.y}, r, ofs, 0, AUX);
}
template <int AUX>
__device__ inline void buffer_store(__amdgpu_buffer_rsrc_t r, uint32_t ofs, uint4 v) {
    __builtin_amdgcn_raw_buffer_store_b128((unsigned __attribute__((ext_vector_type(4)))){v.x, v.y, v.z, v.w}, r, ofs,
                                           0, AUX);
}

// A lane's CPL L values as bytes in natural disparity order (u8 planes):
// pair k holds disparities k and k + CPL/2 (split layout), so the bytes are
// gathered with v_perm.
template <int CPL>
__device__ inline typename Raw<CPL>::T pack_u8(const u16x2 (&l)[CPL / 2]) {
    constexpr uint32_t kLoBytes = 0x06020400u;  // (a.b0, b.b0, a.b2, b.b2) of perm(b, a)
    constexpr uint32_t kPairLo = 0x05040100u;   // (a.lo16, b.lo16)
    constexpr uint32_t kPairHi = 0x07060302u;   // (a.hi16, b.hi16)
    if constexpr (CPL == 2) {
        return (uint16_t)__builtin_amdgcn_perm(0u, as1(l[0]), 0x0C0C0200u);
    } else if constexpr (CPL == 4) {
        return (uint32_t)__builtin_amdgcn_perm(as1(l[1]), as1(l[0]), kLoBytes);
    } else if constexpr (CPL == 8) {
        const uint32_t t01 = __builtin_amdgcn_perm(as1(l[1]), as1(l[0]), kLoBytes);
        const uint32_t t23 = __builtin_amdgcn_perm(as1(l[3]), as1(l[2]), kLoBytes);
        return make_uint2(__builtin_amdgcn_perm(t23, t01, kPairLo), __builtin_amdgcn_perm(t23, t01, kPairHi));
    } else {
        uint32_t t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) t[i] = __builtin_amdgcn_perm(as1(l[2 * i + 1]), as1(l[2 * i]), kLoBytes);
        return make_uint4(__builtin_amdgcn_perm(t[1], t[0], kPairLo), __builtin_amdgcn_perm(t[3], t[2], kPairLo),
                          __builtin_amdgcn_perm(t[1], t[0], kPairHi), __builtin_amdgcn_perm(t[3], t[2], kPairHi));
    }
}

// Packs a lane's L values in natural disparity order (u8 or u16) and stores
// them at byte offset `ofs` of the L_r plane.  NT: non-temporal stores (the
// frame's planes exceed the memory-side cache); otherwise device-scope (sc1)
// stores, which measured faster than plain ones: the planes still reach the
// memory-side cache for the WTA, and the L2 keeps more of the cost lines
// that the opposite direction of a slice re-reads.
template <int CPL, typename LT, bool NT = false>
__device__ inline void store_l(__amdgpu_buffer_rsrc_t r, uint32_t ofs, const u16x2 (&l)[CPL / 2]) {
    constexpr int A = NT ? 2 : 16;
    constexpr uint32_t kPairLo = 0x05040100u;   // (a.lo16, b.lo16)
    constexpr uint32_t kPairHi = 0x07060302u;   // (a.hi16, b.hi16)
    if constexpr (sizeof(LT) == 1) {
        buffer_store<A>(r, ofs, pack_u8<CPL>(l));
    } else {
        constexpr int NP = CPL / 2;
        if constexpr (CPL == 2) {
            buffer_store<A>(r, ofs, as1(l[0]));
        } else {
            // dword i = (d_2i, d_2i+1) from pairs 2i and 2i+1 (low halves,
            // then high halves)
            uint32_t w[NP];
#pragma unroll
            for (int i = 0; i < NP / 2; ++i) {
                w[i] = __builtin_amdgcn_perm(as1(l[2 * i + 1]), as1(l[2 * i]), kPairLo);
                w[NP / 2 + i] = __builtin_amdgcn_perm(as1(l[2 * i + 1]), as1(l[2 * i]), kPairHi);
            }
            if constexpr (NP == 2) {
                buffer_store<A>(r, ofs, make_uint2(w[0], w[1]));
            } else {
#pragma unroll
                for (int i = 0; i < NP / 4; ++i)
                    buffer_store<A>(r, ofs + 16 * i, make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]));
            }
        }
    }
}

// Census words one lane needs for one step of the fused variant: the base
// word of its group's pixel and the CPL match words of columns x - d for its
// disparities d = q*CPL .. q*CPL + CPL - 1 (contiguous, lowest column first).
template <int CPL>
struct CensusStep {
    uint64_t base;
    uint64_t m[CPL];
};

template <int CPL>
__device__ inline void load_census(__amdgpu_buffer_rsrc_t rcl, __amdgpu_buffer_rsrc_t rcr, uint32_t base_ofs,
                                   uint32_t match_ofs, CensusStep<CPL>& cs) {
    const auto b = __builtin_amdgcn_raw_buffer_load_b64(rcl, base_ofs, 0, 0);
    cs.base = ((uint64_t)b[1] << 32) | b[0];
#pragma unroll
    for (int i = 0; i < CPL / 2; ++i) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rcr, match_ofs + 16 * i, 0, 0);
        cs.m[2 * i] = ((uint64_t)v[1] << 32) | v[0];
        cs.m[2 * i + 1] = ((uint64_t)v[3] << 32) | v[2];
    }
}

// Hamming costs (Eq. 2) of a lane's CPL disparities, packed as the u16 pairs
// of the split layout.  Cell c (disparity q*CPL + c) uses match word
// m[CPL - 1 - c]; cells with c > valid_c (x - d < 0) cost cmax.  sel[k] puts
// the costs of cells k and k + CPL/2 into the two halves of pair k, or 0xFFFF
// for padded levels.
template <int CPL, bool ALL_VALID>
__device__ inline void census_costs(const CensusStep<CPL>& cs, int valid_c, uint32_t cmax,
                                    const uint32_t (&sel)[CPL / 2], u16x2 (&c)[CPL / 2]) {
    constexpr int NP = CPL / 2;
    uint32_t pc[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        const uint64_t x = cs.base ^ cs.m[CPL - 1 - i];
        pc[i] = (uint32_t)__popcll(x);
        if constexpr (!ALL_VALID) pc[i] = i > valid_c ? cmax : pc[i];
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) c[k] = as2(__builtin_amdgcn_perm(pc[k + NP], pc[k], sel[k]));
}

// Selector of pair k for the fused variant: low half = cell k (S1 byte 0),
// high half = cell k + CPL/2 (S0 byte 0, selector 4); `pad` for d >= D.
template <int CPL>
__device__ inline uint32_t pack_selector(int k, int d0, int D, uint32_t pad) {
    constexpr int NP = CPL / 2;
    const uint32_t slo = (d0 + k < D) ? 0x0C00u : pad;
    const uint32_t shi = (d0 + k + NP < D) ? 0x0C04u : pad;
    return slo | (shi << 16);
}

// Cost loads run PF steps ahead of the recurrence so that their latency
// overlaps the dependent min-plus chain of the steps in between.
template <int CPL> struct Prefetch { static constexpr int N = CPL >= 16 ? 8 : 16; };
template <int CPL> struct FusedPrefetch { static constexpr int N = CPL >= 16 ? 2 : 4; };

// Where aggregate_wave puts each step's L values: by default the direction's
// L_r plane in global memory.  A sink (the final pass's LDS ring) instead
// receives put(step, L) for every step and chunk_done() after every Prefetch
// steps and after the last step.
struct PlaneSink {};

// ADAPT: the P2 of each step adapts to the base image's intensity change
// along the path (adaptive_p2); the intensities are prefetched with the costs.
template <int G, int CPL, typename LT, int KIND, bool FUSED, bool ADAPT = false, bool NT = false,
          typename SINK = PlaneSink>
__device__ inline void aggregate_wave(const SliceArgs& a, int first_slice, int lane, SINK* sink = nullptr) {
    constexpr bool kToPlane = std::is_same_v<SINK, PlaneSink>;
    static_assert(!(FUSED && ADAPT), "adaptive P2 uses the cost-volume variant");
    constexpr int NP = CPL / 2;
    constexpr int Dp = G * CPL;
    constexpr int kDpShift = Dp == 64 ? 6 : (Dp == 128 ? 7 : 8);
    constexpr int PF = FUSED ? FusedPrefetch<CPL>::N : Prefetch<CPL>::N;
    // per-step input: raw cost bytes, or census words (fused variant)
    using RawT = std::conditional_t<FUSED, CensusStep<CPL>, typename Raw<CPL>::T>;

    const int rx = a.rx, ry = a.ry;
    const int W = a.W, H = a.H;
    const int grp = lane / G, q = lane % G;
    const int nslices = KIND == kHoriz ? H : W;
    const int steps = KIND == kHoriz ? W : H;
    // groups past the last slice repeat the last slice (identical stores)
    const int jg = min(grp, nslices - 1 - first_slice);

    // Byte planes (Cmax + largest step penalty <= 255) keep every register
    // value far below 0x7C00, so the minimum of three runs as one packed f16
    // minimum (vmin3h).  That needs finite stand-ins for "no candidate":
    //   * padded levels d >= D get cost 255 (not 0xFFFF).  Their L stays in
    //     [255, 255 + P2] and never undercuts a real level: real L <= Cmax +
    //     P2 <= 255, and the path minimum m is at most Cmax, so m + P2 <=
    //     255 <= L(pad) + P1.
    //   * the d - 1 / d + 1 candidate beyond the lane group's ends is 0x0FFF
    //     (OR-ed into a value below 0x1000), above every real candidate.
    //   * P1 is capped at the largest step penalty: a larger P1 never wins
    //     against m + P2 in Eq. 3 (L(d +- 1) >= m), and neither does the cap.
    // 16-bit planes keep saturating u16 arithmetic with 0xFFFF.
    constexpr bool kF16 = sizeof(LT) == 1;
    const uint32_t pad = kF16 ? 0x0C0Du : 0x0D0Du;  // v_perm bytes: 0x00FF or 0xFFFF
    uint32_t sel[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k)
        sel[k] = FUSED ? pack_selector<CPL>(k, q * CPL, a.D, pad) : unpack_selector<CPL>(k, q * CPL, a.D, pad);
    const uint32_t inf = kF16 ? 0x0FFFu : 0xFFFFu;
    const uint32_t edge_lo = q == 0 ? inf << 16 : 0u;  // no d-1 below d = 0
    const uint32_t edge_hi = q == G - 1 ? inf : 0u;    // no d+1 above Dp-1
    const uint32_t P1c = kF16 ? (uint32_t)(ADAPT ? a.P1 : min(a.P1, a.P2)) : (uint32_t)a.P1;
    const u16x2 P1v = as2(P1c * 0x10001u), P2v = as2((uint32_t)a.P2 * 0x10001u);

    const uint32_t plane_bytes = (uint32_t)a.plane;  // cost plane, u8
    const __amdgpu_buffer_rsrc_t rc = buffer_rsrc(a.cost, FUSED ? 0u : plane_bytes);
    // the match buffer starts kCensusGuard words early: a lane's window of
    // CPL words may begin left of column 0 (those words are never used)
    const uint32_t census_bytes = 8u * (uint32_t)W * (uint32_t)H;
    const __amdgpu_buffer_rsrc_t rcl = buffer_rsrc(a.census_l, FUSED ? census_bytes : 0u);
    const __amdgpu_buffer_rsrc_t rcr =
        buffer_rsrc(a.census_r - kCensusGuard, FUSED ? census_bytes + 8u * kCensusGuard : 0u);
    const __amdgpu_buffer_rsrc_t rl = buffer_rsrc(a.lplane, plane_bytes * (uint32_t)sizeof(LT));
    const __amdgpu_buffer_rsrc_t rim = buffer_rsrc(a.img, ADAPT ? (uint32_t)W * (uint32_t)H : 0u);

    // Group 0's position: byte offset `bo` of its pixel in a u8 [H][W][Dp]
    // plane and, for diagonal slices, its column xc (kept in [0, W)).
    int bo, xc;
    if constexpr (KIND == kHoriz) {
        xc = rx > 0 ? 0 : W - 1;
        bo = (first_slice * W + xc) * Dp;
    } else {
        xc = first_slice;
        bo = ((ry > 0 ? 0 : H - 1) * W + xc) * Dp;
    }
    const int bstep = (KIND == kHoriz ? rx : ry * W + (KIND == kDiag ? rx : 0)) * Dp;
    const int qofs = q * CPL;
    // byte offset of the lane relative to group 0 (horizontal: rows below;
    // vertical: columns to the right; diagonal: columns to the right, or
    // W - jg columns to the left once the group's column has wrapped)
    const int lofs = (KIND == kHoriz ? jg * W : jg) * Dp + qofs;
    const int lofs_wrapped = (jg - W) * Dp + qofs;
    auto lane_ofs = [&](int b, int x) -> uint32_t {
        if constexpr (KIND == kDiag) return (uint32_t)(b + (x + jg >= W ? lofs_wrapped : lofs));
        return (uint32_t)(b + lofs);
    };
    auto advance = [&](int& b, int& x) {
        b += bstep;
        if constexpr (KIND == kHoriz) x += rx;
        if constexpr (KIND == kDiag) {
            x += rx;
            const int under = x >> 31;             // -1 if x < 0
            const int over = (W - 1 - x) >> 31;    // -1 if x >= W
            const int wrap = (under & W) - (over & W);
            x += wrap;
            b += wrap * Dp;
        }
    };

    u16x2 L[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) L[k] = as2(0u);
    u16x2 mm = as2(0u);
    // restart column of a diagonal group: where it crosses the side border
    const int border = rx > 0 ? 0 : W - 1;

    // smallest column any group of the wavefront is at (uniform): when it is
    // >= Dp - 1, every lane's disparities are valid (x - d >= 0)
    int xmin_all = 0;
    // ADAPT: this step's P2 (looked up during the previous step; at a path
    // start L and mm are 0 and the P2 of that step does not matter)
    uint32_t p2cur = (uint32_t)a.P2;
    auto step = [&](const RawT& raw, uint32_t iv, uint32_t inext, int t) {
        if constexpr (FUSED) {
            if constexpr (KIND == kHoriz)
                xmin_all = xc;
            else if constexpr (KIND == kVert)
                xmin_all = xc;
            else
                xmin_all = xc + 64 / G - 1 >= W ? 0 : xc;  // a wrapped group sits at a small column
        }
        if constexpr (KIND == kDiag) {
            const int xl = xc + jg >= W ? xc + jg - W : xc + jg;
            if (xl == border) {
#pragma unroll
                for (int k = 0; k < NP; ++k) L[k] = as2(0u);
                mm = as2(0u);
            }
        }
        u16x2 c[NP];
        if constexpr (FUSED) {
            // the lane's disparities are valid (x - d >= 0) for cells
            // c <= x - q*CPL; x of the lane's group is group 0's column + jg
            // (horizontal: same column; diagonal: wrapped)
            int xg;
            if constexpr (KIND == kHoriz)
                xg = xc;
            else if constexpr (KIND == kVert)
                xg = xc + jg;
            else
                xg = xc + jg >= W ? xc + jg - W : xc + jg;
            const int valid_c = xg - q * CPL;
            if (xmin_all >= Dp - 1)
                census_costs<CPL, true>(raw, valid_c, (uint32_t)a.cmax, sel, c);
            else
                census_costs<CPL, false>(raw, valid_c, (uint32_t)a.cmax, sel, c);
        } else {
            unpack_costs<CPL>(raw, sel, c);
        }
        u16x2 lp[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) lp[k] = vadds(L[k], P1v);
        const uint32_t prev = from_lower<G>(as1(lp[NP - 1])) | edge_lo;
        const uint32_t next = from_upper<G>(as1(lp[0])) | edge_hi;
        const u16x2 lo0 = as2(__builtin_amdgcn_alignbit(as1(lp[NP - 1]), prev, 16));
        const u16x2 hiN = as2(__builtin_amdgcn_alignbit(next, as1(lp[0]), 16));
        u16x2 p2v = P2v;
        uint32_t p2next = 0;
        if constexpr (ADAPT) {
            p2v = as2(p2cur * 0x10001u);
            // the next step's P2, from the intensity change to the next pixel;
            // the LDS read completes while this step runs
            const uint32_t g = inext > iv ? inext - iv : iv - inext;
            p2next = a.p2lut[g];
        }
        const u16x2 mp2 = vadds(mm, p2v);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const u16x2 lo = k == 0 ? lo0 : lp[k - 1];
            const u16x2 hi = k == NP - 1 ? hiN : lp[k + 1];
            const u16x2 R = kF16 ? vmin(vmin3h(lo, hi, L[k]), mp2) : vmin(vmin(lo, hi), vmin(L[k], mp2));
            L[k] = vadds(R - mm, c[k]);
        }
        // minimum over the lane's cells, replicated in both halves
        u16x2 tm;
        if constexpr (kF16 && NP >= 4) {
            u16x2 t = vmin3h(L[0], L[1], L[2]);
#pragma unroll
            for (int k = 3; k + 1 < NP; k += 2) t = vmin3h(t, L[k], L[k + 1]);
            if constexpr (NP % 2 == 0) t = vmin(t, L[NP - 1]);
            tm = vmin(t, t.yx);
        } else {
            u16x2 t[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) t[k] = L[k];
#pragma unroll
            for (int w = 1; w < NP; w *= 2)
#pragma unroll
                for (int k = 0; k + w < NP; k += 2 * w) t[k] = vmin(t[k], t[k + w]);
            tm = vmin(t[0], t[0].yx);
        }
        mm = as2(group_min<G>(as1(tm)));
        if constexpr (kToPlane)
            store_l<CPL, LT, NT>(rl, lane_ofs(bo, xc) * (uint32_t)sizeof(LT), L);
        else
            sink->put(t, L);
        advance(bo, xc);
        if constexpr (ADAPT) p2cur = p2next;
    };

    // ring[j] holds the raw costs of the step congruent to j modulo PF.  The
    // lookahead position leads by PF - 1 steps and runs past the slice's end
    // near the finish; those loads are never consumed (and past the plane
    // they return 0).
    auto load = [&](int b, int x) -> RawT {
        if constexpr (FUSED) {
            // pixel index of the lane's group: byte offset / Dp, with the
            // lane's disparity offset qofs removed
            const int pix = (int)((lane_ofs(b, x) - (uint32_t)qofs) / (uint32_t)Dp);
            RawT cs;
            load_census<CPL>(rcl, rcr, 8u * (uint32_t)pix,
                             8u * (uint32_t)(pix + kCensusGuard - qofs - (CPL - 1)), cs);
            return cs;
        } else {
            return buffer_load_raw<CPL>(rc, lane_ofs(b, x));
        }
    };
    // intensity of the lane's group pixel (ADAPT): pixel index = (byte
    // offset - qofs) / Dp; past the image the range check returns 0
    auto load_i = [&](int b, int x) -> uint32_t {
        if constexpr (ADAPT)
            return __builtin_amdgcn_raw_buffer_load_b8(rim, (lane_ofs(b, x) - (uint32_t)qofs) >> kDpShift, 0, 0);
        else
            return 0u;
    };
    RawT ring[PF];
    uint32_t iring[ADAPT ? PF : 1];
    int ba = bo, xa = xc;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        if (j) advance(ba, xa);
        ring[j] = load(ba, xa);
        if constexpr (ADAPT) iring[j] = load_i(ba, xa);
    }
    int k = 0;
    for (; k + PF <= steps; k += PF) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const RawT raw = ring[j];
            // slot j + 1 (mod PF) holds the next step's intensity: slot 0 was
            // refilled with step k + PF at j = 0
            const uint32_t iv = ADAPT ? iring[ADAPT ? j : 0] : 0u;
            advance(ba, xa);
            ring[j] = load(ba, xa);
            if constexpr (ADAPT) iring[j] = load_i(ba, xa);
            step(raw, iv, ADAPT ? iring[ADAPT ? (j + 1) % PF : 0] : 0u, k + j);
        }
        if constexpr (!kToPlane) sink->chunk_done();
    }
#pragma unroll
    for (int j = 0; j < PF; ++j)
        if (k + j < steps)
            step(ring[j], ADAPT ? iring[ADAPT ? j : 0] : 0u, ADAPT ? iring[ADAPT ? (j + 1) % PF : 0] : 0u, k + j);
    if constexpr (!kToPlane)
        if (k < steps) sink->chunk_done();
}

// ---------------------------------------------------------------------------
// Sum over directions and winner-take-all (Eq. 4), one block per row.
// Lane = pixel: each lane walks its pixel's disparities in runs of 16, sums
// the planes as packed u16 pairs and forms keys (S << 8) | d with one v_perm
// per cell (padded levels get a 0xFF top byte, so they never win).  The left
// disparity is the smallest key of the pixel.  The right view: pixel x at
// disparity d is right pixel x - d, so every (x, d) offers its key to column
// x - d with an LDS atomic minimum; the lanes of a wavefront hit consecutive
// words, and targets x - d < 0 land in a guard region in front of the row.
// The column's winner is argmin_d S(x + d, d), ties to the smallest d.
// ---------------------------------------------------------------------------
// The post stage (3x3 median of both maps, then the left-right check) of
// one pair, read by post_row.
struct PostArgs {
    const uint16_t* dl;
    const uint16_t* dr;
    uint16_t* out;
    int W, H, median, lrcheck, thr;
    int subpixel = 0;  // dl in 1/16 pixel: the check uses its rounding
};

struct WtaArgs {
    const void* lbuf;
    size_t plane;
    uint16_t* dl;  // left disparity (raw, or the final output)
    uint16_t* dr;  // right disparity or nullptr
    int W, H, D, Dp, nplanes;
    int subpixel = 0;  // dl in 1/16 pixel: parabola vertex through S(d-1), S(d), S(d+1)
    // The post stage run inside the WTA launch (rowcnt != nullptr): per-row
    // counters (zeroed by the census launch of the same frame), `contrib`
    // blocks writing raw rows per image row (2 when one launch makes D_L and
    // D_R with separate blocks), and the post stage's arguments.
    int* rowcnt = nullptr;
    int contrib = 1;
    PostArgs post{};
};

// floor(num / den) for den > 0
__device__ inline int floor_div(int num, int den) {
    const int q = num / den;
    return (num % den != 0 && num < 0) ? q - 1 : q;
}

constexpr int kWtaGuard = 256;  // >= max disparity

// Sums of 16 disparities d0..d0+15 of one pixel over NPL planes as 8 packed
// pairs; pair k holds disparities dpair(k) (see below).  Every plane's load
// is issued before the first add, so a lane has all NPL loads in flight.
// NT: the loads are non-temporal (planes that did not fit the memory-side
// cache are streamed once).
template <bool NT>
__device__ inline uint4 load16(const void* p) {
    typedef unsigned v4 __attribute__((ext_vector_type(4)));
    if constexpr (NT) {
        const v4 t = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
        return make_uint4(t.x, t.y, t.z, t.w);
    } else {
        return *reinterpret_cast<const uint4*>(p);
    }
}

template <typename LT, int NPL, bool NT>
__device__ inline void sum16(const LT* base, size_t plane, uint32_t (&S)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) S[k] = 0;
    if constexpr (sizeof(LT) == 1) {
        // bytes b0..b3 of dword i -> pairs (b0, b2) and (b1, b3)
        uint4 q[NPL];
#pragma unroll
        for (int p = 0; p < NPL; ++p) q[p] = load16<NT>(base + plane * p);
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            const uint32_t w[4] = {q[p].x, q[p].y, q[p].z, q[p].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                S[2 * i] = as1(as2(S[2 * i]) + as2(__builtin_amdgcn_perm(0u, w[i], 0x0C020C00u)));
                S[2 * i + 1] = as1(as2(S[2 * i + 1]) + as2(__builtin_amdgcn_perm(0u, w[i], 0x0C030C01u)));
            }
        }
    } else {
        // u16 pairs are already (d, d + 1)
        uint4 q[NPL][2];
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            q[p][0] = load16<NT>(base + plane * p);
            q[p][1] = load16<NT>(base + plane * p + 8);
        }
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            const uint32_t w[8] = {q[p][0].x, q[p][0].y, q[p][0].z, q[p][0].w,
                                   q[p][1].x, q[p][1].y, q[p][1].z, q[p][1].w};
#pragma unroll
            for (int k = 0; k < 8; ++k) S[k] = as1(as2(S[k]) + as2(w[k]));
        }
    }
}

// Disparities (relative to the run) held by pair k: u8 planes pair 2i =
// (4i, 4i + 2), pair 2i + 1 = (4i + 1, 4i + 3); u16 planes pair k = (2k, 2k+1).
template <typename LT>
__device__ inline void pair_disps(int k, int& lo, int& hi) {
    if constexpr (sizeof(LT) == 1) {
        lo = 4 * (k >> 1) + (k & 1);
        hi = lo + 2;
    } else {
        lo = 2 * k;
        hi = lo + 1;
    }
}

// Minimum over aligned groups of G consecutive lanes (G = 4, 8 or 16);
// every lane of the group receives it.
__device__ inline uint32_t lanes_min(uint32_t v, int G) {
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppQuadPerm1032, 0xF, 0xF, true));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppQuadPerm2301, 0xF, 0xF, true));
    if (G >= 8) v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowHalfMirror, 0xF, 0xF, true));
    if (G >= 16) v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowMirror, 0xF, 0xF, true));
    return v;
}

// The winner-take-all of one lane's 16 disparities d0 .. d0+15 of pixel
// (x, y), given their summed costs S (pairs as pair_disps<LT>): keys
// (S << 8) | d with a 0xFF top byte for padded levels; the pixel's smallest
// key over its G lanes (consecutive, aligned) is D_L (1/16-pixel vertex with
// sub-pixel output); with `right`, every (x, d) offers its key to column
// x - d of the row's right-view keys (LDS, atomic minimum; targets x - d < 0
// land in a guard region in front of the row).  s_out (debug): S u16
// [H][W][D].
template <typename LT>
__device__ inline void wta_cells(const WtaArgs& a, int y, int x, int g, int G, const uint32_t (&S)[8],
                                 uint32_t* keyR, bool right, uint16_t* s_out = nullptr, bool valid = true) {
    right = right && valid;
    if (!valid) s_out = nullptr;
    const int d0 = 16 * g;
    uint32_t best = ~0u;
    // right-view targets x - d0 - 15 .. x - d0 from one base address
    uint32_t* tgt = keyR + (x - d0 - 15);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int dlo, dhi;
        pair_disps<LT>(k, dlo, dhi);
        const uint32_t dpair = (uint32_t)(d0 + dlo) | ((uint32_t)(d0 + dhi) << 8);
        // key = [d, S.lo16, 0] with a 0xFF top byte for padded levels
        const uint32_t klo = __builtin_amdgcn_perm(S[k], dpair, d0 + dlo < a.D ? 0x0C050400u : 0x0D050400u);
        const uint32_t khi = __builtin_amdgcn_perm(S[k], dpair, d0 + dhi < a.D ? 0x0C070601u : 0x0D070601u);
        best = min(best, min(klo, khi));
        if (right) {
            if (d0 + dlo < a.D) atomicMin(tgt + (15 - dlo), klo);
            if (d0 + dhi < a.D) atomicMin(tgt + (15 - dhi), khi);
        }
        if (s_out) {
            uint16_t* o = s_out + ((size_t)y * a.W + x) * a.D;
            if (d0 + dlo < a.D) o[d0 + dlo] = (uint16_t)(S[k] & 0xFFFFu);
            if (d0 + dhi < a.D) o[d0 + dhi] = (uint16_t)(S[k] >> 16);
        }
    }
    best = lanes_min(best, G);
    const int dbest = (int)(best & 0xFF);
    uint32_t outv = (uint32_t)dbest;
    if (a.subpixel) {
        // S(dbest - 1) and S(dbest + 1) from the lanes holding them; the
        // vertex of the parabola through the three, rounded half up to
        // 1/16: f = floor((16 (a - c) + den) / (2 den)), den = a + c - 2b
        uint32_t va = ~0u, vc = ~0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int dlo, dhi;
            pair_disps<LT>(k, dlo, dhi);
            const uint32_t slo = S[k] & 0xFFFFu, shi = S[k] >> 16;
            if (d0 + dlo == dbest - 1) va = slo;
            if (d0 + dhi == dbest - 1) va = shi;
            if (d0 + dlo == dbest + 1) vc = slo;
            if (d0 + dhi == dbest + 1) vc = shi;
        }
        va = lanes_min(va, G);
        vc = lanes_min(vc, G);
        int f = 0;
        if (dbest > 0 && dbest < a.D - 1) {
            const int b = (int)((best >> 8) & 0xFFFFu);
            const int den = (int)va + (int)vc - 2 * b;
            if (den > 0) f = floor_div(16 * ((int)va - (int)vc) + den, 2 * den);
        }
        outv = (uint32_t)(16 * dbest + f);
    }
    if (g == 0 && valid) a.dl[(size_t)y * a.W + x] = (uint16_t)outv;
}

__device__ inline void wta_fold_post(const WtaArgs& a, int y, uint16_t* rview);

template <typename LT, int NPL, bool NT, bool FOLD>
__device__ inline void wta_row_impl(const WtaArgs& a, int y, uint32_t* keyR_smem) {
    uint32_t* keyR = keyR_smem + kWtaGuard;  // keyR[t], t in [-kWtaGuard, W)
    const bool right = a.dr != nullptr;
    if (right)
        for (int i = threadIdx.x; i < a.W + kWtaGuard; i += blockDim.x) keyR_smem[i] = ~0u;
    __syncthreads();
    const LT* planes = reinterpret_cast<const LT*>(a.lbuf);
    // thread (x, g) takes disparities 16g .. 16g + 15 of pixel x; the G runs
    // of a pixel sit on consecutive lanes, so its loads are contiguous
    const int G = a.Dp >> 4;
    const int gshift = G == 4 ? 2 : (G == 8 ? 3 : 4);
    for (int i = threadIdx.x; i < a.W * G; i += blockDim.x) {
        const int x = i >> gshift, g = i & (G - 1);
        uint32_t S[8];
        sum16<LT, NPL, NT>(planes + ((size_t)y * a.W + x) * a.Dp + 16 * g, a.plane, S);
        wta_cells<LT>(a, y, x, g, G, S, keyR, right);
    }
    if (right) {
        __syncthreads();
        for (int i = threadIdx.x; i < a.W; i += blockDim.x)
            a.dr[(size_t)y * a.W + i] = (uint16_t)(keyR[i] & 0xFF);
    }
    if constexpr (FOLD) wta_fold_post(a, y, reinterpret_cast<uint16_t*>(keyR_smem));
}

// One row of the WTA; the plane count (2, 4 or 8) is a template constant of
// the row's code, so the plane loads unroll.  NT: non-temporal plane loads,
// for planes that exceed the memory-side cache and were stored
// non-temporally.  FOLD: the post stage runs inside the launch (a.rowcnt
// set; wta_fold_post), a separate instantiation so that the plain kernel
// keeps its registers.
template <typename LT, bool NT = false, bool FOLD = false>
__device__ inline void wta_row(const WtaArgs& a, int y, uint32_t* keyR_smem) {
    if (a.nplanes == 2)
        wta_row_impl<LT, 2, NT, FOLD>(a, y, keyR_smem);
    else if (a.nplanes == 4)
        wta_row_impl<LT, 4, NT, FOLD>(a, y, keyR_smem);
    else
        wta_row_impl<LT, 8, NT, FOLD>(a, y, keyR_smem);
}

// ---------------------------------------------------------------------------
// Final pass: the last path direction fused with the sum over directions and
// the winner-take-all (Sec. 3.3), so that direction's L_r plane is never
// written to memory nor read back.  The fused direction is horizontal
// (right-to-left; left-to-right in the 2-path set): the right-view keys need
// whole rows, and a row is the slice of a horizontal direction.
//
// A block has 4 wavefronts, one per SIMD of its CU, in two roles:
//   * 2 producer waves run the recurrence of Eq. 3 along their rows (G = 64
//     lanes per row, 32 when Dp = 64, so a lane holds CPL = Dp / G = 2 or 4
//     disparities) exactly as aggregate_wave does, but put each step's L
//     values into an LDS ring of two chunks of K steps (K = the cost
//     prefetch depth) instead of a plane, and wait at a block barrier after
//     every chunk.  Each recurrence is a dependent chain issued at one
//     instruction per cycle slot of its SIMD, so no other producer shares
//     that SIMD;
//   * 2 consumer waves take chunk c after the barrier that completes it,
//     while the producers work on chunk c + 1.  A chunk has K * R * Dp / 16
//     (pixel, run of 16 disparities) items, M per consumer lane: each adds
//     the P - 1 planes stored by the aggregation launch and the chunk's L
//     values, and runs wta_cells.  The stored planes do not depend on the
//     producers, so a lane loads its items' plane bytes FinalAhead chunks
//     before it needs them (registers), which keeps the memory latency off
//     the per-chunk barrier interval.
// All waves pass the same number of barriers (one after the right-view key
// initialisation, one per chunk, one at the end), after which the block
// writes the right view of its rows from the LDS keys.
// ---------------------------------------------------------------------------
struct FinalArgs {
    SliceArgs agg;          // the fused direction: cost volume, rx = +-1, ry = 0
    const uint8_t* planes;  // the other P - 1 directions' u8 planes, contiguous
    size_t plane;           // bytes per plane (W * H * Dp)
    WtaArgs wta;            // outputs D_L (dl) and D_R (dr, or nullptr), W, H, D, Dp
    uint16_t* s_out;        // debug: S u16 [H][W][D], or nullptr
};

constexpr int kFinalThreads = 256;  // 2 producer + 2 consumer waves

template <int Dp>
struct FinalLayout {
    static constexpr int G = Dp == 64 ? 32 : 64;  // lanes per row
    static constexpr int CPL = Dp / G;             // disparities per lane: 2 or 4
    static constexpr int K = Prefetch<CPL>::N;     // steps per chunk
    static constexpr int NPROD = 2, NC = 2;        // producer and consumer waves
    static constexpr int RW = 64 / G;              // rows per producer wave
    static constexpr int R = NPROD * RW;           // rows per block
    static constexpr int ITEMS = K * R * (Dp / 16);
    static constexpr int M = ITEMS / (64 * NC);    // items per consumer lane and chunk
    static constexpr int ring_bytes = 2 * K * R * Dp;
    static_assert(M * 64 * NC == ITEMS, "whole items per consumer lane");
};

// Rows per final-pass block and its LDS bytes (ring, then the rows' right-
// view keys).
__host__ __device__ inline int final_rows(int Dp) { return Dp == 64 ? 4 : 2; }
__host__ __device__ inline size_t final_smem_bytes(int Dp, int W, bool right) {
    const int R = final_rows(Dp);
    return (size_t)2 * 16 * R * Dp + (right ? (size_t)4 * R * (W + kWtaGuard) : 0);
}

// Chunks of plane loads a consumer lane keeps in flight, within about 64
// registers: 4 * M * NPL registers per chunk.
template <int M, int NPL>
struct FinalAhead {
    static constexpr int n = 16 / (M * NPL);
    static constexpr int N = n < 1 ? 1 : (n > 3 ? 3 : n);
};

// A producer's sink: step t's L values of row slot `row` go to
// ring[(t / K) % 2][t % K][row][Dp] as bytes in disparity order.
template <int Dp>
struct LdsRingSink {
    uint8_t* ring;
    int row, q;
    __device__ void put(int t, const u16x2 (&l)[FinalLayout<Dp>::CPL / 2]) {
        using L = FinalLayout<Dp>;
        const int buf = (t / L::K) & 1, j = t % L::K;
        auto* dst = reinterpret_cast<typename Raw<L::CPL>::T*>(ring + ((buf * L::K + j) * L::R + row) * Dp + q * L::CPL);
        *dst = pack_u8<L::CPL>(l);
    }
    __device__ void chunk_done() { __syncthreads(); }
};

// Consumer item i of chunk c: pixel (x, y) and its run g, or invalid past
// the row's end or the image's last row (the same for the pixel's Dp / 16
// lanes).
template <int Dp>
struct FinalItem {
    int j, row, g, x, y;
    bool valid;
    __device__ FinalItem(const FinalArgs& f, int y0, int c, int i) {
        using L = FinalLayout<Dp>;
        constexpr int Gp = Dp / 16;
        g = i % Gp;
        const int pix = i / Gp;
        j = pix % L::K;
        row = pix / L::K;
        const int t = c * L::K + j;
        y = y0 + row;
        valid = t < f.wta.W && y < f.wta.H;
        x = f.agg.rx < 0 ? f.wta.W - 1 - t : t;
    }
};

// Plane bytes of an item: one range-checked buffer load per plane, with the
// byte offset of an invalid item past the plane's end (the hardware returns
// zeros), so no branch surrounds a load and the loads of later chunks stay
// in flight while earlier ones are used.  NT: non-temporal (planes that
// exceed the memory-side cache).
template <int NPL, bool NT>
__device__ inline void load_planes16(const __amdgpu_buffer_rsrc_t (&rp)[NPL], uint32_t ofs, uint4 (&q)[NPL]) {
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rp[p], ofs, 0, NT ? 2 : 0);
        q[p] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

template <int Dp>
__device__ inline uint32_t final_item_offset(const FinalArgs& f, const FinalItem<Dp>& it) {
    return it.valid ? (uint32_t)(((size_t)it.y * f.wta.W + it.x) * Dp + 16 * it.g) : 0xFFFFFFF0u;
}

// One item of a chunk: every lane runs it (invalid items only skip the
// stores and key updates inside wta_cells).
template <int Dp, int NPL>
__device__ inline void final_item_finish(const FinalArgs& f, const FinalItem<Dp>& it, int buf, const uint8_t* ring,
                                         uint32_t* keyR, const uint4 (&q)[NPL]) {
    using L = FinalLayout<Dp>;
    uint32_t S[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) S[k] = 0;
    auto add = [&](const uint4& v) {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            S[2 * k] = as1(as2(S[2 * k]) + as2(__builtin_amdgcn_perm(0u, w[k], 0x0C020C00u)));
            S[2 * k + 1] = as1(as2(S[2 * k + 1]) + as2(__builtin_amdgcn_perm(0u, w[k], 0x0C030C01u)));
        }
    };
#pragma unroll
    for (int p = 0; p < NPL; ++p) add(q[p]);
    add(*reinterpret_cast<const uint4*>(ring + ((buf * L::K + it.j) * L::R + it.row) * Dp + 16 * it.g));
    const int W = f.wta.W;
    wta_cells<uint8_t>(f.wta, it.y, it.x, it.g, Dp / 16, S, keyR + it.row * (W + kWtaGuard) + kWtaGuard,
                       f.wta.dr != nullptr, f.s_out, it.valid);
}

template <int Dp, int NPL, bool NT>
__device__ inline void final_pass_block(const FinalArgs& f, int blk, uint8_t* smem) {
    using L = FinalLayout<Dp>;
    const int W = f.wta.W, H = f.wta.H;
    const int y0 = blk * L::R;
    uint8_t* ring = smem;
    uint32_t* keyR = reinterpret_cast<uint32_t*>(smem + L::ring_bytes);
    const bool right = f.wta.dr != nullptr;
    const int kpitch = W + kWtaGuard;
    if (right)
        for (int i = threadIdx.x; i < L::R * kpitch; i += blockDim.x) keyR[i] = ~0u;
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (wave < L::NPROD) {
        // rows y0 + wave * RW .. (a row past the image repeats the last row;
        // the consumers skip it)
        LdsRingSink<Dp> sink{ring, wave * L::RW + lane / L::G, lane % L::G};
        aggregate_wave<L::G, L::CPL, uint8_t, kHoriz, false, false, false, LdsRingSink<Dp>>(
            f.agg, min(y0 + wave * L::RW, H - 1), lane, &sink);
    } else {
        const int ctid = (wave - L::NPROD) * 64 + lane;
        const int nchunks = (W + L::K - 1) / L::K;
        __amdgpu_buffer_rsrc_t rp[NPL];
#pragma unroll
        for (int p = 0; p < NPL; ++p) rp[p] = buffer_rsrc(f.planes + f.plane * p, (uint32_t)f.plane);
        constexpr int A = FinalAhead<L::M, NPL>::N;
        // plane bytes of the lane's M items of chunks c .. c + A - 1, slot c % A
        uint4 q[A][L::M][NPL];
        auto item = [&](int c, int m) { return FinalItem<Dp>(f, y0, c, ctid + m * 64 * L::NC); };
#pragma unroll
        for (int s = 0; s < A; ++s)
#pragma unroll
            for (int m = 0; m < L::M; ++m) load_planes16<NPL, NT>(rp, final_item_offset<Dp>(f, item(s, m)), q[s][m]);
        auto chunk = [&](int c, uint4 (&qs)[L::M][NPL]) {
            __syncthreads();  // chunk c is in the ring
#pragma unroll
            for (int m = 0; m < L::M; ++m) final_item_finish<Dp, NPL>(f, item(c, m), c & 1, ring, keyR, qs[m]);
#pragma unroll
            for (int m = 0; m < L::M; ++m) load_planes16<NPL, NT>(rp, final_item_offset<Dp>(f, item(c + A, m)), qs[m]);
        };
        int c0 = 0;
        for (; c0 + A <= nchunks; c0 += A) {
#pragma unroll
            for (int s = 0; s < A; ++s) chunk(c0 + s, q[s]);
        }
#pragma unroll
        for (int s = 0; s < A; ++s)
            if (c0 + s < nchunks) chunk(c0 + s, q[s]);  // the same for every consumer wave
    }
    __syncthreads();
    if (right) {
        for (int row = 0; row < L::R && y0 + row < H; ++row)
            for (int i = threadIdx.x; i < W; i += blockDim.x)
                f.wta.dr[(size_t)(y0 + row) * W + i] = (uint16_t)(keyR[row * kpitch + kWtaGuard + i] & 0xFF);
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

// One row of the post stage.  Each thread takes 4 columns per pass so that
// the neighbour loads of a pass are in flight together (a 640-wide row is
// one pass of a 256-thread block); the median and check switches are
// template constants, so no branch splits those loads.  With the check on,
// the first pass loads the D_L and D_R neighbourhoods together (72 loads),
// so the two maps' load latencies overlap; the D_R medians of the whole row
// go to LDS before the barrier, and the check after it reads them at x - d.
template <bool LR, bool MED>
__device__ inline void post_row_impl(const PostArgs& a, int y, uint16_t* rview) {
    constexpr int U = 4;
    const int nt = blockDim.x, x0 = threadIdx.x;
    auto med = [&](const uint16_t* img, int x) -> uint32_t {
        if constexpr (MED)
            return median9(img, a.W, a.H, x, y);
        else
            return img[(size_t)y * a.W + x];
    };
    auto finish = [&](int x, int v) {
        if (x >= a.W) return;
        int o = v;
        if constexpr (LR) {
            const int d = a.subpixel ? (v + 8) >> 4 : v;  // integer disparity of the check
            o = kInvalid;
            if (x - d >= 0) {
                const int e = rview[x - d];
                if (abs(d - e) <= a.thr) o = v;
            }
        }
        a.out[(size_t)y * a.W + x] = (uint16_t)o;
    };
    // first pass: columns x0 + u * nt
    uint32_t dv[U], rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int x = min(x0 + u * nt, a.W - 1);
        dv[u] = med(a.dl, x);
        if constexpr (LR) rv[u] = med(a.dr, x);
    }
    if constexpr (LR) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (x0 + u * nt < a.W) rview[x0 + u * nt] = (uint16_t)rv[u];
        for (int xb = x0 + U * nt; xb < a.W; xb += U * nt) {
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = med(a.dr, min(xb + u * nt, a.W - 1));
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (xb + u * nt < a.W) rview[xb + u * nt] = (uint16_t)rv[u];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) finish(x0 + u * nt, (int)dv[u]);
    for (int xb = x0 + U * nt; xb < a.W; xb += U * nt) {
#pragma unroll
        for (int u = 0; u < U; ++u) dv[u] = med(a.dl, min(xb + u * nt, a.W - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) finish(xb + u * nt, (int)dv[u]);
    }
}

__device__ inline void post_row(const PostArgs& a, int y, uint16_t* rview) {
    if (a.lrcheck) {
        if (a.median)
            post_row_impl<true, true>(a, y, rview);
        else
            post_row_impl<true, false>(a, y, rview);
    } else {
        if (a.median)
            post_row_impl<false, true>(a, y, rview);
        else
            post_row_impl<false, false>(a, y, rview);
    }
}

// The post stage inside the WTA launch, without any wait: row r's median
// and check need the raw maps of rows r - 1 .. r + 1, so a block that has
// written its raw row y counts itself into rows y - 1 .. y + 1, and the
// block whose count completes a row (the last of the blocks that write its
// neighbourhood, in whatever order they ran) runs that row's post stage and
// clears its counter.  Every wave waits for its raw-map stores to complete
// (a block barrier alone does not wait for global stores), then one thread
// releases them with a device-scope fence (a write-back of this XCD's L2,
// so one per block, not one per wave) before the counting, and acquires the
// other blocks' rows after it (they may have been written through another
// L2).
__device__ inline void wta_fold_post(const WtaArgs& a, int y, uint16_t* rview) {
    __shared__ int todo[3];
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): expcnt and lgkmcnt left at their maxima
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __builtin_amdgcn_s_waitcnt(0x0F70);  // the write-back has completed
        for (int k = 0; k < 3; ++k) {
            const int r = y - 1 + k;
            todo[k] = 0;
            if (r < 0 || r >= a.H) continue;
            const int need = a.contrib * ((r > 0) + 1 + (r < a.H - 1));
            if (atomicAdd(&a.rowcnt[r], 1) + 1 == need) {
                atomicExch(&a.rowcnt[r], 0);
                todo[k] = 1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0x0F70);  // the invalidation has completed before the barrier
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
        if (todo[k]) {
            post_row(a.post, y - 1 + k, rview);
            __syncthreads();  // rview is reused by the next row
        }
    }
}


}  // namespace dev
}  // namespace sgm

/*
 * Plain, single-threaded CPU oracle for the SGM disparity pipeline of
 * Hernandez-Juarez et al., "Embedded real-time stereo estimation via
 * Semi-Global Matching on the GPU" (arXiv 1610.04121).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so the GPU kernels can be checked against a slow,
 * obviously correct definition.  It shares no code, header or table with the
 * GPU library.  Plain loops, int32 arithmetic, no intrinsics, no threads.
 *
 * Every result is an exactly defined integer, so each step below is the
 * plain definition written out, in the order the paper's pipeline (Sec. 2)
 * runs them:
 *   census (Sec. 3.1, Eq. 1; plus the full-window census variant),
 *   matching cost (Eq. 2),
 *   per-direction aggregation (Eq. 3), sum over directions (Eq. 4),
 *   winner-take-all (Eq. 4), right-view disparity, 3x3 median (Sec. 2),
 *   left-right consistency check (listed as a post-filter in Sec. 5).
 * Readings of points the paper leaves open are named where they are used.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EBOUND (-3) /* a bound the paper implies was violated */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Out-of-image samples take the nearest border pixel (clamp-to-edge); the
 * paper leaves corner cases out of its census pseudocode (Sec. 3.1). */
static int pix(const uint8_t *img, int W, int H, int x, int y)
{
    return img[clampi(y, 0, H - 1) * W + clampi(x, 0, W - 1)];
}

/* s(u, v) = 1 if u >= v else 0 (Sec. 3.1, next to Eq. 1). */
static uint64_t s_cmp(int u, int v) { return u >= v ? 1u : 0u; }

static int popcount64(uint64_t v)
{
    int n = 0;
    while (v) { n += (int)(v & 1u); v >>= 1; }
    return n;
}

/* Full census over a cw x ch window (cw, ch odd, cw*ch <= 64): bit
 * k = (j + ry) * cw + (i + rx) holds s(I(x+i, y+j), I(x, y)) for
 * i in [-rx, rx], j in [-ry, ry].  The centre bit is always 1. */
int oracle_census_full(const uint8_t *img, int W, int H, int cw, int ch, uint64_t *out)
{
    if (W < 1 || H < 1 || cw < 1 || ch < 1 || !(cw & 1) || !(ch & 1) || cw * ch > 64)
        return ORC_EINVAL;
    int rx = (cw - 1) / 2, ry = (ch - 1) / 2;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int c = pix(img, W, H, x, y);
            uint64_t word = 0;
            for (int j = -ry; j <= ry; j++)
                for (int i = -rx; i <= rx; i++) {
                    int k = (j + ry) * cw + (i + rx);
                    word |= s_cmp(pix(img, W, H, x + i, y + j), c) << k;
                }
            out[(size_t)y * W + x] = word;
        }
    return ORC_OK;
}

/* Center-symmetric census, Eq. 1 generalised to a cw x ch window: first, for
 * i = 1..rx and j = -ry..ry (j fastest), s(I(x+i, y+j), I(x-i, y-j)); then,
 * for j = 1..ry, s(I(x, y+j), I(x, y-j)).  Bit 0 is the first comparison.
 * For 9x7 this is the paper's 31-pair feature. */
int oracle_census_csct(const uint8_t *img, int W, int H, int cw, int ch, uint64_t *out)
{
    if (W < 1 || H < 1 || cw < 1 || ch < 1 || !(cw & 1) || !(ch & 1) || (cw * ch - 1) / 2 > 64)
        return ORC_EINVAL;
    int rx = (cw - 1) / 2, ry = (ch - 1) / 2;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            uint64_t word = 0;
            int k = 0;
            for (int i = 1; i <= rx; i++)
                for (int j = -ry; j <= ry; j++)
                    word |= s_cmp(pix(img, W, H, x + i, y + j), pix(img, W, H, x - i, y - j)) << k++;
            for (int j = 1; j <= ry; j++)
                word |= s_cmp(pix(img, W, H, x, y + j), pix(img, W, H, x, y - j)) << k++;
            out[(size_t)y * W + x] = word;
        }
    return ORC_OK;
}

/* Matching cost, Eq. 2: MC(x,y,d) = bitcount(cB(x,y) XOR cM(x-d,y)).  Where
 * x - d < 0 there is no candidate in the match image; the cost is then the
 * largest possible one, cmax (the number of census bits that can differ). */
int oracle_cost_volume(const uint64_t *cbase, const uint64_t *cmatch, int W, int H, int D,
                       int cmax, uint8_t *mc)
{
    if (W < 1 || H < 1 || D < 1 || cmax < 0 || cmax > 255) return ORC_EINVAL;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            for (int d = 0; d < D; d++) {
                int c = cmax;
                if (x - d >= 0)
                    c = popcount64(cbase[(size_t)y * W + x] ^ cmatch[(size_t)y * W + x - d]);
                mc[((size_t)y * W + x) * D + d] = (uint8_t)c;
            }
    return ORC_OK;
}

/* Aggregated cost of one path direction r = (rx, ry), Eq. 3:
 *   L_r(p,d) = C(p,d) + min( L_r(p-r,d), L_r(p-r,d-1)+P1, L_r(p-r,d+1)+P1,
 *                            min_i L_r(p-r,i)+P2 ) - min_k L_r(p-r,k).
 * Readings: where p-r lies outside the image the path starts and
 * L_r(p,d) = C(p,d); the d-1 and d+1 terms are absent at d = 0 and d = D-1.
 * A path is a straight line of pixels entering at the image border, so a
 * diagonal path is cut where it leaves the image (the paper's wrap-around of
 * diagonal slices is a schedule, not a different result).
 *
 * Pixels are visited so that p - r is always done before p: rows in the order
 * of ry, and within a row in the order of rx.  Only the previous row (or the
 * previous pixel of the current row) is kept.  If lr_out is non-NULL the full
 * L_r[H][W][D] is written there; if sum is non-NULL, L_r is added into it.
 * Returns ORC_EBOUND if any value leaves [C, C + P2] (the bound that
 * the last term of Eq. 3 guarantees). */
/* Matching cost with the RIGHT image as base (the second SGM of the
 * full left-right check, a reading of the post-filter named in Sec. 5):
 * C_R(x, y, d) = popcount(cR(x, y) XOR cL(x + d, y)) for x + d < W, and Cmax
 * where x + d falls outside the image (the mirror of Eq. 2). */
int oracle_cost_volume_right(const uint64_t *cright, const uint64_t *cleft, int W, int H, int D,
                             int cmax, uint8_t *mc)
{
    if (W < 1 || H < 1 || D < 1 || cmax < 0 || cmax > 255) return ORC_EINVAL;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            for (int d = 0; d < D; d++) {
                int c = cmax;
                if (x + d < W)
                    c = popcount64(cright[(size_t)y * W + x] ^ cleft[(size_t)y * W + x + d]);
                mc[((size_t)y * W + x) * D + d] = (uint8_t)c;
            }
    return ORC_OK;
}

/* Eq. 3 along direction r.  With img == NULL the penalty P2 is the constant
 * of Eq. 3.  With the base image img, the P2 of a step from p - r to p is
 * max(P1, floor(P2 / (1 + |I(p) - I(p - r)|))): smaller across intensity
 * edges (a reading of the adaptive P2 the paper lists as later work,
 * Sec. 5). */
int oracle_aggregate_img(const uint8_t *mc, const uint8_t *img, int W, int H, int D, int P1, int P2,
                         int rx, int ry, int32_t *lr_out, uint32_t *sum)
{
    if (W < 1 || H < 1 || D < 1 || P1 < 0 || P2 < 0) return ORC_EINVAL;
    if (rx < -1 || rx > 1 || ry < -1 || ry > 1 || (rx == 0 && ry == 0)) return ORC_EINVAL;
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)W * D);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)W * D);
    if (!prev || !cur) { free(prev); free(cur); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (int yi = 0; yi < H; yi++) {
        int y = ry >= 0 ? yi : H - 1 - yi;
        for (int xi = 0; xi < W; xi++) {
            int x = rx >= 0 ? xi : W - 1 - xi;
            int px = x - rx, py = y - ry;
            const uint8_t *c = mc + ((size_t)y * W + x) * D;
            int32_t *l = cur + (size_t)x * D;
            if (px < 0 || px >= W || py < 0 || py >= H) {
                for (int d = 0; d < D; d++) l[d] = c[d];
            } else {
                /* the predecessor is in this row (horizontal paths) or the
                 * previous one */
                const int32_t *lp = (ry == 0 ? cur : prev) + (size_t)px * D;
                int32_t m = lp[0];
                for (int k = 1; k < D; k++) if (lp[k] < m) m = lp[k];
                int p2 = P2;
                if (img) {
                    int g = abs((int)img[(size_t)y * W + x] - (int)img[(size_t)py * W + px]);
                    p2 = P2 / (1 + g);
                    if (p2 < P1) p2 = P1;
                }
                for (int d = 0; d < D; d++) {
                    int32_t best = lp[d];
                    if (d >= 1 && lp[d - 1] + P1 < best) best = lp[d - 1] + P1;
                    if (d <= D - 2 && lp[d + 1] + P1 < best) best = lp[d + 1] + P1;
                    if (m + p2 < best) best = m + p2;
                    l[d] = c[d] + best - m;
                }
            }
            for (int d = 0; d < D; d++) {
                if (l[d] < c[d] || l[d] > c[d] + (P1 > P2 ? P1 : P2)) rc = ORC_EBOUND;
                if (lr_out) lr_out[((size_t)y * W + x) * D + d] = l[d];
                if (sum) sum[((size_t)y * W + x) * D + d] += (uint32_t)l[d];
            }
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    free(prev);
    free(cur);
    return rc;
}

int oracle_aggregate(const uint8_t *mc, int W, int H, int D, int P1, int P2, int rx, int ry,
                     int32_t *lr_out, uint32_t *sum)
{
    return oracle_aggregate_img(mc, NULL, W, H, D, P1, P2, rx, ry, lr_out, sum);
}

/* The path directions: 2 paths = left-to-right and top-to-bottom (Sec. 4);
 * 4 = the axial ones; 8 = axial plus diagonal. */
static const int DIRS[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1},
                               {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};

int oracle_direction(int n_paths, int index, int *rx, int *ry)
{
    if (!(n_paths == 2 || n_paths == 4 || n_paths == 8) || index < 0 || index >= n_paths)
        return ORC_EINVAL;
    if (n_paths == 2) index = index == 0 ? 0 : 2;
    *rx = DIRS[index][0];
    *ry = DIRS[index][1];
    return ORC_OK;
}

/* Winner-take-all of Eq. 4 on the summed costs: the disparity of least
 * S(p, d).  Ties go to the smallest d (the paper does not say). */
void oracle_wta_left(const uint32_t *S, int W, int H, int D, uint16_t *dl)
{
    for (size_t p = 0; p < (size_t)W * H; p++) {
        int best = 0;
        for (int d = 1; d < D; d++)
            if (S[p * D + d] < S[p * D + best]) best = d;
        dl[p] = (uint16_t)best;
    }
}

/* Right-view disparity from the same summed costs: right pixel (x, y) sees
 * left pixel (x + d, y) at disparity d, so
 *   D_R(x, y) = argmin over d in [0, min(D, W - x)) of S(x + d, y, d),
 * ties to the smallest d.  This is the input of the left-right check, which
 * the paper names as future work without defining it. */
void oracle_wta_right(const uint32_t *S, int W, int H, int D, uint16_t *dr)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int dlim = W - x < D ? W - x : D;
            int best = 0;
            uint32_t bv = S[((size_t)y * W + x) * D + 0];
            for (int d = 1; d < dlim; d++) {
                uint32_t v = S[((size_t)y * W + x + d) * D + d];
                if (v < bv) { bv = v; best = d; }
            }
            dr[(size_t)y * W + x] = (uint16_t)best;
        }
}

/* 3x3 median (Sec. 2, stage 4) with clamp-to-edge neighbours: the 5th
 * smallest of the 9 values. */
/* Sub-pixel refinement (a reading of the sub-pixel estimation the paper
 * names as later work, Sec. 5): the vertex of the parabola through
 * (d-1, S(d-1)), (d, S(d)), (d+1, S(d+1)) at the winner d, in 1/16 pixel.
 * With a = S(d-1), b = S(d), c = S(d+1) and den = a + c - 2b (>= 0 because
 * b is the minimum), the vertex lies at d + (a - c) / (2 den); it is rounded
 * half up to 1/16: f = floor((16 (a - c) + den) / (2 den)), in [-8, 8].
 * f = 0 when d = 0, d = D - 1 or den = 0.  Output q = 16 d + f. */
void oracle_subpixel(const uint32_t *S, const uint16_t *dl, int W, int H, int D, uint16_t *q)
{
    for (int i = 0; i < W * H; i++) {
        int d = dl[i], f = 0;
        if (d > 0 && d < D - 1) {
            const uint32_t *s = S + (size_t)i * D;
            long long a = s[d - 1], b = s[d], c = s[d + 1];
            long long den = a + c - 2 * b;
            if (den > 0) {
                long long num = 16 * (a - c) + den, div = 2 * den;
                long long fl = num / div;
                if (num % div != 0 && num < 0) fl -= 1; /* floor for negative numerators */
                f = (int)fl;
            }
        }
        q[i] = (uint16_t)(16 * d + f);
    }
}

/* Left-right check on sub-pixel left disparities: the rounded integer
 * disparity di = (q + 8) / 16 indexes and is compared as in
 * oracle_lr_check; a valid pixel keeps q. */
void oracle_lr_check_q4(const uint16_t *q, const uint16_t *dr, int W, int H, int thr, uint16_t *out)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int qq = q[y * W + x], di = (qq + 8) >> 4;
            uint16_t o = 0xFFFF;
            if (x - di >= 0) {
                int e = dr[y * W + x - di];
                if (abs(di - e) <= thr) o = (uint16_t)qq;
            }
            out[y * W + x] = o;
        }
}

void oracle_median3(const uint16_t *in, int W, int H, uint16_t *out)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            uint16_t v[9];
            int n = 0;
            for (int j = -1; j <= 1; j++)
                for (int i = -1; i <= 1; i++)
                    v[n++] = in[(size_t)clampi(y + j, 0, H - 1) * W + clampi(x + i, 0, W - 1)];
            for (int a = 1; a < 9; a++) { /* insertion sort */
                uint16_t t = v[a];
                int b = a - 1;
                while (b >= 0 && v[b] > t) { v[b + 1] = v[b]; b--; }
                v[b + 1] = t;
            }
            out[(size_t)y * W + x] = v[4];
        }
}

/* Left-right consistency: keep D_L(x,y) where the right-view disparity at the
 * matched pixel agrees within thr, i.e. x - D_L >= 0 and
 * |D_L(x,y) - D_R(x - D_L(x,y), y)| <= thr; elsewhere write 0xFFFF. */
void oracle_lr_check(const uint16_t *dl, const uint16_t *dr, int W, int H, int thr, uint16_t *out)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int d = dl[(size_t)y * W + x];
            uint16_t o = 0xFFFF;
            if (x - d >= 0) {
                int e = dr[(size_t)y * W + x - d];
                int diff = d > e ? d - e : e - d;
                if (diff <= thr) o = (uint16_t)d;
            }
            out[(size_t)y * W + x] = o;
        }
}

#define ORC_MEDIAN 1u
#define ORC_LRCHECK 2u
#define ORC_CSCT 4u
#define ORC_LRFULL 8u /* D_R from a second SGM with the right image as base */
#define ORC_SUBPIXEL 16u /* left disparities in 1/16 pixel (oracle_subpixel) */
#define ORC_ADAPTIVE 32u /* P2 of each step from the base image's gradient */

/* The whole pipeline for one pair.  Optional outputs (NULL to skip):
 * census_l/census_r [H][W] u64, S [H][W][D] u32, dl_raw/dr_raw [H][W]. */
int oracle_sgm(const uint8_t *left, const uint8_t *right, int W, int H, int D, int P1, int P2,
               int n_paths, int cw, int ch, unsigned flags, int lr_thr, uint16_t *out,
               uint64_t *census_l, uint64_t *census_r, uint32_t *S_out, uint16_t *dl_raw,
               uint16_t *dr_raw)
{
    if (W < 1 || H < 1 || D < 1 || D > 256 || P1 < 0 || P2 < 0) return ORC_EINVAL;
    if (!(n_paths == 2 || n_paths == 4 || n_paths == 8)) return ORC_EINVAL;
    size_t npx = (size_t)W * H, ncell = npx * (size_t)D;
    int csct = (flags & ORC_CSCT) != 0;
    int cmax = csct ? (cw * ch - 1) / 2 : cw * ch - 1;
    uint64_t *cl = census_l ? census_l : (uint64_t *)malloc(npx * 8);
    uint64_t *cr = census_r ? census_r : (uint64_t *)malloc(npx * 8);
    uint8_t *mc = (uint8_t *)malloc(ncell);
    uint32_t *S = S_out ? S_out : (uint32_t *)malloc(ncell * 4);
    uint16_t *dl = (uint16_t *)malloc(npx * 2), *dr = (uint16_t *)malloc(npx * 2);
    uint16_t *t1 = (uint16_t *)malloc(npx * 2), *t2 = (uint16_t *)malloc(npx * 2);
    int rc = ORC_OK;
    if (!cl || !cr || !mc || !S || !dl || !dr || !t1 || !t2) { rc = ORC_ENOMEM; goto done; }

    rc = csct ? oracle_census_csct(left, W, H, cw, ch, cl) : oracle_census_full(left, W, H, cw, ch, cl);
    if (rc) goto done;
    rc = csct ? oracle_census_csct(right, W, H, cw, ch, cr) : oracle_census_full(right, W, H, cw, ch, cr);
    if (rc) goto done;
    rc = oracle_cost_volume(cl, cr, W, H, D, cmax, mc);
    if (rc) goto done;
    memset(S, 0, ncell * 4);
    for (int r = 0; r < n_paths; r++) {
        int rx, ry;
        oracle_direction(n_paths, r, &rx, &ry);
        int a = oracle_aggregate_img(mc, (flags & ORC_ADAPTIVE) ? left : NULL, W, H, D, P1, P2, rx, ry, NULL, S);
        if (a) { rc = a; goto done; }
    }
    for (size_t i = 0; i < ncell; i++)
        if (S[i] > 65535u) { rc = ORC_EBOUND; goto done; }

    oracle_wta_left(S, W, H, D, dl);
    if (flags & ORC_LRFULL) {
        /* the same pipeline with the right image as base: its own costs,
         * the same path directions, the smallest minimising d */
        uint32_t *SR = (uint32_t *)malloc(ncell * 4);
        if (!SR) { rc = ORC_ENOMEM; goto done; }
        rc = oracle_cost_volume_right(cr, cl, W, H, D, cmax, mc);
        memset(SR, 0, ncell * 4);
        for (int r = 0; r < n_paths && !rc; r++) {
            int rx, ry;
            oracle_direction(n_paths, r, &rx, &ry);
            rc = oracle_aggregate_img(mc, (flags & ORC_ADAPTIVE) ? right : NULL, W, H, D, P1, P2, rx, ry, NULL, SR);
        }
        for (size_t i = 0; i < ncell && !rc; i++)
            if (SR[i] > 65535u) rc = ORC_EBOUND;
        if (!rc) oracle_wta_left(SR, W, H, D, dr);
        free(SR);
        if (rc) goto done;
    } else {
        oracle_wta_right(S, W, H, D, dr);
    }
    if (flags & ORC_SUBPIXEL) {
        oracle_subpixel(S, dl, W, H, D, t1);
        memcpy(dl, t1, npx * 2);
    }
    if (dl_raw) memcpy(dl_raw, dl, npx * 2);
    if (dr_raw) memcpy(dr_raw, dr, npx * 2);
    if (flags & ORC_MEDIAN) {
        oracle_median3(dl, W, H, t1);
        oracle_median3(dr, W, H, t2);
        memcpy(dl, t1, npx * 2);
        memcpy(dr, t2, npx * 2);
    }
    if ((flags & ORC_LRCHECK) && (flags & ORC_SUBPIXEL))
        oracle_lr_check_q4(dl, dr, W, H, lr_thr, out);
    else if (flags & ORC_LRCHECK)
        oracle_lr_check(dl, dr, W, H, lr_thr, out);
    else
        memcpy(out, dl, npx * 2);
done:
    if (!census_l) free(cl);
    if (!census_r) free(cr);
    if (!S_out) free(S);
    free(mc); free(dl); free(dr); free(t1); free(t2);
    return rc;
}

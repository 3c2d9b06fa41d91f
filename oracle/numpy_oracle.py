"""Second, independently written CPU oracle in numpy - TEST INFRASTRUCTURE.

Same definitions as the C oracle (census with clamp-to-edge, Eq. 1 and the
full-window variant; cost Eq. 2 with the largest cost where x - d < 0;
aggregation Eq. 3 with the path starting at the image border; WTA Eq. 4 with
ties to the smallest d; right-view WTA along x + d; 3x3 median with edge
replication; left-right check), but a different structure: whole-image array
shifts instead of per-pixel loops, and each direction advanced one row (or one
column) at a time for all scanlines at once.  It is slow in other ways than
the C one and is meant for small images.
"""
from __future__ import annotations

import numpy as np


def _shift(img: np.ndarray, dx: int, dy: int) -> np.ndarray:
    """out[y, x] = img[clamp(y + dy), clamp(x + dx)]."""
    H, W = img.shape
    ys = np.clip(np.arange(H) + dy, 0, H - 1)
    xs = np.clip(np.arange(W) + dx, 0, W - 1)
    return img[np.ix_(ys, xs)]


def census_full(img, cw=9, ch=7):
    img = img.astype(np.int32)
    rx, ry = cw // 2, ch // 2
    out = np.zeros(img.shape, dtype=np.uint64)
    for j in range(-ry, ry + 1):
        for i in range(-rx, rx + 1):
            bit = (_shift(img, i, j) >= img).astype(np.uint64)
            out |= bit << np.uint64((j + ry) * cw + (i + rx))
    return out


def census_csct(img, cw=9, ch=7):
    img = img.astype(np.int32)
    rx, ry = cw // 2, ch // 2
    pairs = [(i, j) for i in range(1, rx + 1) for j in range(-ry, ry + 1)]
    pairs += [(0, j) for j in range(1, ry + 1)]
    out = np.zeros(img.shape, dtype=np.uint64)
    for k, (i, j) in enumerate(pairs):
        bit = (_shift(img, i, j) >= _shift(img, -i, -j)).astype(np.uint64)
        out |= bit << np.uint64(k)
    return out


def _popcount(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64)
    n = np.zeros(v.shape, dtype=np.int32)
    for b in range(64):
        n += ((v >> np.uint64(b)) & np.uint64(1)).astype(np.int32)
    return n


def cost_volume(cl, cr, D, cmax):
    H, W = cl.shape
    mc = np.full((H, W, D), cmax, dtype=np.int32)
    for d in range(min(D, W)):
        mc[:, d:, d] = _popcount(cl[:, d:] ^ cr[:, :W - d])
    return mc


def _step(prev, c, P1, P2):
    """One application of Eq. 3 to a batch of predecessor vectors [n][D]."""
    prev = prev.astype(np.int64)
    m = prev.min(axis=1, keepdims=True)
    big = np.iinfo(np.int64).max // 4
    lo = np.concatenate([np.full_like(prev[:, :1], big), prev[:, :-1]], axis=1)
    hi = np.concatenate([prev[:, 1:], np.full_like(prev[:, :1], big)], axis=1)
    best = np.minimum.reduce([prev, lo + P1, hi + P1, np.broadcast_to(m + P2, prev.shape)])
    return c + best - m


def aggregate(mc, P1, P2, rx, ry):
    """L_r[H][W][D] for direction (rx, ry), int64."""
    mc = mc.astype(np.int64)
    H, W, D = mc.shape
    L = np.zeros_like(mc)
    if ry == 0:
        xs = range(W) if rx > 0 else range(W - 1, -1, -1)
        first = True
        for x in xs:
            if first:
                L[:, x] = mc[:, x]
                first = False
            else:
                L[:, x] = _step(L[:, x - rx], mc[:, x], P1, P2)
        return L
    ys = range(H) if ry > 0 else range(H - 1, -1, -1)
    first = True
    for y in ys:
        if first:
            L[y] = mc[y]
            first = False
            continue
        prev_row = L[y - ry]
        cur = mc[y].copy()
        # pixels whose predecessor column x - rx exists continue a path
        xs = np.arange(W)
        px = xs - rx
        ok = (px >= 0) & (px < W)
        cur[ok] = _step(prev_row[px[ok]], mc[y][ok], P1, P2)
        L[y] = cur
    return L


DIRS4 = [(1, 0), (-1, 0), (0, 1), (0, -1)]
DIRS8 = DIRS4 + [(1, 1), (-1, 1), (1, -1), (-1, -1)]
DIRS2 = [(1, 0), (0, 1)]


def median3(a):
    p = np.pad(a, 1, mode="edge")
    H, W = a.shape
    stack = np.stack([p[j:j + H, i:i + W] for j in range(3) for i in range(3)], axis=0)
    return np.sort(stack, axis=0)[4].astype(a.dtype)


def sgm(left, right, D, P1=7, P2=86, n_paths=4, cw=9, ch=7, median=False, lr=False,
        csct=False, lr_thr=1):
    cen = census_csct if csct else census_full
    cmax = (cw * ch - 1) // 2 if csct else cw * ch - 1
    cl, cr = cen(left, cw, ch), cen(right, cw, ch)
    mc = cost_volume(cl, cr, D, cmax)
    dirs = {2: DIRS2, 4: DIRS4, 8: DIRS8}[n_paths]
    S = sum(aggregate(mc, P1, P2, rx, ry) for rx, ry in dirs)
    H, W, _ = S.shape
    dl = np.argmin(S, axis=2).astype(np.uint16)
    dr = np.zeros((H, W), dtype=np.uint16)
    for x in range(W):
        dlim = min(D, W - x)
        diag = S[:, x + np.arange(dlim), np.arange(dlim)]
        dr[:, x] = np.argmin(diag, axis=1)
    if median:
        dl, dr = median3(dl), median3(dr)
    if not lr:
        return dict(out=dl, S=S, cl=cl, cr=cr)
    out = np.full((H, W), 0xFFFF, dtype=np.uint16)
    xs = np.arange(W)[None, :].repeat(H, 0)
    ys = np.arange(H)[:, None].repeat(W, 1)
    tgt = xs - dl.astype(np.int64)
    ok = tgt >= 0
    e = dr[ys[ok], tgt[ok]].astype(np.int64)
    good = np.abs(dl[ok].astype(np.int64) - e) <= lr_thr
    vals = np.where(good, dl[ok], 0xFFFF).astype(np.uint16)
    out[ok] = vals
    return dict(out=out, S=S, cl=cl, cr=cr)

"""Seeded synthetic stereo pairs.

The paper measures accuracy on a public driving benchmark and speed on
640x480 pairs; neither data set is available here, so every input is
generated from a seed.  This module is the only code shared by the GPU path
and the CPU oracle: it draws images and nothing else.  It contains none of
the method's arithmetic (no census, no cost, no aggregation).

Randomness is a counter-based SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): draw ``i`` of a
stream is ``mix(base + (i + 1) * GAMMA)`` with ``base`` derived from
``(seed, stream)``, so any draw can be recomputed independently.  All image
arithmetic is integer, so a pair is bit-identical on every machine.

Scenes (disparities held in Q8, i.e. 1/256 px, integer disparity
``(q + 128) >> 8``):

* ``R`` - background plane at d=8 plus 3 rectangles of constant d in [10,60)
  with sides in [W/8, W/3] x [H/8, H/3], painted in increasing d.
* ``RS`` - scene R plus 2 slanted planar rectangles,
  d = d0 + gx (x - xc) + gy (y - yc), |gx|,|gy| <= 0.2 px/px.
* ``K`` - road-like: ground plane with d rising linearly from 0 (top row) to
  100 (bottom row), 5 box obstacles at d in [20,120), and rectangles covering
  about 10% of the area whose left texture is 128 + N(0, 0.5) (low texture).
  Disparities scale by D/128 when ``scale_to_d`` is given.

The left image is 3x3 box-blurred uniform noise.  The right image is the left
warped by the disparity field (z-buffer: the larger disparity wins), holes
filled from an independent blurred-noise field, then ``0.9 v + 2 N(0,1)``
rounded half-up and clamped to u8 (the Gaussian is an Irwin-Hall(12) sum of
u16 draws).  Ground truth is the left-view integer disparity, 0xFFFF where the
pixel is occluded in the right view or leaves the image.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
INVALID = 0xFFFF


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _stream_id(name: str) -> int:
    """FNV-1a 64 of the stream name: a fixed, documented string hash."""
    h = 0xCBF29CE484222325
    for b in name.encode():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def draws(seed: int, stream: str, n: int, offset: int = 0) -> np.ndarray:
    """Draws ``offset .. offset+n-1`` of stream ``stream`` as uint64."""
    with np.errstate(over="ignore"):
        base = _mix(np.array([(seed * 0x9E3779B97F4A7C15 + _stream_id(stream))
                              & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
        idx = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        return _mix(base + idx * GAMMA)


class Stream:
    """Sequential reader over one counter-based stream."""

    def __init__(self, seed: int, name: str):
        self.seed, self.name, self.pos = seed, name, 0

    def u64(self, n: int) -> np.ndarray:
        out = draws(self.seed, self.name, n, self.pos)
        self.pos += n
        return out

    def below(self, n: int, count: int = 1) -> np.ndarray:
        """Uniform integers in [0, n) (n < 2**32), by the multiply-shift map."""
        u = self.u64(count) >> np.uint64(32)
        return ((u * np.uint64(n)) >> np.uint64(32)).astype(np.int64)

    def range(self, lo: int, hi: int) -> int:
        """One uniform integer in [lo, hi)."""
        return lo + int(self.below(max(hi - lo, 1))[0])

    def gauss16(self, count: int) -> np.ndarray:
        """Irwin-Hall(12) integer Gaussian: about 2**16 * N(0, 1)."""
        u = self.u64(3 * count)
        parts = np.stack([(u >> np.uint64(s)) & np.uint64(0xFFFF) for s in (0, 16, 32, 48)], axis=1)
        parts = parts.reshape(count, 12).astype(np.int64)
        return parts.sum(axis=1) - 393210


def _blurred_noise(st: Stream, w: int, h: int) -> np.ndarray:
    u = (st.u64((w + 2) * (h + 2)) & np.uint64(0xFF)).astype(np.int64).reshape(h + 2, w + 2)
    acc = np.zeros((h, w), dtype=np.int64)
    for dy in range(3):
        for dx in range(3):
            acc += u[dy:dy + h, dx:dx + w]
    return ((acc + 4) // 9).astype(np.uint8)


@dataclass
class StereoPair:
    left: np.ndarray      # u8 [H][W]
    right: np.ndarray     # u8 [H][W]
    gt: np.ndarray        # u16 [H][W], left-view integer disparity, 0xFFFF = occluded
    sha_left: str
    sha_right: str


def _rects(st: Stream, w: int, h: int, n: int, wlo, whi, hlo, hhi):
    out = []
    for _ in range(n):
        rw = st.range(max(wlo, 1), max(whi, wlo + 1) + 1)
        rh = st.range(max(hlo, 1), max(hhi, hlo + 1) + 1)
        rw, rh = min(rw, w), min(rh, h)
        x0 = st.range(0, w - rw + 1)
        y0 = st.range(0, h - rh + 1)
        out.append((x0, y0, rw, rh))
    return out


def disparity_field(scene: str, w: int, h: int, max_disp: int, seed: int,
                    scale_to_d: bool = False):
    """Q8 disparity field (int64 [H][W]) and, for scene K, a low-texture mask."""
    st = Stream(seed, "scene")
    q = np.full((h, w), 8 * 256, dtype=np.int64)
    lowtex = np.zeros((h, w), dtype=bool)
    xs = np.arange(w, dtype=np.int64)[None, :]
    ys = np.arange(h, dtype=np.int64)[:, None]
    if scene in ("R", "RS"):
        rects = _rects(st, w, h, 3, w // 8, w // 3, h // 8, h // 3)
        ds = [st.range(10, 60) for _ in rects]
        for (x0, y0, rw, rh), d in sorted(zip(rects, ds), key=lambda t: t[1]):
            q[y0:y0 + rh, x0:x0 + rw] = d * 256
        if scene == "RS":
            for (x0, y0, rw, rh) in _rects(st, w, h, 2, w // 8, w // 3, h // 8, h // 3):
                d0 = st.range(10, 60)
                gx = st.range(-51, 52)
                gy = st.range(-51, 52)
                xc, yc = x0 + rw // 2, y0 + rh // 2
                plane = d0 * 256 + gx * (xs - xc) + gy * (ys - yc)
                q[y0:y0 + rh, x0:x0 + rw] = plane[y0:y0 + rh, x0:x0 + rw]
    elif scene == "K":
        num = max_disp if scale_to_d else 128
        q = (100 * 256 * num // 128) * ys // max(h - 1, 1) + 0 * xs
        for (x0, y0, rw, rh) in _rects(st, w, h, 5, w // 16, w // 6, h // 8, h // 3):
            d = st.range(20, 120) * num // 128
            q[y0:y0 + rh, x0:x0 + rw] = d * 256
        area, target = 0, (w * h) // 10
        while area < target:
            (x0, y0, rw, rh), = _rects(st, w, h, 1, w // 16, w // 5, h // 16, h // 5)
            lowtex[y0:y0 + rh, x0:x0 + rw] = True
            area = int(lowtex.sum())
    else:
        raise ValueError(f"unknown scene {scene!r}")
    q = np.clip(q, 0, (max_disp - 1) * 256)
    return q, lowtex


def make_pair(w: int, h: int, max_disp: int, scene: str, seed: int,
              scale_to_d: bool = False, sigma: int = 2, gain_tenths: int = 9) -> StereoPair:
    """One seeded stereo pair of the given scene (see module docstring)."""
    q, lowtex = disparity_field(scene, w, h, max_disp, seed, scale_to_d)
    d = (q + 128) >> 8
    left = _blurred_noise(Stream(seed, "texture"), w, h)
    if lowtex.any():
        g = Stream(seed, "lowtex").gauss16(int(lowtex.sum()))
        # 128 + 0.5 N(0,1), rounded half-up
        left[lowtex] = np.clip((128 * 2 ** 17 + g + 2 ** 16) // 2 ** 17, 0, 255).astype(np.uint8)

    # forward warp with a z-buffer: left pixel (x, y) lands on (x - d, y)
    yy, xx = np.nonzero(np.ones((h, w), dtype=bool))
    dd = d[yy, xx]
    xt = xx - dd
    ok = xt >= 0
    yy, xx, dd, xt = yy[ok], xx[ok], dd[ok], xt[ok]
    flat = yy * w + xt
    zbuf = np.full(h * w, -1, dtype=np.int64)
    np.maximum.at(zbuf, flat, dd)
    win = dd == zbuf[flat]
    v = _blurred_noise(Stream(seed, "holes"), w, h).astype(np.int64).reshape(-1)
    v[flat[win]] = left[yy[win], xx[win]]
    gt = np.full((h, w), INVALID, dtype=np.uint16)
    gt[yy[win], xx[win]] = dd[win].astype(np.uint16)

    g = Stream(seed, "sensor").gauss16(h * w)
    num = gain_tenths * v * 2 ** 16 + 10 * sigma * g + 5 * 2 ** 16
    right = np.clip(num // (10 * 2 ** 16), 0, 255).astype(np.uint8).reshape(h, w)
    left = np.ascontiguousarray(left)
    return StereoPair(left, right, gt,
                      hashlib.sha256(left.tobytes()).hexdigest(),
                      hashlib.sha256(right.tobytes()).hexdigest())


def noise_image(w: int, h: int, seed: int, stream: str = "noise", blur: bool = False) -> np.ndarray:
    """Plain uniform (or 3x3-blurred) u8 noise."""
    st = Stream(seed, stream)
    if blur:
        return _blurred_noise(st, w, h)
    return (st.u64(w * h) & np.uint64(0xFF)).astype(np.uint8).reshape(h, w)


def shifted_pair(w: int, h: int, shift: int, seed: int, blur: bool = False):
    """Constant-shift pair: right(x, y) = left(x + shift, y); columns that have
    no source are filled with independent noise."""
    big = noise_image(w + shift, h, seed, "shift-src", blur)
    left = np.ascontiguousarray(big[:, :w])
    right = np.ascontiguousarray(big[:, shift:shift + w])
    return left, right


# Workloads used by tests and the benchmark (shapes follow the paper's 640x480,
# D=128 pairs and a 1242x375 driving-camera frame).
WORKLOADS = {
    "small_320x240_d64_p4": dict(w=320, h=240, max_disp=64, n_paths=4, scene="R",
                                 seed=1610041210, median=False, lr=False),
    "vga_640x480_d128_p4": dict(w=640, h=480, max_disp=128, n_paths=4, scene="RS",
                                seed=1610041211, median=True, lr=True),
    "drive_1242x375_d128_p8": dict(w=1242, h=375, max_disp=128, n_paths=8, scene="K",
                                   seed=1610041212, median=True, lr=True),
}
P1_DEFAULT, P2_DEFAULT = 7, 86


def workload_pair(name: str) -> StereoPair:
    cfg = WORKLOADS[name]
    return make_pair(cfg["w"], cfg["h"], cfg["max_disp"], cfg["scene"], cfg["seed"])


BATCH_SHAPES = [(320, 240), (640, 480), (1242, 375), (1280, 720)]


def batch_items(n: int = 64, seed: int = 1610041213):
    """Shapes and parameters of a heterogeneous batch of pairs."""
    st = Stream(seed, "shape")
    items = []
    for i in range(n):
        w, h = BATCH_SHAPES[int(st.below(len(BATCH_SHAPES))[0])]
        dmax = (64, 128)[int(st.below(2)[0])]
        paths = (4, 8)[int(st.below(2)[0])]
        items.append(dict(w=w, h=h, max_disp=dmax, n_paths=paths, scene="R", seed=seed * 1000 + i))
    return items


SERVE_SIZES = [(640, 480), (1242, 375), (1280, 720), (1920, 1080)]
SERVE_DISP = [128, 256]


def serve_kinds(seed: int = 1610041214):
    """The (size, disparity range) combinations of the served request mix,
    8 paths with median and LR check, one seeded pair each: the road scene K
    with its disparities scaled to the range (ground plane 0 .. 100 D / 128,
    obstacles at [20, 120) D / 128)."""
    kinds = []
    for k, ((w, h), d) in enumerate((s, d) for s in SERVE_SIZES for d in SERVE_DISP):
        kinds.append(dict(w=w, h=h, max_disp=d, n_paths=8, median=True, lr=True, scene="K", scale_to_d=True,
                          seed=seed * 100 + k))
    return kinds


def spec_pair(spec: dict) -> StereoPair:
    """The pair a workload spec (w, h, max_disp, scene, seed and optional
    scale_to_d) describes."""
    return make_pair(spec["w"], spec["h"], spec["max_disp"], spec["scene"], seed=spec["seed"],
                     scale_to_d=spec.get("scale_to_d", False))

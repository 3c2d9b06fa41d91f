"""CPU oracle for the SGM pipeline (arXiv 1610.04121) - TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it.

Two independent implementations live here:

* ``sgm_oracle.c`` - plain single-threaded C, loaded through ctypes
  (:func:`sgm`, :func:`census`, :func:`cost_volume`, :func:`aggregate`, ...);
* ``numpy_oracle.py`` - a separately written numpy version (vectorised over
  scanlines and disparities) used as a second opinion on small inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgm_oracle.c")
_LIB = os.path.join(_HERE, "libsgm_oracle.so")

MEDIAN, LRCHECK, CSCT, LRFULL, SUBPIXEL, ADAPTIVE = 1, 2, 4, 8, 16, 32
OK, EINVAL, ENOMEM, EBOUND = 0, -1, -2, -3


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc -O2 (no intrinsics, no threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i = ctypes.c_int
        L.oracle_census_full.argtypes = [P, i, i, i, i, P]
        L.oracle_census_csct.argtypes = [P, i, i, i, i, P]
        L.oracle_cost_volume.argtypes = [P, P, i, i, i, i, P]
        L.oracle_cost_volume_right.argtypes = [P, P, i, i, i, i, P]
        L.oracle_aggregate.argtypes = [P, i, i, i, i, i, i, i, P, P]
        L.oracle_aggregate_img.argtypes = [P, P, i, i, i, i, i, i, i, P, P]
        L.oracle_direction.argtypes = [i, i, P, P]
        L.oracle_wta_left.argtypes = [P, i, i, i, P]
        L.oracle_wta_right.argtypes = [P, i, i, i, P]
        L.oracle_median3.argtypes = [P, i, i, P]
        L.oracle_lr_check.argtypes = [P, P, i, i, i, P]
        L.oracle_lr_check_q4.argtypes = [P, P, i, i, i, P]
        L.oracle_subpixel.argtypes = [P, P, i, i, i, P]
        L.oracle_sgm.argtypes = [P, P, i, i, i, i, i, i, i, i, ctypes.c_uint, i, P, P, P, P, P, P]
        for f in ("oracle_census_full", "oracle_census_csct", "oracle_cost_volume", "oracle_cost_volume_right",
                  "oracle_aggregate", "oracle_aggregate_img", "oracle_direction", "oracle_sgm"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u8(img):
    img = np.ascontiguousarray(img, dtype=np.uint8)
    assert img.ndim == 2
    return img


def census(img, cw=9, ch=7, csct=False) -> np.ndarray:
    img = _u8(img)
    H, W = img.shape
    out = np.zeros((H, W), dtype=np.uint64)
    f = lib().oracle_census_csct if csct else lib().oracle_census_full
    rc = f(_p(img), W, H, cw, ch, _p(out))
    if rc:
        raise ValueError(f"oracle census rc={rc}")
    return out


def cmax_of(cw=9, ch=7, csct=False) -> int:
    return (cw * ch - 1) // 2 if csct else cw * ch - 1


def cost_volume(cbase, cmatch, D, cmax) -> np.ndarray:
    cbase = np.ascontiguousarray(cbase, dtype=np.uint64)
    cmatch = np.ascontiguousarray(cmatch, dtype=np.uint64)
    H, W = cbase.shape
    mc = np.zeros((H, W, D), dtype=np.uint8)
    rc = lib().oracle_cost_volume(_p(cbase), _p(cmatch), W, H, D, cmax, _p(mc))
    if rc:
        raise ValueError(f"oracle cost rc={rc}")
    return mc


def cost_volume_right(cright, cleft, D, cmax) -> np.ndarray:
    """Costs with the right image as base: C_R(x, d) = HD(cR(x), cL(x + d))."""
    cright = np.ascontiguousarray(cright, dtype=np.uint64)
    cleft = np.ascontiguousarray(cleft, dtype=np.uint64)
    H, W = cright.shape
    mc = np.zeros((H, W, D), dtype=np.uint8)
    rc = lib().oracle_cost_volume_right(_p(cright), _p(cleft), W, H, D, cmax, _p(mc))
    if rc:
        raise ValueError(f"oracle cost rc={rc}")
    return mc


def aggregate(mc, P1, P2, rx, ry, check_bound=True, img=None) -> np.ndarray:
    """L_r[H][W][D] (int32) of one direction from a cost volume [H][W][D];
    with img (u8 [H][W], the base image) the P2 of each step adapts to the
    intensity change along the path."""
    mc = np.ascontiguousarray(mc, dtype=np.uint8)
    H, W, D = mc.shape
    out = np.zeros((H, W, D), dtype=np.int32)
    if img is None:
        rc = lib().oracle_aggregate(_p(mc), W, H, D, P1, P2, rx, ry, _p(out), None)
    else:
        img = _u8(img)
        assert img.shape == (H, W)
        rc = lib().oracle_aggregate_img(_p(mc), _p(img), W, H, D, P1, P2, rx, ry, _p(out), None)
    if rc == EBOUND and not check_bound:
        rc = OK
    if rc:
        raise ValueError(f"oracle aggregate rc={rc}")
    return out


def directions(n_paths):
    out = []
    for r in range(n_paths):
        rx, ry = ctypes.c_int(), ctypes.c_int()
        rc = lib().oracle_direction(n_paths, r, ctypes.byref(rx), ctypes.byref(ry))
        if rc:
            raise ValueError("bad n_paths")
        out.append((rx.value, ry.value))
    return out


def wta_left(S):
    S = np.ascontiguousarray(S, dtype=np.uint32)
    H, W, D = S.shape
    out = np.zeros((H, W), dtype=np.uint16)
    lib().oracle_wta_left(_p(S), W, H, D, _p(out))
    return out


def wta_right(S):
    S = np.ascontiguousarray(S, dtype=np.uint32)
    H, W, D = S.shape
    out = np.zeros((H, W), dtype=np.uint16)
    lib().oracle_wta_right(_p(S), W, H, D, _p(out))
    return out


def subpixel(S, dl):
    """Q4 left disparities from summed costs S[H][W][D] and winners dl."""
    S = np.ascontiguousarray(S, dtype=np.uint32)
    dl = np.ascontiguousarray(dl, dtype=np.uint16)
    H, W, D = S.shape
    out = np.zeros((H, W), dtype=np.uint16)
    lib().oracle_subpixel(_p(S), _p(dl), W, H, D, _p(out))
    return out


def lr_check_q4(q, dr, thr=1):
    q = np.ascontiguousarray(q, dtype=np.uint16)
    dr = np.ascontiguousarray(dr, dtype=np.uint16)
    H, W = q.shape
    out = np.zeros_like(q)
    lib().oracle_lr_check_q4(_p(q), _p(dr), W, H, thr, _p(out))
    return out


def median3(img):
    img = np.ascontiguousarray(img, dtype=np.uint16)
    H, W = img.shape
    out = np.zeros_like(img)
    lib().oracle_median3(_p(img), W, H, _p(out))
    return out


def lr_check(dl, dr, thr=1):
    dl = np.ascontiguousarray(dl, dtype=np.uint16)
    dr = np.ascontiguousarray(dr, dtype=np.uint16)
    H, W = dl.shape
    out = np.zeros_like(dl)
    lib().oracle_lr_check(_p(dl), _p(dr), W, H, thr, _p(out))
    return out


class Result:
    """Outputs of one oracle run."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def sgm(left, right, max_disp, P1=7, P2=86, n_paths=4, cw=9, ch=7, median=False, lr=False,
        csct=False, lr_thr=1, keep_sums=False, lr_full=False, subpixel=False, adaptive=False) -> Result:
    """Whole pipeline for one pair; returns out, dl_raw, dr_raw, census_l/r
    and (when keep_sums) the summed costs S[H][W][D].  lr_full: the right
    disparity comes from a second SGM with the right image as base."""
    left, right = _u8(left), _u8(right)
    H, W = left.shape
    assert right.shape == left.shape
    out = np.zeros((H, W), dtype=np.uint16)
    dl = np.zeros((H, W), dtype=np.uint16)
    dr = np.zeros((H, W), dtype=np.uint16)
    cl = np.zeros((H, W), dtype=np.uint64)
    cr = np.zeros((H, W), dtype=np.uint64)
    S = np.zeros((H, W, max_disp), dtype=np.uint32) if keep_sums else None
    flags = (MEDIAN if median else 0) | (LRCHECK if lr else 0) | (CSCT if csct else 0) | \
        (LRFULL if lr_full else 0) | (SUBPIXEL if subpixel else 0) | (ADAPTIVE if adaptive else 0)
    rc = lib().oracle_sgm(_p(left), _p(right), W, H, max_disp, P1, P2, n_paths, cw, ch, flags,
                          lr_thr, _p(out), _p(cl), _p(cr), _p(S), _p(dl), _p(dr))
    if rc:
        raise ValueError(f"oracle_sgm rc={rc}")
    return Result(out=out, dl_raw=dl, dr_raw=dr, census_l=cl, census_r=cr, S=S)

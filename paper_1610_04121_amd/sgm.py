"""Thin ctypes binding of the SGM C ABI (include/sgm.h).

Only argument marshalling lives here: tensors are passed as device pointers
and every step of the pipeline runs in the HIP library.  There is no CPU
fallback; if ``libsgm.so`` is missing or cannot be loaded the calls raise.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsgm.so")

SGM_OK, SGM_EINVAL, SGM_ENOMEM, SGM_EHIP, SGM_EBUSY, SGM_ECANCELED = 0, -1, -2, -3, -4, -5
MEDIAN3, LRCHECK, CENSUS_CSCT, GRAPH, LR_FULL, SUBPIXEL, ADAPTIVE_P2 = 1, 2, 4, 8, 16, 32, 64
TUNE_FUSED_AGG, TUNE_FUSED_CENSUS_COST, TUNE_FINAL_PASS, TUNE_POST_IN_WTA = 1, 2, 4, 8
INVALID = 0xFFFF

EXPORTS = [
    "sgm_validate", "sgm_create", "sgm_set_options", "sgm_compute", "sgm_destroy",
    "sgm_last_error", "sgm_footprint_bytes", "sgm_debug_census", "sgm_debug_sums",
    "sgm_debug_raw_disparity", "sgm_path_walk", "sgm_profile_enable", "sgm_profile_read",
    "sgm_debug_stage", "sgm_set_tuning", "sgm_get_tuning",
    "sgm_batch_create", "sgm_batch_compute", "sgm_batch_footprint", "sgm_batch_destroy",
    "sgm_compute_batch",
    "sgm_server_create", "sgm_server_set_policy", "sgm_server_request_bytes", "sgm_server_submit",
    "sgm_server_poll", "sgm_server_wait", "sgm_server_cancel", "sgm_server_get_stats", "sgm_server_destroy",
    "sgm_server_create_ex", "sgm_debug_phase_sums", "sgm_compute_noalloc", "sgm_batch_set_tuning",
    "sgm_batch_set_graph", "sgm_debug_fail_alloc", "sgm_batch_set_grid", "sgm_debug_valu_probe",
    "sgm_server_set_watchdog",
]
NOALLOC_MAX_BYTES = 256 << 20

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELED, REQ_FAILED = range(5)
FINAL = (REQ_DONE, REQ_CANCELED, REQ_FAILED)


class ServerStats(ctypes.Structure):
    """Mirror of sgm_server_stats."""
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "canceled", "failed",
                                              "groups", "grouped_requests", "pending", "running")] + \
               [(n, ctypes.c_size_t) for n in ("bytes_in_use", "peak_bytes", "budget_bytes")] + \
               [(n, ctypes.c_uint64) for n in ("timed_out", "draining_groups")]


class Item(ctypes.Structure):
    """Mirror of sgm_item."""
    _fields_ = [("w", ctypes.c_int), ("h", ctypes.c_int), ("max_disp", ctypes.c_int),
                ("n_paths", ctypes.c_int), ("flags", ctypes.c_uint),
                ("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("out", ctypes.c_void_p)]


ITEM_THRESHOLD_SET = 0x100


def item_lr_threshold(t: int) -> int:
    """SGM_ITEM_LR_THRESHOLD(t): an item's left-right threshold as flag bits."""
    if not 0 <= t <= 255:
        raise ValueError("item lr_threshold must be in [0, 255]")
    return ITEM_THRESHOLD_SET | (t << 16)
STAGES = ("census_cost", "aggregate", "wta", "post")


class SGMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sgm error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libsgm.so (torch is imported first so that the process has one
    HIP runtime: the one torch ships)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1610_04121_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, i, u = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint
    L.sgm_validate.argtypes = [i, i, i, i, i, i, i, i, u]
    L.sgm_validate.restype = i
    L.sgm_create.argtypes = [i, i, i, i, i, i, i, i]
    L.sgm_create.restype = P
    L.sgm_set_options.argtypes = [P, u, i]
    L.sgm_set_options.restype = i
    L.sgm_compute.argtypes = [P, P, P, P, P]
    L.sgm_compute.restype = i
    L.sgm_destroy.argtypes = [P]
    L.sgm_destroy.restype = None
    L.sgm_last_error.argtypes = []
    L.sgm_last_error.restype = ctypes.c_char_p
    L.sgm_footprint_bytes.argtypes = [i, i, i, i, u]
    L.sgm_footprint_bytes.restype = ctypes.c_size_t
    L.sgm_debug_census.argtypes = [P, P, P, P]
    L.sgm_debug_census.restype = i
    L.sgm_debug_sums.argtypes = [P, P, P, P, P]
    L.sgm_debug_sums.restype = i
    L.sgm_debug_raw_disparity.argtypes = [P, P, P, P, P, P]
    L.sgm_debug_raw_disparity.restype = i
    L.sgm_path_walk.argtypes = [i, i, i, i, i, i, P, P, P]
    L.sgm_path_walk.restype = i
    L.sgm_batch_create.argtypes = [i, i, i, i]
    L.sgm_batch_create.restype = P
    L.sgm_batch_compute.argtypes = [P, ctypes.POINTER(Item), i, P]
    L.sgm_batch_compute.restype = i
    L.sgm_batch_footprint.argtypes = [P, ctypes.POINTER(Item), i]
    L.sgm_batch_footprint.restype = ctypes.c_size_t
    L.sgm_batch_set_tuning.argtypes = [P, i, i]
    L.sgm_batch_set_tuning.restype = i
    L.sgm_batch_set_graph.argtypes = [P, i]
    L.sgm_batch_set_graph.restype = i
    L.sgm_debug_fail_alloc.argtypes = [i, i]
    L.sgm_debug_fail_alloc.restype = None
    L.sgm_batch_set_grid.argtypes = [P, i]
    L.sgm_batch_set_grid.restype = i
    L.sgm_debug_valu_probe.argtypes = [i, i, i, P, P]
    L.sgm_debug_valu_probe.restype = i
    L.sgm_batch_destroy.argtypes = [P]
    L.sgm_batch_destroy.restype = None
    L.sgm_compute_batch.argtypes = [ctypes.POINTER(Item), i, i, i, i, i, P]
    L.sgm_compute_batch.restype = i
    L.sgm_server_create.argtypes = [ctypes.c_size_t, i, i, i, i, i]
    L.sgm_server_create.restype = P
    L.sgm_server_create_ex.argtypes = [ctypes.c_size_t, i, i, i, i, i, i]
    L.sgm_server_create_ex.restype = P
    L.sgm_debug_phase_sums.argtypes = [P, P, P, i, P, P]
    L.sgm_debug_phase_sums.restype = i
    L.sgm_server_set_policy.argtypes = [P, i, i, ctypes.c_uint64, i]
    L.sgm_server_set_policy.restype = i
    L.sgm_server_request_bytes.argtypes = [P, ctypes.POINTER(Item)]
    L.sgm_server_request_bytes.restype = ctypes.c_size_t
    L.sgm_server_submit.argtypes = [P, ctypes.POINTER(Item), ctypes.POINTER(ctypes.c_uint64)]
    L.sgm_server_submit.restype = i
    L.sgm_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_double)]
    L.sgm_server_poll.restype = i
    L.sgm_server_wait.argtypes = [P, ctypes.c_uint64, i, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_double)]
    L.sgm_server_wait.restype = i
    L.sgm_server_cancel.argtypes = [P, ctypes.c_uint64]
    L.sgm_server_cancel.restype = i
    L.sgm_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.sgm_server_get_stats.restype = i
    L.sgm_server_set_watchdog.argtypes = [P, i]
    L.sgm_server_set_watchdog.restype = i
    L.sgm_server_destroy.argtypes = [P]
    L.sgm_server_destroy.restype = None
    L.sgm_set_tuning.argtypes = [P, i, i, i]
    L.sgm_set_tuning.restype = i
    L.sgm_get_tuning.argtypes = [P, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.sgm_get_tuning.restype = i
    L.sgm_debug_stage.argtypes = [P, P, P, i, P, P]
    L.sgm_debug_stage.restype = i
    L.sgm_profile_enable.argtypes = [P, i]
    L.sgm_profile_enable.restype = i
    L.sgm_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    L.sgm_profile_read.restype = i
    L.sgm_compute_noalloc.argtypes = [i, i, i, i, i, i, i, i, u, i, P, P, P, P]
    L.sgm_compute_noalloc.restype = i
    _lib = L
    return L


def last_error() -> str:
    return lib().sgm_last_error().decode()


def _check(rc: int):
    if rc < 0:
        raise SGMError(rc, last_error())
    return rc


def validate(width, height, max_disp, P1=7, P2=86, n_paths=4, census_w=9, census_h=7, flags=0) -> int:
    return lib().sgm_validate(width, height, max_disp, P1, P2, n_paths, census_w, census_h, flags)


def footprint_bytes(width, height, max_disp, n_paths=4, flags=0) -> int:
    return lib().sgm_footprint_bytes(width, height, max_disp, n_paths, flags)


def compute_noalloc(left, right, max_disp, P1=7, P2=86, n_paths=4, census_w=9, census_h=7, median=False,
                    lrcheck=False, csct=False, lr_threshold=1, lr_full=False, subpixel=False, adaptive_p2=False,
                    out=None, stream=None):
    """sgm_compute_noalloc: the whole pipeline with its workspace in the
    library's static device scratch (no device allocation by the library;
    ``out`` is allocated here only when not given)."""
    import torch
    h, w = left.shape
    if out is None:
        out = torch.empty((h, w), dtype=torch.uint16, device=left.device)
    flags = ((MEDIAN3 if median else 0) | (LRCHECK if lrcheck else 0) | (CENSUS_CSCT if csct else 0)
             | (LR_FULL if lr_full else 0) | (SUBPIXEL if subpixel else 0) | (ADAPTIVE_P2 if adaptive_p2 else 0))
    _check(lib().sgm_compute_noalloc(w, h, max_disp, P1, P2, n_paths, census_w, census_h, flags, lr_threshold,
                                     _ptr(left, "torch.uint8", (h, w)), _ptr(right, "torch.uint8", (h, w)),
                                     _ptr(out, "torch.uint16", (h, w)), _stream(stream)))
    return out


def path_walk(width, height, rx, ry, slice_index):
    """(xs, ys, restart) of the pixels one aggregation slice visits."""
    import numpy as np
    n = max(width, height)
    xs = np.zeros(n, dtype=np.int32)
    ys = np.zeros(n, dtype=np.int32)
    rs = np.zeros(n, dtype=np.uint8)
    k = _check(lib().sgm_path_walk(width, height, rx, ry, slice_index, n,
                                   xs.ctypes.data, ys.ctypes.data, rs.ctypes.data))
    return xs[:k], ys[:k], rs[:k].astype(bool)


def _ptr(t, dtype_name: str, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if str(t.dtype) != dtype_name:
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class SGM:
    """One context: a fixed image size and parameter set.

    ``compute(left, right, out)`` enqueues the pipeline on the current torch
    stream (or ``stream``) and returns ``out`` (u16 [H][W])."""

    def __init__(self, width, height, max_disp, P1=7, P2=86, n_paths=4, census_w=9, census_h=7,
                 median=False, lrcheck=False, csct=False, lr_threshold=1, graph=False, lr_full=False,
                 subpixel=False, adaptive_p2=False):
        self.width, self.height, self.max_disp = width, height, max_disp
        self.n_paths = n_paths
        self.params = dict(P1=P1, P2=P2, census_w=census_w, census_h=census_h)
        self._ctx = lib().sgm_create(width, height, max_disp, P1, P2, n_paths, census_w, census_h)
        if not self._ctx:
            raise SGMError(SGM_EINVAL, last_error())
        self.set_options(median=median, lrcheck=lrcheck, csct=csct, lr_threshold=lr_threshold, graph=graph,
                         lr_full=lr_full, subpixel=subpixel, adaptive_p2=adaptive_p2)

    def set_options(self, median=False, lrcheck=False, csct=False, lr_threshold=1, graph=False, lr_full=False,
                    subpixel=False, adaptive_p2=False):
        """lr_full (with lrcheck): the right map of the check comes from a
        second SGM with the right image as base.  subpixel: output in 1/16
        pixel (see SGM_SUBPIXEL in sgm.h).  adaptive_p2: the P2 of each step
        shrinks with the base image's intensity change (SGM_ADAPTIVE_P2)."""
        flags = ((MEDIAN3 if median else 0) | (LRCHECK if lrcheck else 0) | (CENSUS_CSCT if csct else 0)
                 | (GRAPH if graph else 0) | (LR_FULL if lr_full else 0) | (SUBPIXEL if subpixel else 0)
                 | (ADAPTIVE_P2 if adaptive_p2 else 0))
        _check(lib().sgm_set_options(self._ctx, flags, lr_threshold))
        self.params.update(median=median, lrcheck=lrcheck, csct=csct, lr_threshold=lr_threshold, lr_full=lr_full,
                           subpixel=subpixel, adaptive_p2=adaptive_p2)

    def autotune(self, left=None, right=None, **kw) -> dict:
        """Times every aggregation kernel shape and keeps the fastest (see tune.py)."""
        from . import tune
        return tune.autotune(self, left, right, **kw)

    def set_tuning(self, lanes_h=0, lanes_v=0, fused=False, census_cost=False, final_pass=False,
                   post_in_wta=False):
        """Kernel shapes (never change results): lanes per horizontal /
        other aggregation slice (0, 0 = default); ``fused``: the aggregation
        computes costs from census words (no cost volume); ``census_cost``:
        one census + cost launch builds the cost volume (9x7 windows);
        ``final_pass``: the last direction runs fused with the sum and the
        winner-take-all (SGM_TUNE_FINAL_PASS); ``post_in_wta``: the median
        and left-right check run inside the winner-take-all launch
        (SGM_TUNE_POST_IN_WTA)."""
        flags = (TUNE_FUSED_AGG if fused else 0) | (TUNE_FUSED_CENSUS_COST if census_cost else 0) | \
            (TUNE_FINAL_PASS if final_pass else 0) | (TUNE_POST_IN_WTA if post_in_wta else 0)
        _check(lib().sgm_set_tuning(self._ctx, lanes_h, lanes_v, flags))

    def tuning(self):
        """(lanes_h, lanes_v, fused, census_cost, final_pass, post_in_wta) in effect."""
        gh, gv, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().sgm_get_tuning(self._ctx, ctypes.byref(gh), ctypes.byref(gv), ctypes.byref(f)))
        return (gh.value, gv.value, bool(f.value & TUNE_FUSED_AGG), bool(f.value & TUNE_FUSED_CENSUS_COST),
                bool(f.value & TUNE_FINAL_PASS), bool(f.value & TUNE_POST_IN_WTA))

    @property
    def shape(self):
        return (self.height, self.width)

    def compute(self, left, right, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.uint16, device=left.device)
        _check(lib().sgm_compute(self._ctx, _ptr(left, "torch.uint8", self.shape),
                                 _ptr(right, "torch.uint8", self.shape),
                                 _ptr(out, "torch.uint16", self.shape), _stream(stream)))
        return out

    def debug_census(self, img, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.uint64, device=img.device)
        _check(lib().sgm_debug_census(self._ctx, _ptr(img, "torch.uint8", self.shape),
                                      _ptr(out, "torch.uint64", self.shape), _stream(stream)))
        return out

    def debug_sums(self, left, right, out=None, stream=None):
        import torch
        shape = (self.height, self.width, self.max_disp)
        if out is None:
            out = torch.empty(shape, dtype=torch.uint16, device=left.device)
        _check(lib().sgm_debug_sums(self._ctx, _ptr(left, "torch.uint8", self.shape),
                                    _ptr(right, "torch.uint8", self.shape),
                                    _ptr(out, "torch.uint16", shape), _stream(stream)))
        return out

    def debug_phase_sums(self, left, right, phase, stream=None):
        """Partial sums u16 [H][W][D]: phase 0 = every direction but the one
        the final pass fuses, phase 1 = all directions (sgm_debug_phase_sums)."""
        import torch
        shape = (self.height, self.width, self.max_disp)
        out = torch.empty(shape, dtype=torch.uint16, device=left.device)
        _check(lib().sgm_debug_phase_sums(self._ctx, _ptr(left, "torch.uint8", self.shape),
                                          _ptr(right, "torch.uint8", self.shape), phase,
                                          _ptr(out, "torch.uint16", shape), _stream(stream)))
        return out

    def debug_stage(self, left, right, which, stream=None):
        """which = -1: cost volume C; which = r: L_r of direction r (u16
        [H][W][D]); with lr_full, -2: right-base costs, n_paths + r: right-base
        L_r."""
        import torch
        shape = (self.height, self.width, self.max_disp)
        out = torch.empty(shape, dtype=torch.uint16, device=left.device)
        _check(lib().sgm_debug_stage(self._ctx, _ptr(left, "torch.uint8", self.shape),
                                     _ptr(right, "torch.uint8", self.shape), which,
                                     _ptr(out, "torch.uint16", shape), _stream(stream)))
        return out

    def debug_raw_disparity(self, left, right, stream=None):
        import torch
        dl = torch.empty(self.shape, dtype=torch.uint16, device=left.device)
        dr = torch.empty(self.shape, dtype=torch.uint16, device=left.device)
        _check(lib().sgm_debug_raw_disparity(self._ctx, _ptr(left, "torch.uint8", self.shape),
                                             _ptr(right, "torch.uint8", self.shape),
                                             _ptr(dl, "torch.uint16", self.shape),
                                             _ptr(dr, "torch.uint16", self.shape), _stream(stream)))
        return dl, dr

    def profile(self, enable: bool = True, every: int = 1):
        """Record per-stage HIP events in every `every`-th compute() call."""
        _check(lib().sgm_profile_enable(self._ctx, every if enable else 0))

    def profile_read(self):
        """(calls, {stage: total ms}) over the calls recorded since the last read."""
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int(0)
        _check(lib().sgm_profile_read(self._ctx, ms, ctypes.byref(n)))
        return n.value, dict(zip(STAGES, list(ms)))

    def close(self):
        if getattr(self, "_ctx", None):
            lib().sgm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _items(pairs):
    """pairs: dicts with left, right, out (device tensors), max_disp, n_paths and
    optional median, lrcheck, subpixel, lr_full, adaptive_p2, csct, lr_threshold."""
    arr = (Item * len(pairs))()
    for k, p in enumerate(pairs):
        h, w = p["left"].shape
        flags = (MEDIAN3 if p.get("median") else 0) | (LRCHECK if p.get("lrcheck") else 0) | \
            (SUBPIXEL if p.get("subpixel") else 0) | (LR_FULL if p.get("lr_full") else 0) | \
            (ADAPTIVE_P2 if p.get("adaptive_p2") else 0) | (CENSUS_CSCT if p.get("csct") else 0)
        if p.get("lr_threshold", 1) != 1:
            flags |= item_lr_threshold(p["lr_threshold"])
        arr[k] = Item(w, h, p["max_disp"], p["n_paths"], flags,
                      _ptr(p["left"], "torch.uint8", (h, w)), _ptr(p["right"], "torch.uint8", (h, w)),
                      _ptr(p["out"], "torch.uint16", (h, w)))
    return arr


class Batch:
    """Runs many pairs of different shapes with one launch per stage."""

    def __init__(self, P1=7, P2=86, census_w=9, census_h=7, graph=False):
        self._b = lib().sgm_batch_create(P1, P2, census_w, census_h)
        if not self._b:
            raise SGMError(SGM_EINVAL, last_error())
        self.params = dict(P1=P1, P2=P2, census_w=census_w, census_h=census_h)
        self.tuning = (0, 0)
        self.grid = 0
        self.graph = False
        if graph:
            self.set_graph(True)

    def set_grid(self, max_workgroups: int):
        """Workgroups of the persistent aggregation grid (sgm_batch_set_grid;
        0 = fill the device, 1 = one CU takes the queue)."""
        _check(lib().sgm_batch_set_grid(self._b, max_workgroups))
        self.grid = max_workgroups

    def set_graph(self, enable: bool):
        """Replay a captured hipGraph per batch signature (sgm_batch_set_graph)."""
        _check(lib().sgm_batch_set_graph(self._b, 1 if enable else 0))
        self.graph = bool(enable)

    def compute(self, pairs, stream=None):
        arr = _items(pairs)
        _check(lib().sgm_batch_compute(self._b, arr, len(pairs), _stream(stream)))
        return [p["out"] for p in pairs]

    def footprint(self, pairs) -> int:
        arr = _items(pairs)
        return lib().sgm_batch_footprint(self._b, arr, len(pairs))

    def set_tuning(self, lanes_h=0, lanes_v=0):
        """Lanes per horizontal / other aggregation slice for every pair (16
        or 32; 0 = the per-pair default).  Never changes results."""
        _check(lib().sgm_batch_set_tuning(self._b, lanes_h, lanes_v))
        self.tuning = (lanes_h, lanes_v)

    def autotune(self, pairs, **kw) -> dict:
        """Times every batch kernel shape and grid size on these pairs and
        keeps the fastest (see tune.autotune_batch)."""
        from . import tune
        return tune.autotune_batch(self, pairs, **kw)

    def close(self):
        if getattr(self, "_b", None):
            lib().sgm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server (see sgm_server_create).

    submit() takes device tensors and returns a ticket; the tensors are kept
    referenced here until the request reaches a final state."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4, streams: int | None = None, P1=7, P2=86,
                 census_w=9, census_h=7, max_group: int = 32, max_pending: int = 4096,
                 max_group_cells: int = 1 << 28, overlap_queue: int = 3):
        """streams defaults to one per slot (groups run concurrently)."""
        if streams is None:
            self._s = lib().sgm_server_create(hbm_budget_bytes, slots, P1, P2, census_w, census_h)
        else:
            self._s = lib().sgm_server_create_ex(hbm_budget_bytes, slots, streams, P1, P2, census_w, census_h)
        if not self._s:
            raise SGMError(SGM_EINVAL, last_error())
        self._held = {}
        self.set_policy(max_group, max_pending, max_group_cells, overlap_queue)

    def set_policy(self, max_group: int = 32, max_pending: int = 4096, max_group_cells: int = 1 << 28,
                   overlap_queue: int = 3):
        _check(lib().sgm_server_set_policy(self._s, max_group, max_pending, max_group_cells, overlap_queue))

    def request_bytes(self, pair) -> int:
        return lib().sgm_server_request_bytes(self._s, _items([pair]))

    def submit(self, pair) -> int:
        """pair: dict as for Batch.compute.  Raises SGMError (code SGM_EBUSY
        when the queue is full)."""
        arr = _items([pair])
        t = ctypes.c_uint64()
        _check(lib().sgm_server_submit(self._s, arr, ctypes.byref(t)))
        self._held[t.value] = (pair["left"], pair["right"], pair["out"])
        return t.value

    def _report(self, fn, ticket, *extra):
        st, lat = ctypes.c_int(), ctypes.c_double()
        _check(fn(self._s, ticket, *extra, ctypes.byref(st), ctypes.byref(lat)))
        if st.value in FINAL:
            self._held.pop(ticket, None)
            return st.value, lat.value
        return st.value, None

    def poll(self, ticket):
        """(status, latency_s or None)."""
        return self._report(lib().sgm_server_poll, ticket)

    def wait(self, ticket, timeout_ms: int = -1):
        return self._report(lib().sgm_server_wait, ticket, timeout_ms)

    def cancel(self, ticket):
        _check(lib().sgm_server_cancel(self._s, ticket))

    def set_watchdog(self, timeout_ms: int):
        """Fail the requests of a group still running timeout_ms after its
        launch (sgm_server_set_watchdog; 0 = off)."""
        _check(lib().sgm_server_set_watchdog(self._s, timeout_ms))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().sgm_server_get_stats(self._s, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None):
            lib().sgm_server_destroy(self._s)
            self._s = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_fail_alloc(after: int, count: int):
    """Allocation-failure hook (sgm_debug_fail_alloc): the next ``after``
    library allocations succeed and the ``count`` after them fail."""
    lib().sgm_debug_fail_alloc(after, count)


def valu_probe(blocks: int, iters: int, sink, stream=None, mode: int = 0):
    """Enqueues a VALU probe (sgm_debug_valu_probe): mode 0, throughput (16
    VALU instructions per wave per round); modes 1-3, dependent chains of 8
    links per round.  4 waves per block; ``sink`` is a device int32 tensor
    of blocks * 256 elements."""
    _check(lib().sgm_debug_valu_probe(mode, blocks, iters, _ptr(sink, "torch.int32", (blocks * 256,)),
                                      _stream(stream)))

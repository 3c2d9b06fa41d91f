"""Host-side checks of the C ABI library: it loads, exports what the header
declares, validates parameters, and its slice scheduler follows the paper's
worked example.  No compute call is made here (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT, gpu_available
from paper_1610_04121_amd import sgm

HEADER = os.path.join(ROOT, "include", "sgm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sgm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sgm.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return sgm.lib()


def test_library_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(sgm.EXPORTS) | (set(declared) - set(sgm.EXPORTS))
    for name in sgm.EXPORTS:
        assert name in declared, f"{name} exported by the binding but not declared"


def test_validate_accepts_the_workload_shapes(lib):
    assert sgm.validate(320, 240, 64, 7, 86, 4) == 0
    assert sgm.validate(640, 480, 128, 7, 86, 4, flags=sgm.MEDIAN3 | sgm.LRCHECK) == 0
    assert sgm.validate(1242, 375, 128, 7, 86, 8) == 0
    assert sgm.validate(1920, 1080, 256, 7, 86, 8) == 0
    assert sgm.validate(1, 1, 1, 0, 0, 2) == 0


@pytest.mark.parametrize("args,frag", [
    ((0, 10, 8, 7, 86, 4, 9, 7, 0), "width"),
    ((10, 0, 8, 7, 86, 4, 9, 7, 0), "height"),
    ((10, 10, 0, 7, 86, 4, 9, 7, 0), "max_disp"),
    ((10, 10, 257, 7, 86, 4, 9, 7, 0), "max_disp"),
    ((10, 10, 8, 7, 86, 3, 9, 7, 0), "n_paths"),
    ((10, 10, 8, 7, 86, 4, 8, 7, 0), "odd"),
    ((10, 10, 8, 7, 86, 4, 9, 9, 0), "64 pixels"),
    ((10, 10, 8, -1, 86, 4, 9, 7, 0), "P1"),
    ((10, 10, 8, 7, -2, 4, 9, 7, 0), "P1 and P2"),
    ((10, 10, 8, 7, 8200, 8, 9, 7, 0), "65535"),
    ((10, 10, 8, 7, 86, 4, 9, 7, 1 << 10), "flag"),
    ((20000, 10, 8, 7, 86, 4, 9, 7, 0), "width"),
])
def test_validate_rejects(lib, args, frag):
    assert sgm.validate(*args) == sgm.SGM_EINVAL
    assert frag in sgm.last_error()


def test_overflow_bound_is_exact(lib):
    # n_paths * (Cmax + P2) <= 65535 with Cmax = 62 (9x7 full census)
    p2_max = 65535 // 8 - 62
    assert sgm.validate(64, 64, 64, 7, p2_max, 8) == 0
    assert sgm.validate(64, 64, 64, 7, p2_max + 1, 8) == sgm.SGM_EINVAL
    # CSCT: Cmax = 31
    assert sgm.validate(64, 64, 64, 7, 65535 // 8 - 31, 8, flags=sgm.CENSUS_CSCT) == 0


def test_footprint_counts_cost_and_paths(lib):
    f4 = sgm.footprint_bytes(640, 480, 128, 4)
    f8 = sgm.footprint_bytes(640, 480, 128, 8)
    cells = 640 * 480 * 128
    assert f4 >= cells * (1 + 4)
    assert f8 - f4 >= 4 * cells
    assert sgm.footprint_bytes(0, 480, 128, 4) == 0


def _golden_walk():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "diag_wrap_example.txt")):
        if line.startswith("#") or not line.strip():
            continue
        x, y, r = line.split()
        rows.append((x, int(y), int(r)))
    return rows


@pytest.mark.parametrize("W,H", [(640, 480), (320, 240), (1242, 375)])
def test_diagonal_wrap_matches_the_papers_example(lib, W, H):
    xs, ys, rs = sgm.path_walk(W, H, -1, 1, 100)
    assert len(xs) == H
    for xstr, y, r in _golden_walk():
        x = eval(xstr, {"W": W})
        assert ys[y] == y and xs[y] == x and int(rs[y]) == r, (xstr, y)
    # no other restart before row 101
    assert not rs[1:101].any()


@pytest.mark.parametrize("W,H", [(7, 5), (5, 7), (1, 4), (6, 1), (33, 17)])
def test_slices_cover_every_pixel_once_and_restart_at_path_starts(lib, W, H):
    for rx, ry in [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, 1), (1, -1), (-1, -1)]:
        n_slices = H if ry == 0 else W
        seen = np.zeros((H, W), dtype=int)
        for s in range(n_slices):
            xs, ys, rs = sgm.path_walk(W, H, rx, ry, s)
            for k in range(len(xs)):
                x, y = xs[k], ys[k]
                seen[y, x] += 1
                # a restart happens exactly where the predecessor p - r is
                # outside the image, i.e. where a textbook path starts
                px, py = x - rx, y - ry
                outside = not (0 <= px < W and 0 <= py < H)
                assert bool(rs[k]) == outside, (rx, ry, s, k)
                if not outside:
                    assert (xs[k - 1], ys[k - 1]) == (px, py)
        assert (seen == 1).all()


def test_create_without_gpu_fails_cleanly(lib):
    if gpu_available():
        pytest.skip("a GPU is present")
    lib.sgm_create.restype = ctypes.c_void_p
    ctx = lib.sgm_create(64, 48, 16, 7, 86, 4, 9, 7)
    assert not ctx
    assert sgm.last_error()
    # invalid parameters are rejected before any HIP call
    assert not lib.sgm_create(0, 48, 16, 7, 86, 4, 9, 7)
    assert "width" in sgm.last_error()


def test_tuner_candidates_and_cache(tmp_path, monkeypatch):
    from paper_1610_04121_amd import tune
    c64 = tune.candidates(64)
    assert all(len(c) == 6 for c in c64)
    assert all(gh in (16, 32) and gv in (16, 32) for gh, gv, *_ in c64)
    assert len(c64) == 9 and len(tune.candidates(65)) == 15 and len(tune.candidates(256)) == 15
    assert len(tune.candidates(128, census_9x7=False)) == 10
    assert not any(f and cc for _, _, f, cc, *_ in tune.candidates(128))
    assert not any(fp for *_, fp, _ in tune.candidates(128))
    # with the final pass offered: stored cost (with and without it), one
    # census + cost launch (with and without), fused costs (never with it)
    cf = tune.candidates(128, final_pass=True)
    assert len(cf) == 25 and len(tune.candidates(64, final_pass=True)) == 15
    assert not any(f and fp for _, _, f, _, fp, _ in cf)
    assert len(set(cf)) == len(cf)
    # the post stage's placement is one fixed choice for every shape
    assert {c[5] for c in tune.candidates(128)} == {False}
    assert {c[5] for c in tune.candidates(128, post_in_wta=True)} == {True}
    monkeypatch.setenv("SGM_TUNE_CACHE", str(tmp_path / "t.json"))
    assert tune.load_cache() == {}
    tune.save_entry("a", {"choice": [32, 16, False]})
    tune.save_entry("b", {"choice": [16, 16, True]})
    assert tune.load_cache()["a"]["choice"] == [32, 16, False]
    assert set(tune.load_cache()) == {"a", "b"}
    (tmp_path / "t.json").write_text("not json")
    assert tune.load_cache() == {}


def test_batch_tuner_candidates_and_key():
    import types
    import numpy as np
    from paper_1610_04121_amd import tune
    c = tune.BATCH_CANDIDATES
    assert len(set(c)) == len(c) == len(tune.BATCH_LANES) * len(tune.BATCH_GRIDS)
    # every lane shape is offered with the device-filling grid and with one
    # workgroup per CU
    assert {g for *_, g in c} == {0, 256}
    assert {(gh, gv) for gh, gv, _ in c} == set(tune.BATCH_LANES)
    b = types.SimpleNamespace(params=dict(P1=7, P2=86, census_w=9, census_h=7))
    img = np.zeros((48, 64), np.uint8)
    base = [dict(left=img, max_disp=32, n_paths=4), dict(left=np.zeros((20, 30), np.uint8), max_disp=64, n_paths=8)]
    k = tune.batch_key(b, base)
    assert tune.batch_key(b, list(reversed(base))) == k  # a multiset of pairs
    # every per-pair option that changes the work changes the key
    for opt, val in [("median", True), ("lrcheck", True), ("subpixel", True), ("lr_full", True),
                     ("adaptive_p2", True), ("csct", True), ("lr_threshold", 3)]:
        assert tune.batch_key(b, [dict(base[0], **{opt: val}), base[1]]) != k, opt


def test_full_lr_flag_rules(lib):
    from paper_1610_04121_amd import sgm
    ok = lib.sgm_validate(64, 48, 32, 7, 86, 4, 9, 7, sgm.LRCHECK | sgm.LR_FULL)
    assert ok == 0
    assert lib.sgm_validate(64, 48, 32, 7, 86, 4, 9, 7, sgm.LR_FULL) == sgm.SGM_EINVAL
    assert "SGM_LRCHECK" in sgm.last_error()
    plain = lib.sgm_footprint_bytes(640, 480, 128, 4, sgm.LRCHECK)
    full = lib.sgm_footprint_bytes(640, 480, 128, 4, sgm.LRCHECK | sgm.LR_FULL)
    # a second cost volume (u8) and a second set of 4 L_r planes (counted as u16)
    assert full - plain >= 640 * 480 * 128 * (1 + 4 * 2)


def test_adaptive_p2_bounds_use_the_larger_penalty(lib):
    # a step's adaptive penalty is max(P1, P2 / (1 + g)): with P1 > P2 the
    # 16-bit sum bound counts P1
    p1 = 65535 // 8 - 62 + 1
    assert sgm.validate(64, 64, 64, p1, 7, 8) == 0
    assert sgm.validate(64, 64, 64, p1, 7, 8, flags=sgm.ADAPTIVE_P2) == sgm.SGM_EINVAL
    assert "max(P1, P2)" in sgm.last_error()
    assert sgm.validate(64, 64, 64, p1 - 1, 7, 8, flags=sgm.ADAPTIVE_P2) == 0


def test_noalloc_rejects_oversized_and_invalid_calls_before_the_gpu():
    # checked on the host before any device call, so this runs without a GPU
    import ctypes
    L = sgm.lib()
    buf = ctypes.c_void_p(4096)  # never dereferenced: the call fails first
    assert L.sgm_compute_noalloc(1920, 1080, 256, 7, 86, 8, 9, 7, 0, 1, buf, buf, ctypes.c_void_p(8192),
                                 None) == sgm.SGM_ENOMEM
    assert "static scratch" in sgm.last_error()
    assert L.sgm_compute_noalloc(640, 480, 128, 7, 86, 3, 9, 7, 0, 1, buf, buf, ctypes.c_void_p(8192),
                                 None) == sgm.SGM_EINVAL
    assert L.sgm_compute_noalloc(64, 48, 32, 7, 86, 4, 9, 7, sgm.GRAPH, 1, buf, buf, ctypes.c_void_p(8192),
                                 None) == sgm.SGM_EINVAL
    assert L.sgm_compute_noalloc(64, 48, 32, 7, 86, 4, 9, 7, 0, 1, buf, buf, buf, None) == sgm.SGM_EINVAL
    assert sgm.NOALLOC_MAX_BYTES == 256 << 20


def test_valu_probe_validates_before_launching(lib):
    from paper_1610_04121_amd import sgm
    assert lib.sgm_debug_valu_probe(0, 0, 16, None, None) == sgm.SGM_EINVAL
    assert "blocks" in sgm.last_error()
    assert lib.sgm_debug_valu_probe(0, 4, 0, None, None) == sgm.SGM_EINVAL
    assert lib.sgm_debug_valu_probe(4, 4, 16, None, None) == sgm.SGM_EINVAL
    assert "mode" in sgm.last_error()
    assert lib.sgm_debug_valu_probe(1, 4, 16, None, None) == sgm.SGM_EINVAL
    assert "null" in sgm.last_error()


def test_server_stats_mirror_matches_the_header():
    # sgm_server_stats: 9 uint64 counters, 3 size_t byte counts, 2 uint64 watchdog counters
    import ctypes

    from paper_1610_04121_amd.sgm import ServerStats
    assert ctypes.sizeof(ServerStats) == 14 * 8
    names = [n for n, _ in ServerStats._fields_]
    assert names[-2:] == ["timed_out", "draining_groups"]
    hdr = open(os.path.join(ROOT, "include", "sgm.h")).read()
    body = hdr[hdr.index("uint64_t submitted, completed"):hdr.index("} sgm_server_stats;")]
    assert "timed_out" in body and body.index("budget_bytes") < body.index("timed_out") < body.index("draining_groups")


@pytest.mark.skipif(gpu_available(), reason="checks the behaviour on a host without a GPU")
def test_creation_fails_cleanly_without_a_device(lib):
    # valid parameters but no device: NULL and a HIP message, no crash
    assert not lib.sgm_create(64, 48, 16, 7, 86, 4, 9, 7)
    assert "hip" in sgm.last_error().lower()
    assert not lib.sgm_batch_create(7, 86, 9, 7)
    assert "hip" in sgm.last_error().lower()
    assert not lib.sgm_server_create(1 << 20, 1, 7, 86, 9, 7)
    assert "hip" in sgm.last_error().lower()
    with pytest.raises(sgm.SGMError):
        sgm.SGM(64, 48, 16)

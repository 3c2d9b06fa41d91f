"""Batched pipeline (one launch per stage over pairs of different shapes)
against the oracle and against separate single-pair calls.  Exact equality."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1610_04121_amd import SGM, synth
from paper_1610_04121_amd.sgm import Batch

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _pairs(specs, dev, seed0, scenes=None):
    import torch
    out = []
    for k, (w, h, d, p, med, lr) in enumerate(specs):
        scene, seed = scenes[k] if scenes else ("RS", seed0 + k)
        pair = synth.make_pair(w, h, d, scene, seed=seed)
        out.append(dict(left=_t(pair.left, dev), right=_t(pair.right, dev), max_disp=d, n_paths=p,
                        median=med, lrcheck=lr, lr_threshold=1,
                        out=torch.empty((h, w), dtype=torch.uint16, device=dev),
                        np_left=pair.left, np_right=pair.right))
    return out


def test_heterogeneous_batch_matches_oracle(gpu):
    import torch
    specs = [(64, 48, 32, 4, False, False), (97, 31, 64, 8, True, True), (40, 70, 130, 2, True, False),
             (33, 33, 200, 8, False, True), (7, 5, 16, 4, True, True), (120, 20, 16, 8, False, False),
             (1, 9, 8, 4, False, True), (50, 1, 70, 8, True, True)]
    pairs = _pairs(specs, gpu, 300)
    _say(f"batch of {len(pairs)} mixed pairs")
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"],
                          median=p["median"], lr=p["lrcheck"]).out
        got = p["out"].cpu().numpy()
        assert (got == want).all(), (k, specs[k], int((got != want).sum()))
    b.close()


@pytest.mark.parametrize("grid", [0, 256, 1])
def test_quads_with_odd_and_even_slice_group_counts(gpu, grid):
    """The aggregation queue hands out quads: opposite axis-aligned directions
    over two slice groups, the rest (diagonals, the 2-path set, the last
    group of an odd count) packed four at a time with empty places.  Items
    whose +-x and +-y group counts are odd, even and one, at 2, 4 and 8
    paths, with and without the full check (a second SGM's planes), for each
    grid size, against the oracle."""
    import torch
    # lanes 32 / 16: a horizontal group is 2 rows, a vertical one 4 columns
    specs = [(9, 5, 16, 4), (8, 4, 16, 4), (12, 6, 20, 8), (1, 1, 4, 4), (13, 7, 33, 2), (9, 6, 8, 8),
             (16, 3, 40, 4), (5, 10, 16, 8)]
    pairs, wants = [], []
    for k, (w, h, d, p) in enumerate(specs):
        pr = synth.make_pair(w, h, d, "RS", seed=52000 + k)
        full = k % 3 == 1
        pairs.append(dict(left=_t(pr.left, gpu), right=_t(pr.right, gpu), max_disp=d, n_paths=p, median=k % 2 == 0,
                          lrcheck=full or k % 4 == 0, lr_full=full,
                          out=torch.full((h, w), 0xABC, dtype=torch.uint16, device=gpu)))
        wants.append(oracle.sgm(pr.left, pr.right, d, 7, 86, p, median=k % 2 == 0, lr=full or k % 4 == 0,
                                lr_full=full).out)
    _say(f"batch quads, grid {grid}")
    b = Batch(7, 86)
    b.set_tuning(32, 16)
    b.set_grid(grid)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, (p, want) in enumerate(zip(pairs, wants)):
        got = p["out"].cpu().numpy()
        assert (got == want).all(), (k, specs[k], int((got != want).sum()))
    b.close()


def test_batch_u16_planes_and_generic_census(gpu):
    import torch
    specs = [(45, 30, 40, 4, True, True), (30, 45, 70, 8, False, True)]
    pairs = _pairs(specs, gpu, 700)
    _say("batch with P2=300 (u16 L_r) and a 7x5 census")
    b = Batch(5, 300, 7, 5)
    b.compute(pairs)
    torch.cuda.synchronize()
    for p in pairs:
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 5, 300, p["n_paths"], 7, 5,
                          median=p["median"], lr=p["lrcheck"]).out
        assert (p["out"].cpu().numpy() == want).all()
    b.close()


def test_workload_batch_matches_sequential_calls(gpu):
    """The 64-pair mixed batch: identical to 64 single-pair calls; oracle on a sample."""
    import torch
    items = synth.batch_items(64)
    specs = [(it["w"], it["h"], it["max_disp"], it["n_paths"], False, False) for it in items]
    pairs = _pairs(specs, gpu, 0, [(it["scene"], it["seed"]) for it in items])
    _say("64-pair workload batch")
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    seq = {}
    for k, p in enumerate(pairs):
        h, w = p["left"].shape
        key = (w, h, p["max_disp"], p["n_paths"])
        if key not in seq:
            seq[key] = SGM(w, h, p["max_disp"], 7, 86, p["n_paths"])
        one = seq[key].compute(p["left"], p["right"])
        torch.cuda.synchronize()
        assert (one.cpu().numpy() == p["out"].cpu().numpy()).all(), k
    for c in seq.values():
        c.close()
    # every pair against the oracle's digest (tests/golden/make_oracle_hashes.py)
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_hashes.json")))["batch64"]
    assert len(golden) == len(pairs)
    for k, (p, g) in enumerate(zip(pairs, golden)):
        assert (g["w"], g["h"], g["max_disp"], g["n_paths"]) == (items[k]["w"], items[k]["h"],
                                                                  items[k]["max_disp"], items[k]["n_paths"])
        assert hashlib.sha256(p["np_left"].tobytes()).hexdigest() == g["sha_left"], k
        assert hashlib.sha256(p["out"].cpu().numpy().tobytes()).hexdigest() == g["out_sha256"], k
    b.close()


def test_batch_reuse_with_smaller_batches(gpu):
    import torch
    specs = [(80, 60, 64, 8, True, True), (60, 80, 48, 4, False, True), (33, 17, 20, 2, True, False)]
    pairs = _pairs(specs, gpu, 900)
    b = Batch(7, 86)
    for n in (3, 2, 1, 3):
        _say(f"reuse round with {n} pairs")
        for p in pairs[:n]:
            p["out"].view(torch.int16).zero_()
        b.compute(pairs[:n])
        torch.cuda.synchronize()
        for p in pairs[:n]:
            want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"],
                              median=p["median"], lr=p["lrcheck"]).out
            assert (p["out"].cpu().numpy() == want).all()
    b.close()


def test_batch_rejects_invalid_items(gpu):
    import torch
    from paper_1610_04121_amd import SGMError
    pairs = _pairs([(20, 10, 8, 4, False, False)], gpu, 1)
    b = Batch(7, 86)
    bad = dict(pairs[0])
    bad["n_paths"] = 3
    with pytest.raises(SGMError):
        b.compute([pairs[0], bad])
    b.close()


def test_batch_subpixel_items(gpu):
    """Pairs with 1/16-pixel output beside integer ones in one batch."""
    import torch
    specs = [(64, 48, 40, 4, True, True), (97, 31, 64, 8, False, False), (40, 70, 130, 2, True, False)]
    pairs = _pairs(specs, gpu, 1300)
    for k, p in enumerate(pairs):
        p["subpixel"] = k != 1
    _say("batch with sub-pixel items")
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"],
                          median=p["median"], lr=p["lrcheck"], subpixel=p["subpixel"]).out
        assert (p["out"].cpu().numpy() == want).all(), k
    b.close()


def test_workload_batch_median_lr_matches_oracle_digests(gpu):
    """The 64-pair mixed batch with median + left-right check on every pair
    (the configuration the benchmark times as batched_median_lr): every pair
    against the oracle's digest and against a single-pair call."""
    import torch
    items = synth.batch_items(64)
    specs = [(it["w"], it["h"], it["max_disp"], it["n_paths"], True, True) for it in items]
    pairs = _pairs(specs, gpu, 0, [(it["scene"], it["seed"]) for it in items])
    _say("64-pair workload batch with median + LR")
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_hashes.json")))
    golden = golden["batch64_median_lr"]
    assert len(golden) == len(pairs)
    seq = {}
    for k, (p, g) in enumerate(zip(pairs, golden)):
        assert (g["w"], g["h"], g["max_disp"], g["n_paths"], g["median"], g["lr"]) == \
            (items[k]["w"], items[k]["h"], items[k]["max_disp"], items[k]["n_paths"], True, True)
        assert hashlib.sha256(p["np_left"].tobytes()).hexdigest() == g["sha_left"], k
        got = p["out"].cpu().numpy()
        assert hashlib.sha256(got.tobytes()).hexdigest() == g["out_sha256"], k
        h, w = p["left"].shape
        key = (w, h, p["max_disp"], p["n_paths"])
        if key not in seq:
            seq[key] = SGM(w, h, p["max_disp"], 7, 86, p["n_paths"], median=True, lrcheck=True)
        one = seq[key].compute(p["left"], p["right"])
        torch.cuda.synchronize()
        assert (one.cpu().numpy() == got).all(), k
    for c in seq.values():
        c.close()
    b.close()


def test_batch_item_thresholds(gpu):
    """Per-item left-right thresholds carried in the item flags."""
    import torch
    specs = [(64, 48, 40, 4, True, True), (50, 30, 32, 8, False, True), (40, 40, 24, 2, True, True)]
    pairs = _pairs(specs, gpu, 1500)
    for p, thr in zip(pairs, (0, 3, 1)):
        p["lr_threshold"] = thr
    _say("batch with per-item thresholds")
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"],
                          median=p["median"], lr=p["lrcheck"], lr_thr=p["lr_threshold"]).out
        assert (p["out"].cpu().numpy() == want).all(), k
    b.close()


def test_batch_full_check_and_adaptive_items(gpu):
    """Items with the full left-right check (a second SGM with the right image
    as base) and with the adaptive P2, beside plain ones, in one batch: each
    against the oracle with the same options."""
    import torch
    specs = [(64, 48, 40, 4, True, True), (97, 31, 64, 8, False, True), (40, 70, 130, 2, True, True),
             (33, 33, 200, 8, True, True), (50, 20, 16, 4, False, False), (120, 20, 70, 8, True, True)]
    opts = [(True, False, False), (False, True, False), (True, True, True), (True, False, True),
            (False, True, False), (False, False, False)]  # (lr_full, adaptive, subpixel)
    pairs = _pairs(specs, gpu, 1700)
    for p, (lf, ad, sub) in zip(pairs, opts):
        p["lr_full"], p["adaptive_p2"], p["subpixel"] = lf and p["lrcheck"], ad, sub
    _say("batch with full-check and adaptive-P2 items")
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"], median=p["median"],
                          lr=p["lrcheck"], lr_full=p["lr_full"], adaptive=p["adaptive_p2"], subpixel=p["subpixel"]).out
        got = p["out"].cpu().numpy()
        assert (got == want).all(), (k, specs[k], opts[k], int((got != want).sum()))
    b.close()


def test_batch_adaptive_items_u16_planes(gpu):
    """Adaptive P2 with P1 above P2 (16-bit planes) in a batch."""
    import torch
    specs = [(45, 30, 40, 4, True, True), (30, 45, 70, 8, False, True)]
    pairs = _pairs(specs, gpu, 1900)
    for p in pairs:
        p["adaptive_p2"] = True
    _say("batch with adaptive P2 and P1 = 200 > P2 = 100")
    b = Batch(200, 100)
    b.compute(pairs)
    torch.cuda.synchronize()
    for p in pairs:
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 200, 100, p["n_paths"], median=p["median"],
                          lr=p["lrcheck"], adaptive=True).out
        assert (p["out"].cpu().numpy() == want).all()
    b.close()


@pytest.mark.parametrize("lanes", [(16, 16), (32, 16), (16, 32), (32, 32)])
def test_batch_kernel_shapes_match_oracle(gpu, lanes):
    """Every lane shape the batch tuner can pick, on pairs of every padded
    disparity range, path count and plane type: bit-exact with the oracle."""
    import torch
    specs = [(64, 48, 40, 4, True, True), (97, 31, 64, 8, False, True), (40, 70, 130, 2, True, False),
             (33, 33, 200, 8, False, True), (120, 20, 16, 8, True, True), (50, 45, 100, 4, False, False)]
    pairs = _pairs(specs, gpu, 2300)
    pairs[3]["adaptive_p2"] = True
    pairs[1]["lr_full"] = True
    _say(f"batch with lanes {lanes}")
    b = Batch(7, 86)
    b.set_tuning(*lanes)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"], median=p["median"],
                          lr=p["lrcheck"], adaptive=p.get("adaptive_p2", False), lr_full=p.get("lr_full", False)).out
        assert (p["out"].cpu().numpy() == want).all(), (k, lanes)
    b.close()


def test_batch_autotune_picks_a_shape_and_caches(gpu, tmp_path, monkeypatch):
    import torch
    from paper_1610_04121_amd import tune
    monkeypatch.setenv("SGM_TUNE_CACHE", str(tmp_path / "tune.json"))
    specs = [(160, 90, 64, 4, True, True), (90, 160, 128, 8, False, True), (200, 60, 100, 2, True, False)]
    pairs = _pairs(specs, gpu, 2500)
    b = Batch(7, 86)
    _say("batch autotune")
    res = b.autotune(pairs)
    assert not res["cached"] and tuple(res["choice"]) in set(tune.BATCH_CANDIDATES)
    assert len(res["candidates"]) == len(tune.BATCH_CANDIDATES)
    b.compute(pairs)
    torch.cuda.synchronize()
    for p in pairs:
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"], median=p["median"],
                          lr=p["lrcheck"]).out
        assert (p["out"].cpu().numpy() == want).all()
    b.close()
    b2 = Batch(7, 86)
    res2 = b2.autotune(list(reversed(pairs)))  # the same multiset of pairs
    assert res2["cached"] and res2["choice"] == res["choice"] and (*b2.tuning, b2.grid) == tuple(res["choice"])
    b2.close()


def test_batch_graph_replays_match_direct_launches(gpu):
    """Graph replay of a mixed batch (plain, full-check, adaptive, sub-pixel
    and post-filtered items): every replay, with eager work on the stream
    between replays, new output buffers, new inputs, a second signature
    captured in between and a larger arena, equals the direct launches."""
    import torch
    specs = [(64, 48, 40, 4, True, True), (97, 31, 64, 8, False, True), (40, 70, 130, 2, True, True),
             (33, 33, 200, 8, True, False), (50, 20, 16, 4, False, False)]
    opts = [(True, False, False), (False, True, False), (True, True, True), (False, False, True),
            (False, False, False)]  # (lr_full, adaptive, subpixel)

    def make(seed0):
        pairs = _pairs(specs, gpu, seed0)
        for p, (lf, ad, sub) in zip(pairs, opts):
            p["lr_full"], p["adaptive_p2"], p["subpixel"] = lf and p["lrcheck"], ad, sub
        return pairs

    def direct(pairs):
        b = Batch(7, 86)
        want = [torch.empty_like(p["out"]) for p in pairs]
        b.compute([dict(p, out=w) for p, w in zip(pairs, want)])
        torch.cuda.synchronize()
        b.close()
        return [w.cpu().numpy() for w in want]

    pairs = make(2300)
    want = direct(pairs)
    g = Batch(7, 86, graph=True)
    scratch = torch.zeros(1 << 20, dtype=torch.float32, device=gpu)
    for rep in range(4):
        _say(f"batch graph replay {rep}")
        for p in pairs:
            p["out"].fill_(0xABC)  # so that a replay that writes nothing fails
        g.compute(pairs)
        scratch.mul_(0.5).add_(1.0)  # eager work on the same stream between replays
        torch.cuda.synchronize()
        for k, p in enumerate(pairs):
            got = p["out"].cpu().numpy()
            assert (got == want[k]).all(), (rep, k, int((got != want[k]).sum()))
        if rep == 1:  # new output buffers: the descriptors are copied again
            for p in pairs:
                p["out"] = torch.empty_like(p["out"])
    # a second signature, then new inputs under the first one again
    sub = pairs[1:3]
    want_sub = direct(sub)
    _say("batch graph: second signature")
    g.compute(sub)
    torch.cuda.synchronize()
    for k, p in enumerate(sub):
        assert (p["out"].cpu().numpy() == want_sub[k]).all(), ("sub", k)
    pairs2 = make(2400)
    want2 = direct(pairs2)
    for rep in range(2):
        _say(f"batch graph: new inputs, replay {rep}")
        g.compute(pairs2)
        torch.cuda.synchronize()
        for k, p in enumerate(pairs2):
            assert (p["out"].cpu().numpy() == want2[k]).all(), ("new inputs", rep, k)
    # a larger batch grows the arena; the first signature replays on the new one
    big = make(2500) + _pairs([(160, 120, 64, 8, True, True)], gpu, 2600)
    want_big = direct(big)
    _say("batch graph: larger batch")
    g.compute(big)
    torch.cuda.synchronize()
    for k, p in enumerate(big):
        assert (p["out"].cpu().numpy() == want_big[k]).all(), ("big", k)
    g.compute(pairs2)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs2):
        assert (p["out"].cpu().numpy() == want2[k]).all(), ("after growth", k)
    g.set_graph(False)
    g.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        assert (p["out"].cpu().numpy() == want[k]).all(), ("direct again", k)
    g.close()


@pytest.mark.parametrize("key,post", [("batch64", False), ("batch64_median_lr", True)])
def test_batch_graph_workload_matches_oracle_digests(gpu, key, post):
    """The 64-pair workload batch (without and with median + LR) through
    graph replay, three replays, against the oracle's digests."""
    import torch
    items = synth.batch_items(64)
    specs = [(it["w"], it["h"], it["max_disp"], it["n_paths"], post, post) for it in items]
    pairs = _pairs(specs, gpu, 0, [(it["scene"], it["seed"]) for it in items])
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_hashes.json")))[key]
    assert len(golden) == len(pairs)
    g = Batch(7, 86, graph=True)
    for rep in range(3):
        _say(f"64-pair batch ({key}) graph replay {rep}")
        for p in pairs:
            p["out"].fill_(0xABC)
        g.compute(pairs)
        torch.cuda.synchronize()
        for k, (p, gd) in enumerate(zip(pairs, golden)):
            assert hashlib.sha256(p["np_left"].tobytes()).hexdigest() == gd["sha_left"], k
            assert hashlib.sha256(p["out"].cpu().numpy().tobytes()).hexdigest() == gd["out_sha256"], (rep, k)
    g.close()


def test_batch_one_workgroup_grid_matches(gpu):
    """The persistent aggregation grid cut to one workgroup (one CU takes the
    whole queue) gives the same results as the full grid: no result depends
    on the order or concurrency of the work items."""
    import torch
    specs = [(64, 48, 40, 4, True, True), (97, 31, 64, 8, False, True), (40, 70, 130, 2, True, True),
             (33, 33, 200, 8, True, False)]
    opts = [(True, False), (False, True), (True, True), (False, False)]  # (lr_full, adaptive)
    pairs = _pairs(specs, gpu, 2700)
    for p, (lf, ad) in zip(pairs, opts):
        p["lr_full"], p["adaptive_p2"] = lf and p["lrcheck"], ad
    b = Batch(7, 86)
    b.compute(pairs)
    torch.cuda.synchronize()
    full = [p["out"].cpu().numpy() for p in pairs]
    _say("batch with a one-workgroup aggregation grid")
    b.set_grid(1)
    for p in pairs:
        p["out"].fill_(0xABC)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        assert (p["out"].cpu().numpy() == full[k]).all(), k
        want = oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"], median=p["median"],
                          lr=p["lrcheck"], lr_full=p["lr_full"], adaptive=p["adaptive_p2"]).out
        assert (full[k] == want).all(), k
    b.close()


@pytest.mark.parametrize("trial", range(16))
def test_fuzz_batches(gpu, trial):
    """Random batches: 1 to 10 items of random sizes (down to 1x1), ranges,
    path counts and options (median, check with its threshold, full check,
    sub-pixel output, adaptive P2, CSCT census), a random kernel shape, direct launches,
    graph replay (twice, with the default grid or one workgroup per CU) or the
    one-workgroup grid; every item against the oracle."""
    import torch
    rng = np.random.default_rng(31000 + trial)
    n = int(rng.integers(1, 11))
    pairs, wants = [], []
    for k in range(n):
        w, h = int(rng.integers(1, 121)), int(rng.integers(1, 61))
        d = int(rng.choice([1, 5, 16, 33, 64, 65, 100, 128, 129, 200, 256]))
        p = int(rng.choice([2, 4, 8]))
        med, lr, sub, adapt, csct = (bool(rng.integers(0, 2)) for _ in range(5))
        full = lr and bool(rng.integers(0, 2))
        thr = int(rng.integers(0, 4))
        if k % 3 == 0:
            pr = synth.make_pair(w, h, d, "RS", seed=31000 + 100 * trial + k)
            l_, r_ = pr.left, pr.right
        else:
            l_ = rng.integers(0, 256, (h, w), dtype=np.uint8)
            r_ = rng.integers(0, 256, (h, w), dtype=np.uint8)
        pairs.append(dict(left=_t(l_, gpu), right=_t(r_, gpu), max_disp=d, n_paths=p, median=med, lrcheck=lr,
                          lr_threshold=thr, lr_full=full, subpixel=sub, adaptive_p2=adapt, csct=csct,
                          out=torch.full((h, w), 0xABC, dtype=torch.uint16, device=gpu)))
        wants.append(oracle.sgm(l_, r_, d, 7, 86, p, median=med, lr=lr, lr_thr=thr, lr_full=full, subpixel=sub,
                                adaptive=adapt, csct=csct).out)
    lanes = [(0, 0), (16, 16), (32, 16), (16, 32), (32, 32)][trial % 5]
    mode = ["direct", "graph", "grid1", "graph_grid256"][trial % 4]
    _say(f"batch fuzz {trial}: {n} items, lanes={lanes}, mode={mode}")
    b = Batch(7, 86, graph=mode.startswith("graph"))
    b.set_tuning(*lanes)
    if mode == "grid1":
        b.set_grid(1)
    if mode == "graph_grid256":
        b.set_grid(256)
    for rep in range(2 if mode.startswith("graph") else 1):
        for p in pairs:
            p["out"].fill_(0xABC)
        b.compute(pairs)
        torch.cuda.synchronize()
        for k, (p, want) in enumerate(zip(pairs, wants)):
            got = p["out"].cpu().numpy()
            assert (got == want).all(), (rep, k, p["left"].shape, p["max_disp"], p["n_paths"],
                                         int((got != want).sum()))
    b.close()

"""Parity of the HIP pipeline (through the C ABI) with the CPU oracle.

All arithmetic is integer, so every comparison is exact equality.  Stage
taps (census words, summed costs S, raw left/right disparities) localise a
mismatch; the whole-pipeline cases cover the benchmark workloads at full size
and a seeded fuzz over shapes, disparity ranges, path counts, census kinds,
penalties and post-filters, including the degenerate cases (1-pixel-wide or
-tall images, more disparities than columns, D = 1, D = 256).
"""
import numpy as np
import pytest

import oracle
from paper_1610_04121_amd import SGM, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rand_pair(rng, W, H):
    return (rng.integers(0, 256, (H, W), dtype=np.uint8),
            rng.integers(0, 256, (H, W), dtype=np.uint8))


@pytest.mark.parametrize("W,H,cw,ch,csct", [
    (40, 30, 9, 7, False), (40, 30, 9, 7, True), (5, 3, 9, 7, False), (1, 1, 9, 7, True),
    (300, 17, 9, 7, False), (33, 21, 5, 5, True), (33, 21, 7, 9, False), (70, 3, 3, 3, False),
])
def test_census_parity(gpu, W, H, cw, ch, csct):
    rng = np.random.default_rng(W * 1000 + H + cw)
    img = rng.integers(0, 256, (H, W), dtype=np.uint8)
    img[: H // 2, : W // 2] = 77  # ties
    _say(f"census {W}x{H} {cw}x{ch} csct={csct}")
    s = SGM(W, H, 8, 7, 86, 4, cw, ch, csct=csct)
    got = _np(s.debug_census(_t(img, gpu)))
    s.close()
    want = oracle.census(img, cw, ch, csct)
    assert (got == want).all()


# (lanes_h, lanes_v, fused aggregation, one census + cost launch)
TUNINGS = [(0, 0, True, False), (16, 16, True, False), (32, 32, True, False), (64, 16, True, False),
           (64, 32, True, False), (32, 16, False, False), (16, 16, False, False), (64, 32, False, False),
           (32, 16, False, True), (16, 16, False, True)]


@pytest.mark.parametrize("tuning", TUNINGS)
@pytest.mark.parametrize("W,H,D,P,csct", [
    (37, 23, 16, 4, False), (29, 31, 20, 8, True), (70, 9, 130, 8, False), (5, 1, 256, 2, False),
    (130, 40, 64, 8, False),
])
def test_cost_and_per_direction_parity(gpu, W, H, D, P, csct, tuning):
    rng = np.random.default_rng(W * 3 + H + D)
    l, r = _rand_pair(rng, W, H)
    _say(f"stages {W}x{H} D={D} P={P} csct={csct} tuning={tuning}")
    s = SGM(W, H, D, 7, 86, P, csct=csct)
    s.set_tuning(*tuning)
    tl, tr = _t(l, gpu), _t(r, gpu)
    cost = _np(s.debug_stage(tl, tr, -1))
    cl, cr = oracle.census(l, csct=csct), oracle.census(r, csct=csct)
    mc = oracle.cost_volume(cl, cr, D, oracle.cmax_of(csct=csct))
    bad = np.argwhere(cost != mc)
    assert len(bad) == 0, f"cost: {len(bad)} cells differ, first {bad[:5].tolist()}"
    for k, (rx, ry) in enumerate(oracle.directions(P)):
        got = _np(s.debug_stage(tl, tr, k))
        want = oracle.aggregate(mc, 7, 86, rx, ry)
        bad = np.argwhere(got != want)
        assert len(bad) == 0, (f"L_r ({rx},{ry}): {len(bad)} cells differ, first {bad[:5].tolist()} "
                               f"got {got[tuple(bad[0])] if len(bad) else None} want {want[tuple(bad[0])] if len(bad) else None}")
    s.close()


@pytest.mark.parametrize("W,H,D,P,csct,P1,P2", [
    (37, 23, 16, 4, False, 7, 86), (29, 31, 20, 8, True, 3, 40), (64, 40, 64, 4, False, 7, 86),
    (50, 45, 130, 8, False, 7, 86), (21, 70, 9, 2, False, 0, 0), (70, 9, 256, 8, False, 10, 300),
    (1, 9, 5, 8, False, 7, 86), (9, 1, 12, 8, True, 7, 86), (3, 3, 1, 4, False, 7, 86),
])
def test_summed_costs_parity(gpu, W, H, D, P, csct, P1, P2):
    rng = np.random.default_rng(W * 7 + H * 13 + D)
    l, r = _rand_pair(rng, W, H)
    _say(f"sums {W}x{H} D={D} P={P} csct={csct} P1={P1} P2={P2}")
    s = SGM(W, H, D, P1, P2, P, csct=csct)
    got = _np(s.debug_sums(_t(l, gpu), _t(r, gpu)))
    s.close()
    want = oracle.sgm(l, r, D, P1, P2, P, csct=csct, keep_sums=True).S
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"{len(bad)} cells differ, first {bad[:5].tolist()}"


@pytest.mark.parametrize("W,H,D,P,csct,P1,P2", [
    (45, 33, 40, 8, False, 60000, 7),    # P1 far above P2 (byte planes)
    (38, 41, 100, 4, False, 500, 193),   # Cmax + P2 = 255: the byte-plane limit
    (50, 20, 64, 8, True, 300, 224),     # CSCT: Cmax + P2 = 255
    (30, 30, 128, 2, False, 0, 193),     # P1 = 0
    (40, 25, 48, 4, False, 9000, 194),   # Cmax + P2 = 256: 16-bit planes
])
@pytest.mark.parametrize("fused", [False, True])
def test_penalty_extremes_per_direction(gpu, W, H, D, P, csct, P1, P2, fused):
    """Every direction's L_r and the output at the ends of the penalty range:
    P1 above P2 (it can never win against m + P2), P2 at the largest value
    byte planes hold, and just past it."""
    rng = np.random.default_rng(W * 11 + H + P1 + P2)
    l, r = _rand_pair(rng, W, H)
    _say(f"penalties {W}x{H} D={D} P={P} csct={csct} P1={P1} P2={P2} fused={fused}")
    s = SGM(W, H, D, P1, P2, P, csct=csct, median=True, lrcheck=True)
    s.set_tuning(0, 0, fused, False)
    tl, tr = _t(l, gpu), _t(r, gpu)
    mc = oracle.cost_volume(oracle.census(l, csct=csct), oracle.census(r, csct=csct), D,
                            oracle.cmax_of(csct=csct))
    for k, (rx, ry) in enumerate(oracle.directions(P)):
        got = _np(s.debug_stage(tl, tr, k))
        want = oracle.aggregate(mc, P1, P2, rx, ry)
        bad = np.argwhere(got != want)
        assert len(bad) == 0, f"L_r ({rx},{ry}): {len(bad)} cells differ, first {bad[:5].tolist()}"
    got = _np(s.compute(tl, tr))
    s.close()
    want = oracle.sgm(l, r, D, P1, P2, P, csct=csct, median=True, lr=True).out
    assert (got == want).all()


@pytest.mark.parametrize("W,H,D,P", [(41, 27, 24, 4), (66, 19, 70, 8), (8, 12, 30, 4)])
def test_raw_disparity_parity(gpu, W, H, D, P):
    rng = np.random.default_rng(W + H + D)
    l, r = _rand_pair(rng, W, H)
    _say(f"raw disparity {W}x{H} D={D} P={P}")
    s = SGM(W, H, D, 7, 86, P)
    dl, dr = s.debug_raw_disparity(_t(l, gpu), _t(r, gpu))
    dl, dr = _np(dl), _np(dr)
    s.close()
    want = oracle.sgm(l, r, D, 7, 86, P, lr=True)
    assert (dl == want.dl_raw).all()
    assert (dr == want.dr_raw).all()


@pytest.mark.parametrize("fused,census_cost,final_pass,post_in_wta", [
    (True, False, False, False), (False, False, False, False), (False, True, False, False),
    (False, False, True, False), (False, True, True, False), (False, True, False, True),
    (True, False, False, True)])
@pytest.mark.parametrize("name", list(synth.WORKLOADS))
def test_workload_full_size_bit_exact(gpu, name, fused, census_cost, final_pass, post_in_wta):
    cfg = synth.WORKLOADS[name]
    pair = synth.workload_pair(name)
    _say(f"workload {name} fused={fused} census_cost={census_cost} final_pass={final_pass} "
         f"post_in_wta={post_in_wta}")
    s = SGM(cfg["w"], cfg["h"], cfg["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, cfg["n_paths"],
            median=cfg["median"], lrcheck=cfg["lr"])
    s.set_tuning(0, 0, fused, census_cost, final_pass, post_in_wta)
    got = _np(s.compute(_t(pair.left, gpu), _t(pair.right, gpu)))
    s.close()
    want = oracle.sgm(pair.left, pair.right, cfg["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT,
                      cfg["n_paths"], median=cfg["median"], lr=cfg["lr"]).out
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"{len(bad)} pixels differ, first {bad[:5].tolist()}"


@pytest.mark.parametrize("trial", range(24))
def test_fuzz_pipeline(gpu, trial):
    rng = np.random.default_rng(9000 + trial)
    W, H = int(rng.integers(1, 71)), int(rng.integers(1, 71))
    D = int(rng.integers(1, 131)) if trial % 6 else int(rng.choice([1, 64, 128, 256]))
    P = int(rng.choice([2, 4, 8]))
    csct = bool(rng.integers(0, 2))
    cmax = 31 if csct else 62
    P1 = int(rng.integers(0, 20))
    P2 = int(rng.integers(0, 65535 // P - cmax + 1)) if trial % 4 == 3 else int(rng.integers(P1, 200))
    med, lr = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
    thr = int(rng.integers(0, 3))
    l, r = _rand_pair(rng, W, H)
    if trial % 5 == 0:
        l = (l // 64 * 64).astype(np.uint8)  # many ties
    tuning = TUNINGS[trial % len(TUNINGS)]
    _say(f"fuzz {trial}: {W}x{H} D={D} P={P} csct={csct} P1={P1} P2={P2} med={med} lr={lr} thr={thr} "
         f"tuning={tuning}")
    s = SGM(W, H, D, P1, P2, P, median=med, lrcheck=lr, csct=csct, lr_threshold=thr)
    s.set_tuning(*tuning)
    got = _np(s.compute(_t(l, gpu), _t(r, gpu)))
    s.close()
    want = oracle.sgm(l, r, D, P1, P2, P, median=med, lr=lr, csct=csct, lr_thr=thr).out
    assert (got == want).all()


def test_repeat_and_two_contexts_identical(gpu):
    pair = synth.make_pair(200, 120, 48, "RS", seed=77)
    _say("repeatability 200x120 D=48")
    a = SGM(200, 120, 48, 7, 86, 8, median=True, lrcheck=True)
    b = SGM(200, 120, 48, 7, 86, 8, median=True, lrcheck=True)
    l, r = _t(pair.left, gpu), _t(pair.right, gpu)
    o1 = _np(a.compute(l, r))
    o2 = _np(a.compute(l, r))
    o3 = _np(b.compute(l, r))
    a.close()
    b.close()
    assert (o1 == o2).all() and (o1 == o3).all()


def test_invalid_calls_raise_before_enqueue(gpu):
    import torch
    from paper_1610_04121_amd import SGMError
    with pytest.raises(SGMError):
        SGM(0, 10, 8)
    s = SGM(32, 16, 8)
    l = torch.zeros((16, 32), dtype=torch.uint8, device=gpu)
    with pytest.raises(ValueError):
        s.compute(l, torch.zeros((16, 31), dtype=torch.uint8, device=gpu))
    with pytest.raises(SGMError):
        s.set_options(lr_threshold=-1)
    s.close()


def test_graph_replay_matches_eager(gpu):
    """Graph mode: several buffer sets, each replayed several times with eager
    work and synchronisation in between; every replay equals the eager run."""
    import torch
    W, H, D = 160, 96, 48
    pairs = [synth.make_pair(W, H, D, "RS", seed=500 + i) for i in range(3)]
    eager = SGM(W, H, D, 7, 86, 8, median=True, lrcheck=True)
    graph = SGM(W, H, D, 7, 86, 8, median=True, lrcheck=True, graph=True)
    bufs = [(_t(p.left, gpu), _t(p.right, gpu), torch.empty((H, W), dtype=torch.uint16, device=gpu))
            for p in pairs]
    want = [_np(eager.compute(l, r)) for l, r, _ in bufs]
    for rep in range(4):
        _say(f"graph replay round {rep}")
        for i, (l, r, o) in enumerate(bufs):
            o.view(torch.int16).zero_()
            graph.compute(l, r, o)
            eager.compute(l, r)  # eager work between replays
            assert (_np(o) == want[i]).all(), (rep, i)
    eager.close()
    graph.close()


@pytest.mark.parametrize("cw,ch,csct,D", [(7, 5, False, 40), (5, 5, True, 70), (9, 7, True, 256), (3, 3, False, 1)])
def test_pipeline_census_windows(gpu, cw, ch, csct, D):
    """Other census windows take the census kernel + cost kernel route; 9x7
    takes the fused census + cost kernel (CSCT and full)."""
    rng = np.random.default_rng(cw * 100 + ch + D)
    l, r = _rand_pair(rng, 300, 37)
    _say(f"census window {cw}x{ch} csct={csct} D={D}")
    s = SGM(300, 37, D, 7, 86, 8, cw, ch, median=True, lrcheck=True, csct=csct)
    s.set_tuning(0, 0, False, True)  # one census + cost launch where the window allows it
    got = _np(s.compute(_t(l, gpu), _t(r, gpu)))
    cost = _np(s.debug_stage(_t(l, gpu), _t(r, gpu), -1))
    s.close()
    want = oracle.sgm(l, r, D, 7, 86, 8, cw, ch, median=True, lr=True, csct=csct).out
    assert (got == want).all()
    mc = oracle.cost_volume(oracle.census(l, cw, ch, csct), oracle.census(r, cw, ch, csct), D,
                            oracle.cmax_of(cw, ch, csct))
    assert (cost == mc).all()


def test_widest_image_with_right_view(gpu):
    """The largest width (16000): the right-view keys of a row fill almost
    all of the 64 KiB of LDS the WTA may use."""
    rng = np.random.default_rng(16000)
    l, r = _rand_pair(rng, 16000, 5)
    _say("16000x5 D=256 2 paths median+LR")
    s = SGM(16000, 5, 256, 7, 86, 2, median=True, lrcheck=True)
    got = _np(s.compute(_t(l, gpu), _t(r, gpu)))
    dl, dr = s.debug_raw_disparity(_t(l, gpu), _t(r, gpu))
    s.close()
    want = oracle.sgm(l, r, 256, 7, 86, 2, median=True, lr=True)
    assert (_np(dr) == want.dr_raw).all()
    assert (got == want.out).all()


@pytest.mark.parametrize("W,H,D,P,csct,median", [
    (37, 23, 16, 4, False, True), (29, 31, 20, 8, True, False), (70, 9, 130, 2, False, True),
    (5, 1, 256, 8, False, False), (130, 40, 64, 8, False, True), (1, 9, 5, 4, False, True),
])
def test_full_lr_check_parity(gpu, W, H, D, P, csct, median):
    """SGM_LR_FULL: right-base costs, right-base L_r of every direction, the
    right map and the final output, each against the oracle."""
    rng = np.random.default_rng(W * 11 + H + D + P)
    l, r = _rand_pair(rng, W, H)
    _say(f"full LR {W}x{H} D={D} P={P} csct={csct} median={median}")
    s = SGM(W, H, D, 7, 86, P, median=median, lrcheck=True, csct=csct, lr_full=True)
    tl, tr = _t(l, gpu), _t(r, gpu)
    cl, cr = oracle.census(l, csct=csct), oracle.census(r, csct=csct)
    cR = oracle.cost_volume_right(cr, cl, D, oracle.cmax_of(csct=csct))
    assert (_np(s.debug_stage(tl, tr, -2)) == cR).all()
    for k, (rx, ry) in enumerate(oracle.directions(P)):
        assert (_np(s.debug_stage(tl, tr, P + k)) == oracle.aggregate(cR, 7, 86, rx, ry)).all(), (rx, ry)
    want = oracle.sgm(l, r, D, 7, 86, P, median=median, lr=True, csct=csct, lr_full=True)
    dl, dr = s.debug_raw_disparity(tl, tr)
    assert (_np(dl) == want.dl_raw).all()
    assert (_np(dr) == want.dr_raw).all()
    assert (_np(s.compute(tl, tr)) == want.out).all()
    s.close()


def test_full_lr_check_headline_workload(gpu):
    """640x480, D=128, 4 paths, median, full left-right check, full size."""
    cfg = synth.WORKLOADS["vga_640x480_d128_p4"]
    pair = synth.workload_pair("vga_640x480_d128_p4")
    _say("headline workload with the full left-right check")
    s = SGM(cfg["w"], cfg["h"], cfg["max_disp"], 7, 86, cfg["n_paths"], median=True, lrcheck=True, lr_full=True)
    got = _np(s.compute(_t(pair.left, gpu), _t(pair.right, gpu)))
    s.close()
    want = oracle.sgm(pair.left, pair.right, cfg["max_disp"], 7, 86, cfg["n_paths"], median=True, lr=True,
                      lr_full=True).out
    assert (got == want).all()


def test_full_lr_check_switch_on_existing_context(gpu):
    """Turning the option on after creation grows the workspace; turning it
    off again gives the plain check back."""
    rng = np.random.default_rng(5)
    l, r = _rand_pair(rng, 90, 50)
    s = SGM(90, 50, 40, 7, 86, 8, median=True, lrcheck=True)
    tl, tr = _t(l, gpu), _t(r, gpu)
    plain = _np(s.compute(tl, tr))
    s.set_options(median=True, lrcheck=True, lr_full=True)
    full = _np(s.compute(tl, tr))
    s.set_options(median=True, lrcheck=True)
    again = _np(s.compute(tl, tr))
    s.close()
    assert (plain == oracle.sgm(l, r, 40, 7, 86, 8, median=True, lr=True).out).all()
    assert (full == oracle.sgm(l, r, 40, 7, 86, 8, median=True, lr=True, lr_full=True).out).all()
    assert (again == plain).all()


@pytest.mark.parametrize("W,H,D,P,median,lr,lr_full,csct", [
    (37, 23, 16, 4, False, False, False, False), (29, 31, 20, 8, True, True, False, True),
    (70, 9, 130, 2, True, False, False, False), (5, 1, 256, 8, False, True, False, False),
    (130, 40, 64, 8, True, True, True, False), (1, 9, 5, 4, True, True, False, False),
    (64, 48, 3, 4, False, True, True, False), (90, 33, 200, 4, True, True, False, False),
])
def test_subpixel_parity(gpu, W, H, D, P, median, lr, lr_full, csct):
    """SGM_SUBPIXEL: the 1/16-pixel left map (raw) and the output, with and
    without median and check, against the oracle."""
    rng = np.random.default_rng(W * 5 + H * 3 + D)
    l, r = _rand_pair(rng, W, H)
    if D > 8:  # smoother pairs so that minima have curvature
        pr = synth.make_pair(W, H, D, "RS", seed=W + H + D)
        l, r = pr.left, pr.right
    _say(f"subpixel {W}x{H} D={D} P={P} median={median} lr={lr} lr_full={lr_full} csct={csct}")
    s = SGM(W, H, D, 7, 86, P, median=median, lrcheck=lr, lr_full=lr_full, csct=csct, subpixel=True)
    tl, tr = _t(l, gpu), _t(r, gpu)
    got = _np(s.compute(tl, tr))
    dl, dr = s.debug_raw_disparity(tl, tr)
    s.close()
    want = oracle.sgm(l, r, D, 7, 86, P, median=median, lr=lr, lr_full=lr_full, csct=csct, subpixel=True)
    assert (_np(dl) == want.dl_raw).all()
    assert (got == want.out).all()


def test_subpixel_headline_workload(gpu):
    cfg = synth.WORKLOADS["vga_640x480_d128_p4"]
    pair = synth.workload_pair("vga_640x480_d128_p4")
    _say("headline workload with sub-pixel output")
    s = SGM(cfg["w"], cfg["h"], cfg["max_disp"], 7, 86, cfg["n_paths"], median=True, lrcheck=True, subpixel=True)
    got = _np(s.compute(_t(pair.left, gpu), _t(pair.right, gpu)))
    s.close()
    want = oracle.sgm(pair.left, pair.right, cfg["max_disp"], 7, 86, cfg["n_paths"], median=True, lr=True,
                      subpixel=True).out
    assert (got == want).all()


@pytest.mark.parametrize("tuning", [(0, 0, False, False), (16, 16, False, False), (64, 32, False, False),
                                    (32, 32, True, False)])
@pytest.mark.parametrize("W,H,D,P", [(37, 23, 16, 8), (70, 9, 130, 4), (130, 40, 64, 8), (5, 33, 256, 2)])
def test_adaptive_p2_per_direction_parity(gpu, W, H, D, P, tuning):
    """SGM_ADAPTIVE_P2: every direction's L_r against the oracle with the
    per-step P2 of the base image (a fused tuning falls back to the cost
    volume)."""
    pr = synth.make_pair(W, H, D, "RS", seed=W * H + D)
    l, r = pr.left, pr.right
    _say(f"adaptive P2 {W}x{H} D={D} P={P} tuning={tuning}")
    s = SGM(W, H, D, 7, 86, P, adaptive_p2=True)
    s.set_tuning(*tuning)
    tl, tr = _t(l, gpu), _t(r, gpu)
    mc = oracle.cost_volume(oracle.census(l), oracle.census(r), D, 62)
    for k, (rx, ry) in enumerate(oracle.directions(P)):
        got = _np(s.debug_stage(tl, tr, k))
        want = oracle.aggregate(mc, 7, 86, rx, ry, img=l)
        bad = np.argwhere(got != want)
        assert len(bad) == 0, f"L_r ({rx},{ry}): {len(bad)} cells differ, first {bad[:3].tolist()}"
    s.close()


@pytest.mark.parametrize("W,H,D,P,median,lr,lr_full,subpixel", [
    (64, 48, 32, 4, True, True, False, False), (97, 31, 64, 8, False, True, True, False),
    (40, 70, 130, 2, True, False, False, True), (200, 60, 48, 8, True, True, True, True),
])
def test_adaptive_p2_pipeline_parity(gpu, W, H, D, P, median, lr, lr_full, subpixel):
    pr = synth.make_pair(W, H, D, "RS", seed=W + 7 * H)
    _say(f"adaptive P2 pipeline {W}x{H} D={D} P={P} median={median} lr={lr} full={lr_full} sub={subpixel}")
    s = SGM(W, H, D, 7, 86, P, median=median, lrcheck=lr, lr_full=lr_full, subpixel=subpixel, adaptive_p2=True)
    got = _np(s.compute(_t(pr.left, gpu), _t(pr.right, gpu)))
    s.close()
    want = oracle.sgm(pr.left, pr.right, D, 7, 86, P, median=median, lr=lr, lr_full=lr_full, subpixel=subpixel,
                      adaptive=True).out
    assert (got == want).all()


@pytest.mark.parametrize("W,H,D,P", [(53, 29, 32, 4), (24, 61, 64, 8)])
def test_adaptive_p2_with_p1_above_p2(gpu, W, H, D, P):
    """With P1 > P2 a step's adaptive penalty max(P1, P2 / (1 + g)) can be P1,
    so L_r reaches Cmax + P1: here 62 + 200 > 255 >= 62 + 100, and the
    planes must be 16-bit although Cmax + P2 fits a byte."""
    pr = synth.make_pair(W, H, D, "RS", seed=W * 5 + H)
    l, r = pr.left, pr.right
    _say(f"adaptive P2 with P1 > P2 {W}x{H} D={D} P={P}")
    s = SGM(W, H, D, 200, 100, P, median=True, lrcheck=True, adaptive_p2=True)
    tl, tr = _t(l, gpu), _t(r, gpu)
    mc = oracle.cost_volume(oracle.census(l), oracle.census(r), D, 62)
    top = 0
    for k, (rx, ry) in enumerate(oracle.directions(P)):
        got = _np(s.debug_stage(tl, tr, k))
        want = oracle.aggregate(mc, 200, 100, rx, ry, img=l)
        top = max(top, int(want.max()))
        bad = np.argwhere(got != want)
        assert len(bad) == 0, f"L_r ({rx},{ry}): {len(bad)} cells differ, first {bad[:3].tolist()}"
    assert top > 255  # the case the byte planes could not hold
    got = _np(s.compute(tl, tr))
    s.close()
    want = oracle.sgm(l, r, D, 200, 100, P, median=True, lr=True, adaptive=True).out
    assert (got == want).all()


def test_adaptive_p2_headline_workload(gpu):
    cfg = synth.WORKLOADS["vga_640x480_d128_p4"]
    pair = synth.workload_pair("vga_640x480_d128_p4")
    _say("headline workload with adaptive P2")
    s = SGM(cfg["w"], cfg["h"], cfg["max_disp"], 7, 86, cfg["n_paths"], median=True, lrcheck=True, adaptive_p2=True)
    got = _np(s.compute(_t(pair.left, gpu), _t(pair.right, gpu)))
    s.close()
    want = oracle.sgm(pair.left, pair.right, cfg["max_disp"], 7, 86, cfg["n_paths"], median=True, lr=True,
                      adaptive=True).out
    assert (got == want).all()


def test_graph_replay_with_all_options(gpu):
    """Graph replay of the two-SGM pipeline with sub-pixel output and
    adaptive P2: every replay equals the oracle, with eager work between."""
    import torch
    W, H, D = 120, 72, 40
    pairs = [synth.make_pair(W, H, D, "RS", seed=800 + i) for i in range(2)]
    opts = dict(median=True, lrcheck=True, lr_full=True, subpixel=True, adaptive_p2=True)
    graph = SGM(W, H, D, 7, 86, 8, graph=True, **opts)
    eager = SGM(W, H, D, 7, 86, 8, **opts)
    bufs = [(_t(p.left, gpu), _t(p.right, gpu), torch.empty((H, W), dtype=torch.uint16, device=gpu)) for p in pairs]
    want = [oracle.sgm(p.left, p.right, D, 7, 86, 8, median=True, lr=True, lr_full=True, subpixel=True,
                       adaptive=True).out for p in pairs]
    for rep in range(3):
        _say(f"graph replay with all options, round {rep}")
        for i, (l, r, o) in enumerate(bufs):
            o.view(torch.int16).zero_()
            graph.compute(l, r, o)
            eager.compute(l, r)
            assert (_np(o) == want[i]).all(), (rep, i)
    graph.close()
    eager.close()


@pytest.mark.parametrize("P", [2, 4, 8])
def test_paths_sweep_full_size_every_kernel_shape(gpu, P):
    """The headline pair at each path count of the benchmark's path sweep, with
    every kernel shape the autotuner may pick for it (the sweep times the
    tuner's choice): bit-exact with the oracle at full size."""
    cfg = synth.WORKLOADS["vga_640x480_d128_p4"]
    pair = synth.workload_pair("vga_640x480_d128_p4")
    want = oracle.sgm(pair.left, pair.right, cfg["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, P,
                      median=cfg["median"], lr=cfg["lr"]).out
    tl, tr = _t(pair.left, gpu), _t(pair.right, gpu)
    s = SGM(cfg["w"], cfg["h"], cfg["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, P,
            median=cfg["median"], lrcheck=cfg["lr"])
    for gh, gv in [(16, 16), (32, 16), (32, 32), (64, 16), (64, 32)]:
        for census_cost in (False, True):
            for final_pass in (False, True):
                _say(f"path sweep P={P} lanes=({gh},{gv}) census_cost={census_cost} final_pass={final_pass}")
                s.set_tuning(gh, gv, False, census_cost, final_pass)
                got = _np(s.compute(tl, tr))
                bad = np.argwhere(got != want)
                assert len(bad) == 0, (gh, gv, census_cost, final_pass,
                                       f"{len(bad)} pixels differ, first {bad[:5].tolist()}")
    s.close()


@pytest.mark.parametrize("final_pass,lanes_h", [(False, 0), (True, 32), (True, 64)])
@pytest.mark.parametrize("W,H,D,P,csct", [
    (37, 23, 16, 4, False), (29, 31, 20, 8, True), (70, 9, 130, 2, False), (64, 40, 64, 8, False),
    (1, 5, 7, 4, False), (5, 1, 256, 2, False), (203, 3, 200, 8, False),
])
def test_phase_sums_parity(gpu, W, H, D, P, csct, final_pass, lanes_h):
    """sgm_debug_phase_sums: phase 0 sums every direction but the one the
    final pass fuses (right-to-left; left-to-right with 2 paths), phase 1
    all of them; with the final pass on, phase 1 is the sum the fused kernel
    forms from the stored planes and its own recurrence."""
    rng = np.random.default_rng(W * 5 + H * 3 + D)
    l, r = _rand_pair(rng, W, H)
    _say(f"phase sums {W}x{H} D={D} P={P} csct={csct} final_pass={final_pass} lanes_h={lanes_h}")
    s = SGM(W, H, D, 7, 86, P, csct=csct)
    s.set_tuning(lanes_h, 16 if lanes_h else 0, False, False, final_pass)
    tl, tr = _t(l, gpu), _t(r, gpu)
    cl, cr = oracle.census(l, csct=csct), oracle.census(r, csct=csct)
    mc = oracle.cost_volume(cl, cr, D, oracle.cmax_of(csct=csct))
    dirs = oracle.directions(P)
    last = (1, 0) if P == 2 else (-1, 0)
    s0 = sum(oracle.aggregate(mc, 7, 86, rx, ry).astype(np.int64) for rx, ry in dirs if (rx, ry) != last)
    s1 = s0 + oracle.aggregate(mc, 7, 86, *last)
    for phase, want in ((0, s0), (1, s1)):
        got = _np(s.debug_phase_sums(tl, tr, phase))
        bad = np.argwhere(got != want)
        assert len(bad) == 0, (phase, f"{len(bad)} cells differ, first {bad[:5].tolist()}")
    s.close()


@pytest.mark.parametrize("trial", range(24))
def test_fuzz_pipeline_final_pass(gpu, trial):
    """The final pass (last direction fused with the sum and the winner-take-
    all) on fuzzed shapes and options, against the oracle, for both of its
    lane widths; raw maps through the debug tap as well."""
    rng = np.random.default_rng(19000 + trial)
    W, H = int(rng.integers(1, 90)), int(rng.integers(1, 40))
    D = int(rng.choice([1, 7, 16, 40, 64, 65, 100, 128, 130, 200, 256]))
    P = int(rng.choice([2, 4, 8]))
    med, lr, sub, csct = (bool(rng.integers(0, 2)) for _ in range(4))
    thr = int(rng.integers(0, 3))
    gh = int(rng.choice([32, 64]))
    l, r = _rand_pair(rng, W, H)
    if trial % 3 == 0:  # textured pairs with a shift, so that disparities vary
        pr = synth.make_pair(W, H, D, "RS", seed=19000 + trial)
        l, r = pr.left, pr.right
    _say(f"final pass fuzz {trial}: {W}x{H} D={D} P={P} med={med} lr={lr} sub={sub} csct={csct} thr={thr} gh={gh}")
    s = SGM(W, H, D, 7, 86, P, median=med, lrcheck=lr, csct=csct, lr_threshold=thr, subpixel=sub)
    s.set_tuning(gh, 16, False, False, True)
    tl, tr = _t(l, gpu), _t(r, gpu)
    got = _np(s.compute(tl, tr))
    want = oracle.sgm(l, r, D, 7, 86, P, median=med, lr=lr, csct=csct, lr_thr=thr, subpixel=sub)
    bad = np.argwhere(got != want.out)
    assert len(bad) == 0, f"{len(bad)} pixels differ, first {bad[:5].tolist()}"
    dl, dr = s.debug_raw_disparity(tl, tr)
    want_raw = oracle.sgm(l, r, D, 7, 86, P, lr=True, csct=csct, subpixel=sub)
    assert (_np(dl) == want_raw.dl_raw).all()
    assert (_np(dr) == want_raw.dr_raw).all()
    s.close()


@pytest.mark.parametrize("trial", range(24))
def test_fuzz_post_in_wta(gpu, trial):
    """The median and left-right check inside the winner-take-all launch (the
    block completing a row's neighbourhood filters it) on fuzzed shapes and
    options, including the full check's two-SGM launch, against the oracle;
    every frame is computed twice so that the row counters left by one frame
    are shown to be clear for the next."""
    rng = np.random.default_rng(23000 + trial)
    W, H = int(rng.integers(1, 120)), int(rng.integers(1, 50))
    if trial < 3:
        H = trial + 1  # one to three rows: rows with fewer neighbours
    D = int(rng.choice([1, 7, 16, 40, 64, 65, 100, 128, 130, 200, 256]))
    P = int(rng.choice([2, 4, 8]))
    med, lr, sub, csct = (bool(rng.integers(0, 2)) for _ in range(4))
    if not (med or lr):
        med = True
    full = lr and bool(rng.integers(0, 2))
    adapt = bool(rng.integers(0, 2))
    thr = int(rng.integers(0, 3))
    tuning = TUNINGS[trial % len(TUNINGS)]
    l, r = _rand_pair(rng, W, H)
    if trial % 3 == 0:
        pr = synth.make_pair(W, H, D, "RS", seed=23000 + trial)
        l, r = pr.left, pr.right
    _say(f"post-in-wta fuzz {trial}: {W}x{H} D={D} P={P} med={med} lr={lr} full={full} sub={sub} csct={csct} "
         f"adapt={adapt} thr={thr} tuning={tuning}")
    s = SGM(W, H, D, 7, 86, P, median=med, lrcheck=lr, csct=csct, lr_threshold=thr, subpixel=sub,
            lr_full=full, adaptive_p2=adapt)
    s.set_tuning(*tuning, False, True)
    assert s.tuning()[5]
    tl, tr = _t(l, gpu), _t(r, gpu)
    want = oracle.sgm(l, r, D, 7, 86, P, median=med, lr=lr, csct=csct, lr_thr=thr, subpixel=sub, lr_full=full,
                      adaptive=adapt).out
    for rep in range(2):
        got = _np(s.compute(tl, tr))
        bad = np.argwhere(got != want)
        assert len(bad) == 0, (rep, f"{len(bad)} pixels differ, first {bad[:5].tolist()}")
    s.close()

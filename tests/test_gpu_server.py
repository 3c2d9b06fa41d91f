"""Request server: results are the same alone and in a mix of concurrent
requests (exact equality), admission never exceeds the memory budget, and the
failure paths (full queue, cancellation, oversize requests, shutdown with work
queued) behave as documented."""
import hashlib
import json
import os
import threading

import numpy as np
import pytest

import oracle
from paper_1610_04121_amd import SGM, SGMError, synth
from paper_1610_04121_amd.sgm import (REQ_CANCELED, REQ_DONE, SGM_EBUSY, SGM_EINVAL, SGM_ENOMEM, Server)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _req(dev, w, h, d, p, med, lr, seed, scene="RS"):
    import torch
    pr = synth.make_pair(w, h, d, scene, seed=seed)
    return dict(left=torch.from_numpy(pr.left).to(dev), right=torch.from_numpy(pr.right).to(dev),
                max_disp=d, n_paths=p, median=med, lrcheck=lr, lr_threshold=1,
                out=torch.zeros((h, w), dtype=torch.uint16, device=dev), np_left=pr.left, np_right=pr.right)


def _alone(req):
    """The same pair through a single-pair context, on its own."""
    import torch
    h, w = req["left"].shape
    c = SGM(w, h, req["max_disp"], 7, 86, req["n_paths"], median=req["median"], lrcheck=req["lrcheck"],
            subpixel=req.get("subpixel", False), lr_full=req.get("lr_full", False),
            adaptive_p2=req.get("adaptive_p2", False))
    out = c.compute(req["left"], req["right"])
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    c.close()
    return res


@pytest.mark.parametrize("slots,streams", [(4, 2), (4, 4), (2, 1)])
def test_mixed_concurrent_requests_match_alone(gpu, slots, streams):
    import torch
    rng = np.random.default_rng(44)
    shapes = [(64, 48), (160, 90), (320, 240), (97, 31), (33, 65), (640, 480)]
    reqs = []
    for k in range(24):
        w, h = shapes[k % len(shapes)]
        reqs.append(_req(gpu, w, h, int(rng.choice([16, 64, 128, 200])), int(rng.choice([2, 4, 8])),
                         bool(rng.integers(0, 2)), bool(rng.integers(0, 2)), 1000 + k))
        reqs[-1]["subpixel"] = k % 3 == 0
    srv = Server(8 << 30, slots=slots, streams=streams, max_group=4, max_group_cells=1 << 40)
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            tickets[i] = srv.submit(reqs[i])

    _say(f"24 requests from two submitting threads, {slots} slots on {streams} streams")
    th = [threading.Thread(target=submit, args=(range(j, len(reqs), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, t in enumerate(tickets):
        st, lat = srv.wait(t, 60000)
        assert st == REQ_DONE and lat is not None and lat > 0, (i, st)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["groups"] < len(reqs)  # some requests were batched together
    assert stats["peak_bytes"] <= stats["budget_bytes"]
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        got = r["out"].cpu().numpy()
        assert (got == _alone(r)).all(), i
    for i in (0, 3, 7):  # small ones against the oracle as well
        r = reqs[i]
        want = oracle.sgm(r["np_left"], r["np_right"], r["max_disp"], 7, 86, r["n_paths"],
                          median=r["median"], lr=r["lrcheck"], subpixel=r["subpixel"]).out
        assert (reqs[i]["out"].cpu().numpy() == want).all(), i


def test_admission_respects_memory_budget(gpu):
    reqs = [_req(gpu, 320, 240, 128, 8, True, True, 50 + k) for k in range(6)]
    probe = Server(1 << 30, slots=1)
    one = probe.request_bytes(reqs[0])
    probe.close()
    budget = 2 * one + one // 2  # two requests fit at a time, never three
    srv = Server(budget, slots=4, streams=4, max_group=8)
    _say(f"budget {budget} bytes, {one} per request")
    ts = [srv.submit(r) for r in reqs]
    for t in ts:
        assert srv.wait(t, 60000)[0] == REQ_DONE
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= 2 * one
    assert st["completed"] == 6
    want = _alone(reqs[0])
    assert (reqs[0]["out"].cpu().numpy() == want).all()


def test_large_requests_run_alone(gpu):
    """Requests above the group cell limit are never grouped; small ones are."""
    big = [_req(gpu, 640, 480, 128, 8, False, False, 60 + k) for k in range(4)]  # 315M cells each
    small = [_req(gpu, 64, 48, 32, 4, False, False, 80 + k) for k in range(6)]
    srv = Server(16 << 30, slots=1, max_group=8, max_group_cells=1 << 28)
    ts = [srv.submit(r) for r in big]
    for t in ts:
        assert srv.wait(t, 60000)[0] == REQ_DONE
    st = srv.stats()
    assert st["groups"] == 4 and st["grouped_requests"] == 4
    ts = [srv.submit(r) for r in [big[0]] + small]  # the small ones queue behind a big one
    for t in ts:
        assert srv.wait(t, 60000)[0] == REQ_DONE
    st = srv.stats()
    srv.close()
    assert st["groups"] < 4 + 7
    for r in small[:2]:
        assert (r["out"].cpu().numpy() == _alone(r)).all()


def test_oversize_and_invalid_requests_rejected(gpu):
    srv = Server(1 << 20, slots=1)
    big = _req(gpu, 320, 240, 64, 4, False, False, 5)
    with pytest.raises(SGMError) as e:
        srv.submit(big)
    assert e.value.code == SGM_ENOMEM
    bad = dict(big)
    bad["max_disp"] = 300
    with pytest.raises(SGMError) as e:
        srv.submit(bad)
    assert e.value.code == SGM_EINVAL
    with pytest.raises(SGMError):
        srv.poll(12345)
    srv.close()


def _busy_server(gpu, n_big):
    """One slot, groups of one, occupied by large requests."""
    big = [_req(gpu, 1920, 1080, 256, 8, True, True, 70 + k, scene="R") for k in range(n_big)]
    srv = Server(48 << 30, slots=1, max_group=1)
    return srv, big


def test_queue_full_and_cancel(gpu):
    import torch
    srv, big = _busy_server(gpu, 4)
    _say("four 1920x1080 D=256 requests on one slot")
    ts = [srv.submit(r) for r in big]
    # at least two are still queued behind the first: each takes milliseconds
    assert srv.stats()["submitted"] == 4
    srv.set_policy(max_group=1, max_pending=1)
    extra = _req(gpu, 64, 48, 16, 4, False, False, 9)
    with pytest.raises(SGMError) as e:
        srv.submit(extra)
    assert e.value.code == SGM_EBUSY
    srv.cancel(ts[3])
    assert srv.poll(ts[3])[0] == REQ_CANCELED
    for t in ts[:3]:
        assert srv.wait(t, 60000)[0] == REQ_DONE
    st = srv.stats()
    srv.close()
    assert st["rejected"] == 1 and st["canceled"] == 1 and st["completed"] == 3
    torch.cuda.synchronize()
    assert (big[3]["out"].view(torch.int16).cpu().numpy() == 0).all()  # never ran
    assert (big[0]["out"].cpu().numpy() == _alone(big[0])).all()


def test_shutdown_with_queued_work(gpu):
    import torch
    srv, big = _busy_server(gpu, 3)
    _say("destroy with requests queued")
    for r in big:
        srv.submit(r)
    srv.close()  # cancels what has not started, waits for the rest
    # the device is still usable afterwards
    r = _req(gpu, 64, 48, 16, 4, True, True, 3)
    s2 = Server(1 << 30, slots=2)
    assert s2.wait(s2.submit(r), 60000)[0] == REQ_DONE
    s2.close()
    torch.cuda.synchronize()
    assert (r["out"].cpu().numpy() == _alone(r)).all()


@pytest.mark.parametrize("grouped", [False, True])
def test_served_mix_full_size_against_oracle_digests(gpu, grouped):
    """Every (size, disparity range) of the served mix, up to 1920x1080 with
    D=256, 8 paths, median + LR, submitted together; each output against the
    oracle's digest (tests/golden/make_oracle_hashes.py).  grouped=True
    forces the batched kernels, False the single-pair kernels."""
    import torch
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_hashes.json")))["serve_kinds"]
    kinds = synth.serve_kinds()
    assert len(golden) == len(kinds)
    reqs = []
    for k, g in zip(kinds, golden):
        pr = synth.spec_pair(k)
        assert pr.sha_left == g["sha_left"] and pr.sha_right == g["sha_right"]
        reqs.append(dict(left=torch.from_numpy(pr.left).to(gpu), right=torch.from_numpy(pr.right).to(gpu),
                         max_disp=k["max_disp"], n_paths=8, median=True, lrcheck=True, lr_threshold=1,
                         out=torch.zeros((k["h"], k["w"]), dtype=torch.uint16, device=gpu)))
    _say(f"served mix at full size, grouped={grouped}")
    srv = Server(48 << 30, slots=4, max_group=8, max_group_cells=(1 << 40) if grouped else (1 << 28))
    ts = [srv.submit(r) for r in reqs]
    for t in ts:
        assert srv.wait(t, 120000)[0] == REQ_DONE
    st = srv.stats()
    srv.close()
    if grouped:
        assert st["groups"] < len(reqs)
    torch.cuda.synchronize()
    for r, g in zip(reqs, golden):
        got = r["out"].cpu().numpy()
        assert hashlib.sha256(got.tobytes()).hexdigest() == g["out_sha256"], (g["w"], g["h"], g["max_disp"])


def test_served_full_check_and_adaptive_requests(gpu):
    """Requests with the full left-right check and with the adaptive P2, in
    groups and alone: each against the oracle with the same options."""
    import torch
    reqs = []
    for k, (w, h, d, p) in enumerate([(96, 64, 48, 8), (160, 90, 100, 4), (64, 48, 32, 2), (97, 31, 64, 8),
                                      (120, 40, 130, 4), (33, 65, 20, 8)]):
        r = _req(gpu, w, h, d, p, True, True, 2100 + k)
        r["lr_full"] = k % 2 == 0
        r["adaptive_p2"] = k % 3 != 2
        reqs.append(r)
    _say("served full-check and adaptive-P2 requests")
    srv = Server(4 << 30, slots=2, max_group=4, max_group_cells=1 << 40, overlap_queue=1)
    ts = [srv.submit(r) for r in reqs]
    for t in ts:
        assert srv.wait(t, 60000)[0] == REQ_DONE
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    torch.cuda.synchronize()
    for k, r in enumerate(reqs):
        want = oracle.sgm(r["np_left"], r["np_right"], r["max_disp"], 7, 86, r["n_paths"], median=True, lr=True,
                          lr_full=r["lr_full"], adaptive=r["adaptive_p2"]).out
        assert (r["out"].cpu().numpy() == want).all(), k


@pytest.mark.parametrize("trial", range(4))
def test_fuzz_served_requests(gpu, trial):
    """Random small requests (sizes down to 1x1, any range, paths and
    options) from two submitting threads under a random group policy and
    slot / stream count; every result against the oracle."""
    import torch
    rng = np.random.default_rng(41000 + trial)
    reqs = []
    for k in range(24):
        w, h = int(rng.integers(1, 100)), int(rng.integers(1, 50))
        d = int(rng.choice([1, 8, 16, 40, 64, 65, 128, 200, 256]))
        p = int(rng.choice([2, 4, 8]))
        med, lr = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
        r = _req(gpu, w, h, d, p, med, lr, 41000 + 100 * trial + k)
        r["lr_full"] = lr and bool(rng.integers(0, 2))
        r["adaptive_p2"] = bool(rng.integers(0, 2))
        r["subpixel"] = bool(rng.integers(0, 2))
        r["lr_threshold"] = int(rng.integers(0, 3))
        r["csct"] = bool(rng.integers(0, 2))
        reqs.append(r)
    slots = int(rng.choice([1, 2, 4]))
    streams = int(rng.integers(1, slots + 1))
    max_group = int(rng.choice([1, 4, 32]))
    overlap = int(rng.choice([1, 3]))
    _say(f"served fuzz {trial}: slots={slots} streams={streams} max_group={max_group} overlap={overlap}")
    srv = Server(2 << 30, slots=slots, streams=streams, max_group=max_group, max_group_cells=1 << 40,
                 overlap_queue=overlap)
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            tickets[i] = srv.submit(reqs[i])

    th = [threading.Thread(target=submit, args=(range(j, len(reqs), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, t in enumerate(tickets):
        assert srv.wait(t, 60000)[0] == REQ_DONE, i
    srv.close()
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        want = oracle.sgm(r["np_left"], r["np_right"], r["max_disp"], 7, 86, r["n_paths"], median=r["median"],
                          lr=r["lrcheck"], lr_thr=r["lr_threshold"], lr_full=r["lr_full"],
                          adaptive=r["adaptive_p2"], subpixel=r["subpixel"], csct=r["csct"]).out
        got = r["out"].cpu().numpy()
        assert (got == want).all(), (i, r["left"].shape, r["max_disp"], int((got != want).sum()))

"""Failure handling forced from the host: allocations that fail through the
library's allocation-failure hook (sgm_debug_fail_alloc).  Every kernel
still runs to completion; a failed call launches nothing, and the calls and
requests after it are unaffected (exact equality with the oracle or with a
single-pair context)."""
import numpy as np
import pytest

import oracle
from paper_1610_04121_amd import SGM, SGMError, synth
from paper_1610_04121_amd.sgm import REQ_DONE, REQ_FAILED, SGM_ENOMEM, Batch, Server, debug_fail_alloc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture
def hook():
    debug_fail_alloc(0, 0)
    yield debug_fail_alloc
    debug_fail_alloc(0, 0)


def _pair(w, h, d, seed):
    return synth.make_pair(w, h, d, "RS", seed=seed)


def test_context_creation_fails_then_recovers(gpu, hook):
    pr = _pair(64, 48, 32, 31)
    _say("context: failed workspace allocation")
    hook(0, 1)
    with pytest.raises(SGMError) as ei:
        SGM(64, 48, 32, 7, 86, 4)
    assert "workspace" in str(ei.value) and "out of memory" in str(ei.value)
    c = SGM(64, 48, 32, 7, 86, 4, median=True, lrcheck=True)
    got = c.compute(_t(pr.left, gpu), _t(pr.right, gpu)).cpu().numpy()
    c.close()
    assert (got == oracle.sgm(pr.left, pr.right, 32, 7, 86, 4, median=True, lr=True).out).all()


def test_workspace_growth_failure_keeps_the_old_options(gpu, hook):
    """The full check needs a larger workspace; when that allocation fails the
    context keeps its options and workspace and computes as before."""
    pr = _pair(80, 40, 48, 32)
    c = SGM(80, 40, 48, 7, 86, 4, median=True)
    l, r = _t(pr.left, gpu), _t(pr.right, gpu)
    _say("context: failed growth for the full check")
    hook(0, 1)
    try:
        c.set_options(median=True, lrcheck=True, lr_full=True)
        grew = True
    except SGMError as e:
        assert e.code == SGM_ENOMEM
        grew = False
    hook(0, 0)
    got = c.compute(l, r).cpu().numpy()
    want = oracle.sgm(pr.left, pr.right, 48, 7, 86, 4, median=True, lr=grew, lr_full=grew).out
    assert (got == want).all()
    c.close()


def test_batch_allocation_failures_then_recovery(gpu, hook):
    import torch
    specs = [(64, 48, 40, 4), (97, 31, 64, 8), (40, 70, 130, 2)]
    pairs = []
    for k, (w, h, d, p) in enumerate(specs):
        pr = _pair(w, h, d, 40 + k)
        pairs.append(dict(left=_t(pr.left, gpu), right=_t(pr.right, gpu), max_disp=d, n_paths=p, median=True,
                          lrcheck=True, out=torch.full((h, w), 0xABC, dtype=torch.uint16, device=gpu),
                          np_left=pr.left, np_right=pr.right))
    wants = [oracle.sgm(p["np_left"], p["np_right"], p["max_disp"], 7, 86, p["n_paths"], median=True, lr=True).out
             for p in pairs]
    # a new runner's first batch allocates the arena, then the pinned and the
    # device descriptor table, then the pinned and the device work table
    for after in range(5):
        b = Batch(7, 86)
        _say(f"batch: allocation {after} of the first batch fails")
        hook(after, 1)
        with pytest.raises(SGMError) as ei:
            b.compute(pairs)
        assert ei.value.code == SGM_ENOMEM
        hook(0, 0)
        b.compute(pairs)
        torch.cuda.synchronize()
        for k, p in enumerate(pairs):
            assert (p["out"].cpu().numpy() == wants[k]).all(), (after, k)
            p["out"].fill_(0xABC)
        b.close()
    b = Batch(7, 86)
    b.set_graph(True)
    _say("batch: graph tables fail to allocate")
    hook(0, 1)
    with pytest.raises(SGMError) as ei:
        b.compute(pairs)
    assert ei.value.code == SGM_ENOMEM
    hook(0, 0)
    b.compute(pairs)
    torch.cuda.synchronize()
    for k, p in enumerate(pairs):
        assert (p["out"].cpu().numpy() == wants[k]).all(), k
    b.close()


def test_server_group_allocation_failure_is_isolated(gpu, hook):
    """A group whose descriptor tables cannot be allocated fails as a whole
    (SGM_REQ_FAILED); requests before and after it complete exactly."""
    import torch
    big = []
    for k in range(2):  # long requests that keep the one slot busy while the rest queue
        pr = _pair(1920, 1080, 256, 60 + k)
        big.append(dict(left=_t(pr.left, gpu), right=_t(pr.right, gpu), max_disp=256, n_paths=8,
                        out=torch.zeros((1080, 1920), dtype=torch.uint16, device=gpu), np=pr))
    small = []
    for k in range(16):
        w, h, d = (64, 48, 32) if k % 2 else (97, 31, 64)
        pr = _pair(w, h, d, 70 + k)
        small.append(dict(left=_t(pr.left, gpu), right=_t(pr.right, gpu), max_disp=d, n_paths=4, median=True,
                          lrcheck=True, out=torch.zeros((h, w), dtype=torch.uint16, device=gpu), np=pr))
    srv = Server(16 << 30, slots=1, max_group=4, max_group_cells=1 << 40)
    _say("server: the first grouped dispatch fails to allocate")
    hook(0, 1)
    tickets = [srv.submit(r) for r in big + small]
    states = [srv.wait(t, 60000)[0] for t in tickets]
    hook(0, 0)
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    assert all(s in (REQ_DONE, REQ_FAILED) for s in states), states
    failed = [i for i, s in enumerate(states) if s == REQ_FAILED]
    # exactly one group: 2 to 4 requests taken from the queue head in order
    assert 2 <= len(failed) <= 4 and stats["failed"] == len(failed), (failed, stats)
    assert failed == list(range(failed[0], failed[0] + len(failed))), failed
    for i, r in enumerate(big + small):
        if i in failed:
            continue
        p = r["np"]
        want = oracle.sgm(p.left, p.right, r["max_disp"], 7, 86, r["n_paths"], median=r.get("median", False),
                          lr=r.get("lrcheck", False)).out if i >= 2 else None
        got = r["out"].cpu().numpy()
        if want is not None:
            assert (got == want).all(), i
        else:
            c = SGM(1920, 1080, 256, 7, 86, 8)
            alone = c.compute(r["left"], r["right"]).cpu().numpy()
            c.close()
            assert (got == alone).all(), i


def test_server_watchdog_fails_a_stuck_group_and_drains_it(gpu):
    """A 1 ms watchdog declares a group of a few ms stuck: its request fails
    at once, its workspace stays reserved until the device completes the
    group (which still writes the exact result), and with the watchdog off
    the next request completes normally."""
    import time

    import torch
    pr = _pair(1920, 1080, 256, 90)
    big = dict(left=_t(pr.left, gpu), right=_t(pr.right, gpu), max_disp=256, n_paths=8,
               out=torch.zeros((1080, 1920), dtype=torch.uint16, device=gpu))
    srv = Server(16 << 30, slots=1, max_group=1)
    srv.set_watchdog(1)
    _say("server watchdog: a 1920x1080, D=256, 8-path request under a 1 ms limit")
    t = srv.submit(big)
    st, _ = srv.wait(t, 60000)
    assert st == REQ_FAILED
    stats = srv.stats()
    assert stats["timed_out"] == 1 and stats["failed"] == 1
    deadline = time.time() + 20
    while srv.stats()["draining_groups"] and time.time() < deadline:
        time.sleep(0.001)
    stats = srv.stats()
    assert stats["draining_groups"] == 0 and stats["bytes_in_use"] == 0, stats
    torch.cuda.synchronize()
    c = SGM(1920, 1080, 256, 7, 86, 8)
    alone = c.compute(big["left"], big["right"]).cpu().numpy()
    c.close()
    assert (big["out"].cpu().numpy() == alone).all()  # the device finished the stuck group
    srv.set_watchdog(0)
    pr2 = _pair(97, 31, 64, 91)
    small = dict(left=_t(pr2.left, gpu), right=_t(pr2.right, gpu), max_disp=64, n_paths=4, median=True,
                 lrcheck=True, out=torch.zeros((31, 97), dtype=torch.uint16, device=gpu))
    t2 = srv.submit(small)
    assert srv.wait(t2, 60000)[0] == REQ_DONE
    srv.close()
    want = oracle.sgm(pr2.left, pr2.right, 64, 7, 86, 4, median=True, lr=True).out
    assert (small["out"].cpu().numpy() == want).all()

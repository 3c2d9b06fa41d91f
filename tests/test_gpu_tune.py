"""Autotuner: picks a valid kernel shape, leaves results unchanged, caches."""
import pytest

from paper_1610_04121_amd import SGM, synth, tune

pytestmark = pytest.mark.gpu


def test_autotune_picks_candidate_and_caches(gpu, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("SGM_TUNE_CACHE", str(tmp_path / "tune.json"))
    pair = synth.make_pair(200, 120, 100, "RS", seed=5)
    l = torch.from_numpy(pair.left).to(gpu)
    r = torch.from_numpy(pair.right).to(gpu)
    print("autotune 200x120 D=100", flush=True)
    ref = SGM(200, 120, 100, 7, 86, 8, median=True, lrcheck=True)
    want = ref.compute(l, r).cpu().numpy()
    ref.close()
    s = SGM(200, 120, 100, 7, 86, 8, median=True, lrcheck=True)
    res = s.autotune(l, r, reps=3, rounds=1)
    assert not res["cached"]
    assert tuple(res["choice"]) in set(tune.candidates(100))
    assert len(res["candidates"]) == len(tune.candidates(100))
    s.set_tuning(32, 16, False, True)  # one census + cost launch
    assert (s.compute(l, r).cpu().numpy() == want).all()
    s.set_tuning(*res["choice"])
    assert s.tuning() == tuple(res["choice"])
    assert (s.compute(l, r).cpu().numpy() == want).all()
    s.close()
    s2 = SGM(200, 120, 100, 7, 86, 8, median=True, lrcheck=True)
    res2 = s2.autotune()
    assert res2["cached"] and res2["choice"] == res["choice"]
    assert s2.tuning() == tuple(res["choice"])
    s2.close()


def test_sgm_tune_environment_sets_the_initial_shape(gpu, monkeypatch):
    import torch

    import oracle
    from paper_1610_04121_amd import SGM, synth
    pr = synth.make_pair(96, 40, 48, "RS", seed=5150)
    l = torch.from_numpy(pr.left).to(gpu)
    r = torch.from_numpy(pr.right).to(gpu)
    want = oracle.sgm(pr.left, pr.right, 48, 7, 86, 4, median=True, lr=True).out
    monkeypatch.setenv("SGM_TUNE", "32,32,2")  # one census + cost launch
    s = SGM(96, 40, 48, 7, 86, 4, median=True, lrcheck=True)
    assert s.tuning() == (32, 32, False, True, False, False)
    assert (s.compute(l, r).cpu().numpy() == want).all()
    s.close()
    # rejected lanes, a shape that does not exist, too few fields, unknown bit, junk
    for bad in ("16,24,0", "16,32,0", "32,16", "32,16,64", "x"):
        monkeypatch.setenv("SGM_TUNE", bad)
        s = SGM(96, 40, 48, 7, 86, 4, median=True, lrcheck=True)
        default = s.tuning()
        assert default[2:] == (False, False, False, False), (bad, default)
        assert (s.compute(l, r).cpu().numpy() == want).all()
        s.close()

"""sgm_compute_noalloc (workspace in the library's static device scratch)
against sgm_compute (workspace from sgm_create) on the same inputs: bit-exact,
on two calls in a row, the second with a smaller input, so the second call
runs on what the first left in the scratch."""
import numpy as np
import pytest

from paper_1610_04121_amd import SGM, synth
from paper_1610_04121_amd.sgm import compute_noalloc

pytestmark = pytest.mark.gpu


def _run_pair(gpu, w, h, d, P, seed, **opts):
    import torch
    pair = synth.make_pair(w, h, d, "RS", seed=seed)
    left = torch.from_numpy(pair.left).to(gpu)
    right = torch.from_numpy(pair.right).to(gpu)
    print(f"noalloc: {w}x{h} D={d} P={P} {opts}", flush=True)
    got = compute_noalloc(left, right, d, 7, 86, P, **opts)
    ctx = SGM(w, h, d, 7, 86, P, median=opts.get("median", False), lrcheck=opts.get("lrcheck", False),
              lr_full=opts.get("lr_full", False), subpixel=opts.get("subpixel", False),
              adaptive_p2=opts.get("adaptive_p2", False))
    want = ctx.compute(left, right)
    torch.cuda.synchronize()
    ctx.close()
    g, wv = got.cpu().numpy(), want.cpu().numpy()
    assert np.array_equal(g, wv), int((g != wv).sum())
    return g


def test_noalloc_matches_sgm_compute_two_calls_second_smaller(gpu):
    # the headline shape, then a smaller one with other options on the same scratch
    _run_pair(gpu, 640, 480, 128, 4, 1610041501, median=True, lrcheck=True)
    _run_pair(gpu, 97, 61, 40, 8, 1610041502, median=True, lrcheck=True, subpixel=True)


def test_noalloc_options_and_ragged_shapes(gpu):
    _run_pair(gpu, 131, 37, 70, 2, 1610041503, lrcheck=True, lr_full=True)
    _run_pair(gpu, 33, 90, 200, 8, 1610041504, median=True, adaptive_p2=True)
    _run_pair(gpu, 1, 7, 5, 4, 1610041505)


def test_noalloc_rejects_a_workspace_beyond_the_scratch(gpu):
    import torch
    from paper_1610_04121_amd import SGMError
    from paper_1610_04121_amd.sgm import SGM_ENOMEM
    left = torch.zeros((1080, 1920), dtype=torch.uint8, device=gpu)
    with pytest.raises(SGMError) as e:
        compute_noalloc(left, left, 256, 7, 86, 8)
    assert e.value.code == SGM_ENOMEM

"""Autotuner for the aggregation kernel shape of a context.

The aggregation runs one group of G lanes per scanline slice (G = 16, 32 or
64 for horizontal slices, 16 or 32 for the others; each lane holds D/G
disparities), either reading the stored cost volume or computing costs from
census words (fused).  None of this changes a result; the best shape depends
on the image size, the disparity range and the path count.  The tuner times
every valid shape on the caller's inputs (whole frames, HIP events on the
context's stream), checks that every shape gives the same disparities, keeps
the fastest and records it in a JSON cache keyed by the context's shape and
parameters ($SGM_TUNE_CACHE, else sgm_tune_cache.json in the temp directory).
"""
from __future__ import annotations

import json
import os
import tempfile


def padded_disp(max_disp: int) -> int:
    return 64 if max_disp <= 64 else (128 if max_disp <= 128 else 256)


def candidates(max_disp: int, census_9x7: bool = True, final_pass: bool = False, post_in_wta: bool = False):
    """(lanes_h, lanes_v, fused, census_cost, final_pass, post_in_wta) shapes the kernels
    provide for this range: the cost volume from separate census and cost
    launches or (9x7 windows) from one, or no cost volume at all (fused).
    With final_pass, the shapes with a stored cost volume are also offered
    with the last direction fused with the sum and the winner-take-all; they
    are left out by default, having measured slower on every workload (the
    fused pass runs a whole row's recurrence after the other directions)."""
    pairs = [(16, 16), (32, 16), (32, 32)]
    if padded_disp(max_disp) >= 128:
        pairs += [(64, 16), (64, 32)]
    costs = [(False, False), (True, False)] + ([(False, True)] if census_9x7 else [])
    out = []
    for gh, gv in pairs:
        for f, cc in costs:
            out.append((gh, gv, f, cc, False, post_in_wta))
            if final_pass and not f:
                out.append((gh, gv, f, cc, True, post_in_wta))
    return out


def cache_path() -> str:
    return os.environ.get("SGM_TUNE_CACHE") or os.path.join(tempfile.gettempdir(), "sgm_tune_cache.json")


def cache_key(ctx) -> str:
    p = ctx.params
    return (f"{ctx.width}x{ctx.height}:d{ctx.max_disp}:p{ctx.n_paths}:P1={p['P1']}:P2={p['P2']}:"
            f"census={p['census_w']}x{p['census_h']}:csct={int(p['csct'])}:median={int(p['median'])}:"
            f"lr={int(p['lrcheck'])}:lrfull={int(p.get('lr_full', False))}:sub={int(p.get('subpixel', False))}:"
            f"adapt={int(p.get('adaptive_p2', False))}")


def load_cache(path: str | None = None) -> dict:
    try:
        with open(path or cache_path()) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_entry(key: str, entry: dict, path: str | None = None):
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _candidates(ctx):
    p = ctx.params
    return candidates(ctx.max_disp, p["census_w"] == 9 and p["census_h"] == 7)


def _frame_ms(ctx, left, right, out, stream, reps: int) -> float:
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ctx.compute(left, right, out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(ctx, left=None, right=None, reps: int = 20, rounds: int = 2, use_cache: bool = True) -> dict:
    """Picks and applies the fastest kernel shape for ``ctx``.  ``left`` and
    ``right`` default to random images of the context's size.  Returns the
    choice, its time per frame and every candidate's time (or the cached
    entry, with ``cached`` set)."""
    import torch
    key = cache_key(ctx)
    if use_cache:
        hit = load_cache().get(key)
        if hit and tuple(hit.get("choice", ())) in set(_candidates(ctx)):  # (older entries lack a field)
            ctx.set_tuning(*hit["choice"])
            return dict(hit, cached=True)
    dev = torch.device("cuda", torch.cuda.current_device())
    if left is None:
        g = torch.Generator(device="cpu").manual_seed(1610)
        left = torch.randint(0, 256, ctx.shape, dtype=torch.uint8, generator=g).to(dev)
        right = torch.roll(left, shifts=ctx.max_disp // 4, dims=1)
    stream = torch.cuda.current_stream()
    out = torch.empty(ctx.shape, dtype=torch.uint16, device=dev)
    ref = None
    times = {}
    for _ in range(rounds):
        for cand in _candidates(ctx):
            ctx.set_tuning(*cand)
            ctx.compute(left, right, out, stream=stream)  # warm-up, and the result check
            stream.synchronize()
            if ref is None:
                ref = out.clone()
            elif not torch.equal(out, ref):
                raise RuntimeError(f"kernel shape {cand} changed the disparities")
            t = _frame_ms(ctx, left, right, out, stream, reps)
            times[cand] = min(times.get(cand, float("inf")), t)
    best = min(times, key=times.get)
    ctx.set_tuning(*best)
    entry = {"choice": list(best), "ms_per_frame": round(times[best], 5),
             "candidates": {",".join(str(int(v)) for v in cand): round(t, 5) for cand, t in times.items()}}
    if use_cache:
        try:
            save_entry(key, entry)
        except OSError:
            pass  # a read-only cache location only costs a re-tune later
    return dict(entry, cached=False)


# (lanes per horizontal slice, lanes per other slice, aggregation workgroups).
# Workgroups 0 lets the persistent grid hold up to two wavefronts per SIMD,
# which hides the latency of one slice's min-plus chain behind another's
# when the queue is long; 256 keeps one wavefront per SIMD (one workgroup per
# CU), which wins when a few long slices set the launch time and would
# otherwise share a SIMD with other slices (two 640x240 pairs at D = 128:
# 64 -> 59 us for the aggregation).
BATCH_LANES = [(0, 0), (16, 16), (32, 16), (16, 32), (32, 32)]
BATCH_GRIDS = [0, 256]
BATCH_CANDIDATES = [(gh, gv, g) for g in BATCH_GRIDS for (gh, gv) in BATCH_LANES]


def batch_key(batch, pairs) -> str:
    """Cache key of a batch: its parameters and the multiset of its pairs'
    shapes and options (the order of the pairs does not change the work)."""
    import hashlib
    p = batch.params
    sig = sorted((tuple(q["left"].shape), q["max_disp"], q["n_paths"], bool(q.get("median")), bool(q.get("lrcheck")),
                  bool(q.get("subpixel")), bool(q.get("lr_full")), bool(q.get("adaptive_p2")), bool(q.get("csct")),
                  int(q.get("lr_threshold", 1))) for q in pairs)
    h = hashlib.sha256(repr(sig).encode()).hexdigest()[:16]
    return f"batch:{len(pairs)}:{h}:P1={p['P1']}:P2={p['P2']}:census={p['census_w']}x{p['census_h']}"


def _apply_batch(batch, cand):
    gh, gv, grid = cand
    batch.set_tuning(gh, gv)
    batch.set_grid(grid)


def autotune_batch(batch, pairs, reps: int = 3, rounds: int = 1, use_cache: bool = True) -> dict:
    """Picks and applies the fastest batched-aggregation kernel shape (lanes
    per horizontal / other slice for every pair, or the per-pair default, and
    the persistent grid's workgroup count) for this set of pairs: times each
    shape on the pairs themselves (HIP events on the current stream), checks
    that every shape gives the same disparities for every pair, and caches
    the choice under batch_key()."""
    import torch
    key = batch_key(batch, pairs)
    if use_cache:
        hit = load_cache().get(key)
        if hit and tuple(hit.get("choice", ())) in set(BATCH_CANDIDATES):
            _apply_batch(batch, tuple(hit["choice"]))
            return dict(hit, cached=True)
    stream = torch.cuda.current_stream()
    ref, times = None, {}
    for _ in range(rounds):
        for cand in BATCH_CANDIDATES:
            _apply_batch(batch, cand)
            batch.compute(pairs, stream=stream)
            stream.synchronize()
            outs = [q["out"].clone() for q in pairs]
            if ref is None:
                ref = outs
            elif not all(torch.equal(a, b) for a, b in zip(outs, ref)):
                raise RuntimeError(f"batch kernel shape {cand} changed the disparities")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                batch.compute(pairs, stream=stream)
            e1.record(stream)
            e1.synchronize()
            times[cand] = min(times.get(cand, float("inf")), e0.elapsed_time(e1) / reps)
    best = min(times, key=times.get)
    _apply_batch(batch, best)
    entry = {"choice": list(best), "ms_per_batch": round(times[best], 4),
             "candidates": {",".join(map(str, c)): round(t, 4) for c, t in times.items()}}
    if use_cache:
        try:
            save_entry(key, entry)
        except OSError:
            pass
    return dict(entry, cached=False)

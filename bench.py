"""Throughput of the SGM disparity pipeline on one MI355X.

A step is one pass of the whole pipeline (census, cost volume, aggregation
along all paths, sum + winner-take-all with the right view, median,
left-right check) over one 640x480 pair with 128 disparity levels and 4
paths, inputs already resident in HBM.  The timed region keeps F frames in
flight (F contexts, each with its own workspace and stream; default F = 1,
so that the stage events time each kernel alone):
frame k runs on context k mod F.  Prints one JSON line:

  value         frames/s over the timed steps (whole job = one GPU);
  gcells_per_s  W*H*D*paths * frames/s / 1e9;
  roofline      the aggregation kernel (the dominant one) against HBM:
                algorithmic bytes per launch / its mean duration, measured
                with HIP events recorded around it on its own stream in the
                timed region, on every 8th frame of each context (with F > 1
                other frames share the GPU meanwhile);
  pipeline      census through WTA (median and LR excluded) against HBM:
                the path's algorithmic bytes per frame / the event-timed
                span of those stages;
  serialized    one frame at a time on one stream (eager and graph replay);
  latency_ms    p50/p99 of single frames, event-bracketed;
  cpu_baseline  the CPU oracle (single thread) on a bounded sample of the
                same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "vga_640x480_d128_p4"
METRIC = "frames/s and Gcells/s (W·H·D·paths) at 640x480 D=128; p50/p99 latency served"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "aggregate_vga_640x480_d128_p4_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1610_04121_amd", "csrc", f)
               for f in ("sgm_device.h", "sgm_kernels.hip", "sgm_common.h")]


def _kernel_sha() -> str:
    """Hash of the sources the single-pair kernels are built from, with
    comments and whitespace removed (edits to those do not change a kernel)."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        text = open(f).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _traffic(tuning):
    """HBM bytes per aggregation launch from committed rocprofv3 counters,
    or None if the counters were taken on another version of the kernels or
    another kernel shape."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    # the recorded shape (lanes_h, lanes_v, fused, census_cost) must match,
    # and every later tuning switch (final pass, post stage inside the WTA)
    # must be off, as in the counted runs
    ref = [int(v) for v in t.get("tuning", [])]
    cur = [int(v) for v in tuning]
    if t.get("kernel_sha") != _kernel_sha() or not ref or cur[:len(ref)] != ref or any(cur[len(ref):]):
        return None
    return t.get("bytes_per_launch")


def summarize_counters(fetch_csv: str, write_csv: str, copy_mib: int, tuning) -> dict:
    """Per-dispatch HBM bytes of every kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
    same counter reads for the device copy of copy_mib MiB that the profiled
    run made (--copy-calibration-mb): the copy dispatches with the largest
    readings (other copies, such as image uploads, are smaller).  When the run
    also made the read-only reduction of --read-calibration-mb, its FETCH_SIZE
    scale is reported as a cross-check of the read scale."""
    import csv
    from collections import defaultdict

    def rows(path, counter):
        acc = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return acc

    def calib(acc, pattern):
        vals = [v for k, vs in acc.items() if pattern in k for v in vs]
        top = max(vals)
        big = [v for v in vals if v >= 0.99 * top]
        return sum(big) / len(big)

    fr, wr = rows(fetch_csv, "FETCH_SIZE"), rows(write_csv, "WRITE_SIZE")
    fetch = {k: sum(v) / len(v) for k, v in fr.items()}
    write = {k: sum(v) / len(v) for k, v in wr.items()}
    copy_kib = copy_mib * 1024.0
    f_fetch, f_write = copy_kib / calib(fr, "copyBuffer"), copy_kib / calib(wr, "copyBuffer")
    kernels = {}
    for k in fetch:
        if "copyBuffer" in k or "at::native" in k or k not in write:
            continue
        rd, wrb = fetch[k] * f_fetch * 1024, write[k] * f_write * 1024
        kernels[k] = {"read_bytes": round(rd), "write_bytes": round(wrb), "fetch_kib": round(fetch[k], 2),
                      "write_kib": round(write[k], 2)}
    agg = next(k for k in kernels if "aggregate_kernel<" in k)
    out = {"kernel": agg, "kernel_sha": _kernel_sha(), "tuning": [int(v) for v in tuning],
           "fetch_scale": round(f_fetch, 4), "write_scale": round(f_write, 4),
           "bytes_per_launch": kernels[agg]["read_bytes"] + kernels[agg]["write_bytes"], "kernels": kernels}
    if any("reduce_kernel" in k for k in fr):
        out["fetch_scale_read_only"] = round(copy_kib / calib(fr, "reduce_kernel"), 4)
    return out


def summarize_trace(csv_path: str, skip_frac: float = 0.2, frames_range=None) -> dict:
    """Frame spans and gaps from a rocprofv3 --kernel-trace CSV of a run of
    whole frames on one stream: a frame starts at each census launch; its
    span runs from the first kernel's start to the last kernel's end, and
    the gap before each kernel is its start minus the previous kernel's end.
    frames_range (first, end) selects frames by launch order; then the first
    skip_frac of them (warm-up) is left out; medians in us."""
    import csv
    rows = []
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            name = r["Kernel_Name"]
            short = name.replace("(anonymous namespace)::", "").split("(")[0].split("<")[0].split("::")[-1]
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short))
    rows.sort()
    frames, cur = [], []
    for r in rows:
        if r[2].startswith("census") and cur:
            frames.append(cur)
            cur = []
        if r[2].startswith("census") or cur:
            cur.append(r)
    if cur:
        frames.append(cur)
    if frames_range:
        frames = frames[frames_range[0]:frames_range[1]]
    frames = frames[int(len(frames) * skip_frac):]
    if not frames:
        return {"frames": 0}
    med = lambda v: round(float(sorted(v)[len(v) // 2]) / 1e3, 3)
    spans = [f[-1][1] - f[0][0] for f in frames]
    busy = [sum(e - s for s, e, _ in f) for f in frames]
    gaps = {}
    for f in frames:
        for a, b in zip(f, f[1:]):
            gaps.setdefault(f"{a[2]} -> {b[2]}", []).append(b[0] - a[1])
    between = [b[0][0] - a[-1][1] for a, b in zip(frames, frames[1:])]
    return {"frames": len(frames), "kernels_per_frame": len(frames[0]),
            "span_us": med(spans), "kernel_time_us": med(busy), "idle_in_frame_us": med([s - b for s, b in zip(spans, busy)]),
            "gap_us": {k: med(v) for k, v in gaps.items()},
            "gap_between_frames_us": med(between) if between else None}


def pipeline_bytes(W: int, H: int, Dp: int, P: int, tuning) -> int:
    """Algorithmic bytes of census, cost, aggregation and WTA for one frame
    (each byte read or written once per kernel that needs it): images in,
    u64 census words of both views, the u8 cost volume, P u8 L_r planes
    written and read back, the raw D_L and D_R maps out.  With the final pass
    (tuning[4]) the last direction's plane is neither written nor read: the
    aggregation launch moves 2 (P - 1) N, the final pass reads the cost
    volume and the P - 1 planes."""
    px, N = W * H, W * H * Dp
    fused, census_cost = bool(tuning[2]), bool(tuning[3])
    if len(tuning) > 4 and bool(tuning[4]) and not fused:
        census, cost = (0, 2 * px + N) if census_cost else (2 * px + 16 * px, 16 * px + N)
        return census + cost + 2 * (P - 1) * N + (N + (P - 1) * N + 4 * px)
    census = 2 * px + 16 * px              # both images in, both census maps out
    if fused:                              # no cost volume: each direction reads census words
        agg = P * 16 * px + P * N
        cost = 0
    elif census_cost:                      # census words stay on chip
        census, cost, agg = 0, 2 * px + N, 2 * P * N
    else:
        cost, agg = 16 * px + N, 2 * P * N
    wta = P * N + 4 * px
    return census + cost + agg + wta


def host_cpu() -> dict:
    """The host's CPU model and core counts (for the CPU baseline's record)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "available": len(os.sched_getaffinity(0))}


def _pinned_oracle_loop(core, left, right, cfg, budget_s, conn):
    """Child process of cpu_baseline: pinned to one core, runs whole oracle
    frames for about budget_s seconds and sends (frames, seconds) back."""
    os.sched_setaffinity(0, {core})
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.sgm(left, right, cfg["max_disp"], 7, 86, cfg["n_paths"], median=cfg["median"], lr=cfg["lr"])
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    conn.send((n, time.perf_counter() - t0, sorted(os.sched_getaffinity(0))))
    conn.close()


def cpu_baseline(pair, cfg, budget_s: float = 12.0):
    """The C oracle (single-threaded, never tuned) on whole frames of the
    workload, in a spawned child process pinned to one host core with
    sched_setaffinity (the GPU process's own threads stay elsewhere)."""
    import multiprocessing as mp
    core = min(os.sched_getaffinity(0))
    ctx = mp.get_context("spawn")
    rd, wr = ctx.Pipe(duplex=False)
    p = ctx.Process(target=_pinned_oracle_loop, args=(core, pair.left, pair.right, cfg, budget_s, wr))
    p.start()
    wr.close()
    while not rd.poll(1.0):  # a child that dies never sends
        if not p.is_alive():
            raise RuntimeError(f"cpu_baseline child exited with code {p.exitcode}")
    n, dt, pinned = rd.recv()
    p.join()
    return {"value": round(n / dt, 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
            "pinned_to": pinned, "host_cpu": host_cpu(),
            "sample": f"{n} full {cfg['w']}x{cfg['h']} D={cfg['max_disp']} {cfg['n_paths']}-path "
                      f"frames ({'median + LR' if cfg['median'] else 'WTA only'}), single thread pinned to core {core}, "
                      f"{dt:.1f} s"}


def _oracle_frame(spec):
    """Seconds for one oracle frame of a pair spec (worker of oracle_timing)."""
    import oracle
    from paper_1610_04121_amd import synth
    pr = synth.spec_pair(spec)
    t0 = time.perf_counter()
    oracle.sgm(pr.left, pr.right, spec["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, spec["n_paths"],
               median=spec.get("median", False), lr=spec.get("lr", False))
    return time.perf_counter() - t0


def oracle_timing() -> dict:
    """The CPU oracle beside the GPU on every workload, on this host: single-
    thread seconds per frame of each single-pair workload (median of 3 for the
    smallest), the makespan of the 64-pair batch with one oracle process per
    core, and single-thread seconds for each (size, D) of the served mix (run
    side by side, one process each)."""
    import multiprocessing as mp

    import oracle
    from paper_1610_04121_amd import synth
    oracle.build()
    cores = min(len(os.sched_getaffinity(0)), 16)
    out = {"cores": cores, "workloads": {}, "served_kinds": []}
    for name, cfg in synth.WORKLOADS.items():
        spec = dict(w=cfg["w"], h=cfg["h"], max_disp=cfg["max_disp"], n_paths=cfg["n_paths"], scene=cfg["scene"],
                    seed=cfg["seed"], median=cfg["median"], lr=cfg["lr"])
        runs = [_oracle_frame(spec) for _ in range(3 if cfg["w"] * cfg["h"] <= 320 * 240 else 1)]
        t = sorted(runs)[len(runs) // 2]
        out["workloads"][name] = {"s_per_frame": round(t, 3), "frames_per_s": round(1 / t, 4), "runs": len(runs)}
        print(f"bench: oracle {name}: {t:.2f} s per frame", file=sys.stderr, flush=True)
    ctx = mp.get_context("spawn")
    items = [dict(it, median=False, lr=False) for it in synth.batch_items(64)]
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        per = pool.map(_oracle_frame, items, chunksize=1)
        out["batch_64"] = {"makespan_s": round(time.perf_counter() - t0, 2), "pairs_per_s": round(64 / (time.perf_counter() - t0), 3),
                           "sum_single_thread_s": round(sum(per), 1), "processes": cores}
    print(f"bench: oracle 64-pair batch: {out['batch_64']['makespan_s']} s on {cores} processes", file=sys.stderr,
          flush=True)
    kinds = synth.serve_kinds()
    with ctx.Pool(min(cores, len(kinds))) as pool:
        per = pool.map(_oracle_frame, kinds, chunksize=1)
    out["served_kinds"] = [{"size": f"{k['w']}x{k['h']}", "max_disp": k["max_disp"], "s_per_frame": round(t, 2)}
                           for k, t in zip(kinds, per)]
    return out


def bench_paths(left, right, cfg, steps: int, warmup: int = 50):
    """The paper's path-count axis: 2 (left-to-right and top-to-bottom), 4
    and 8 paths on the headline pair, one frame at a time, autotuned."""
    import torch

    from paper_1610_04121_amd import SGM, synth
    st = torch.cuda.current_stream()
    out = {}
    for P in (2, 4, 8):
        c = SGM(cfg["w"], cfg["h"], cfg["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, P,
                median=cfg["median"], lrcheck=cfg["lr"])
        c.autotune(left, right, use_cache=False, reps=10, rounds=1)
        o = torch.empty((cfg["h"], cfg["w"]), dtype=torch.uint16, device=left.device)
        for _ in range(warmup):
            c.compute(left, right, o, stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            c.compute(left, right, o, stream=st)
        torch.cuda.synchronize()
        fps = steps / (time.perf_counter() - t0)
        out[str(P)] = {"frames_per_s": round(fps, 1),
                       "gcells_per_s": round(cfg["w"] * cfg["h"] * cfg["max_disp"] * P * fps / 1e9, 1),
                       "lanes": list(c.tuning())}
        c.close()
    return out


def bench_variant(left, right, cfg, tuning, steps: int, warmup: int = 50, **opts):
    """The headline pair with other output options (the full left-right
    check, sub-pixel output), one frame at a time."""
    import torch

    from paper_1610_04121_amd import SGM, synth
    st = torch.cuda.current_stream()
    c = SGM(cfg["w"], cfg["h"], cfg["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, cfg["n_paths"],
            median=cfg["median"], lrcheck=True, **opts)
    c.set_tuning(*tuning)
    o = torch.empty((cfg["h"], cfg["w"]), dtype=torch.uint16, device=left.device)
    for _ in range(warmup):
        c.compute(left, right, o, stream=st)
    torch.cuda.synchronize()
    c.profile(True, every=32)
    t0 = time.perf_counter()
    for _ in range(steps):
        c.compute(left, right, o, stream=st)
    torch.cuda.synchronize()
    fps = steps / (time.perf_counter() - t0)
    n, stage = c.profile_read()
    c.close()
    return {"frames_per_s": round(fps, 1), "stage_ms": {k: round(v / max(n, 1), 5) for k, v in stage.items()}}


def bench_batch(dev, steps: int, warmup: int = 3, post: bool = False):
    """The 64-pair heterogeneous batch: one launch per stage through the
    batch API against 64 plain single-pair launches on one stream (post:
    every pair with median and left-right check)."""
    import torch

    from paper_1610_04121_amd import SGM, synth
    from paper_1610_04121_amd.sgm import Batch

    items = synth.batch_items(64)
    pairs, cells, alg_bytes = [], 0, 0
    for it in items:
        pr = synth.make_pair(it["w"], it["h"], it["max_disp"], it["scene"], seed=it["seed"])
        pairs.append(dict(left=torch.from_numpy(pr.left).to(dev), right=torch.from_numpy(pr.right).to(dev),
                          max_disp=it["max_disp"], n_paths=it["n_paths"], median=post, lrcheck=post,
                          out=torch.empty((it["h"], it["w"]), dtype=torch.uint16, device=dev)))
        cells += it["w"] * it["h"] * it["max_disp"] * it["n_paths"]
        Dp = 64 if it["max_disp"] <= 64 else (128 if it["max_disp"] <= 128 else 256)
        # the batch runs separate census and cost launches; the post stage
        # reads both raw maps' 3x3 neighbourhoods and writes the output
        alg_bytes += pipeline_bytes(it["w"], it["h"], Dp, it["n_paths"], (0, 0, False, False, False))
        if post:
            alg_bytes += 6 * it["w"] * it["h"]
    b = Batch(synth.P1_DEFAULT, synth.P2_DEFAULT)
    st = torch.cuda.current_stream()
    tuned = b.autotune(pairs, use_cache=False)

    def time_batch():
        for _ in range(warmup):
            b.compute(pairs, stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.compute(pairs, stream=st)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_batch = time_batch()
    b.set_graph(True)  # the same launches replayed from a captured graph
    t_graph = time_batch()
    footprint = b.footprint(pairs)
    b.close()

    ctxs = {}
    for p in pairs:
        h, w = p["left"].shape
        key = (w, h, p["max_disp"], p["n_paths"])
        if key not in ctxs:
            ctxs[key] = SGM(w, h, p["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, p["n_paths"],
                            median=post, lrcheck=post)
    seq = [(ctxs[(p["left"].shape[1], p["left"].shape[0], p["max_disp"], p["n_paths"])], p) for p in pairs]

    def run_seq():
        for c, p in seq:
            c.compute(p["left"], p["right"], p["out"], stream=st)

    for _ in range(warmup):
        run_seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_seq()
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / steps
    for c in ctxs.values():
        c.close()
    gbs = alg_bytes / t_batch / 1e9
    return {"pairs": len(pairs), "batches": steps, "ms_per_batch": round(t_batch * 1e3, 4),
            "pairs_per_s": round(len(pairs) / t_batch, 1), "gcells_per_s": round(cells / t_batch / 1e9, 1),
            "graph_ms_per_batch": round(t_graph * 1e3, 4),
            "sequential_ms": round(t_seq * 1e3, 4), "sequential_pairs_per_s": round(len(pairs) / t_seq, 1),
            "speedup_vs_sequential": round(t_seq / t_batch, 3), "workspace_bytes": footprint,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(gbs / 8000.0, 4), "alg_bytes_per_batch": alg_bytes,
                         "basis": "algorithmic bytes of census, cost, aggregation, sum + WTA"
                                  + (" and median + LR" if post else "")
                                  + " of all pairs, over the batch's wall time (direct launches)"},
            "tuning": {"lanes_h_lanes_v_grid": tuned["choice"], "ms_per_batch_by_shape": tuned["candidates"]},
            "shapes": "64 pairs, sizes from {320x240, 640x480, 1242x375, 1280x720}, D from {64, 128}, "
                      "4 or 8 paths, " + ("median + LR check" if post else "no median/LR")}


def bench_batch_small(dev, steps: int = 400, warmup: int = 20, seed: int = 1610041216):
    """A launch-bound batch: 8 small pairs (160x120 to 320x240, D 32 or 64,
    4 paths, median + LR), by direct launches, by graph replay and as 8
    plain single-pair launches on one stream."""
    import numpy as np
    import torch

    from paper_1610_04121_amd import SGM, synth
    from paper_1610_04121_amd.sgm import Batch
    rng = np.random.default_rng(seed)
    pairs = []
    for k in range(8):
        (w, h), d = [(160, 120), (256, 192), (320, 240)][k % 3], int(rng.choice([32, 64]))
        pr = synth.make_pair(w, h, d, "K", seed=seed * 10 + k, scale_to_d=True)
        pairs.append(dict(left=torch.from_numpy(pr.left).to(dev), right=torch.from_numpy(pr.right).to(dev),
                          max_disp=d, n_paths=4, median=True, lrcheck=True,
                          out=torch.empty((h, w), dtype=torch.uint16, device=dev)))
    st = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    b = Batch(synth.P1_DEFAULT, synth.P2_DEFAULT)
    t_direct = timed(lambda: b.compute(pairs, stream=st))
    b.set_graph(True)
    t_graph = timed(lambda: b.compute(pairs, stream=st))
    b.close()
    ctxs = [SGM(p["left"].shape[1], p["left"].shape[0], p["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, 4,
                median=True, lrcheck=True) for p in pairs]

    def seq():
        for c, p in zip(ctxs, pairs):
            c.compute(p["left"], p["right"], p["out"], stream=st)

    t_seq = timed(seq)
    for c in ctxs:
        c.close()
    return {"pairs": len(pairs), "ms_per_batch": round(t_direct, 4), "graph_ms_per_batch": round(t_graph, 4),
            "sequential_ms": round(t_seq, 4), "graph_speedup_vs_direct": round(t_direct / t_graph, 3),
            "shapes": "8 pairs of 160x120, 256x192 or 320x240, D 32 or 64, 4 paths, median + LR"}


def _serve_setup(dev, seed):
    """The served mix's kinds, one device-resident pair per kind."""
    import torch

    from paper_1610_04121_amd import synth
    specs = synth.serve_kinds(seed)
    pool = []
    for k in specs:
        pr = synth.spec_pair(k)
        pool.append((torch.from_numpy(pr.left).to(dev), torch.from_numpy(pr.right).to(dev)))
    return specs, pool


class _OutPool:
    """Output buffers per kind: a request holds one from its submission until
    its completion has been observed.  Taking from an empty pool first waits
    for that kind's oldest outstanding request (never the case at the sizes
    used: the pools hold more than the longest backlog)."""

    def __init__(self, dev, specs, per_kind):
        import torch
        self.free = [[torch.empty((k["h"], k["w"]), dtype=torch.uint16, device=dev) for _ in range(per_kind)]
                     for k in specs]

    def take(self, k, wait_oldest):
        if not self.free[k]:
            wait_oldest(k)
        return self.free[k].pop()

    def give(self, k, t):
        self.free[k].append(t)


def _serve_level(srv, specs, pool, outs, qps, n_req, n_warm, rng):
    """One open-loop level through the server: n_warm warm-up requests, then
    n_req measured ones, Poisson arrivals at qps.  Returns latency stats of
    the measured requests, served frames/s, rejections and the mean group
    size, plus the arrival schedule (for the plain baseline)."""
    import collections

    import numpy as np

    from paper_1610_04121_amd.sgm import FINAL, REQ_DONE, SGM_EBUSY, SGMError
    total = n_warm + n_req
    arrivals = np.cumsum(rng.exponential(1.0 / qps, total))
    which = rng.integers(0, len(specs), total)
    cells = np.array([k["w"] * k["h"] * k["max_disp"] * k["n_paths"] for k in specs], dtype=np.float64)
    outstanding = collections.deque()  # (index, kind, ticket, buffer) in submission order
    lat, done_at, rejected = {}, {}, 0

    def finish(entry, block):
        i, k, t, buf = entry
        st, l = srv.wait(t) if block else srv.poll(t)
        if st not in FINAL:
            return False
        assert st == REQ_DONE, st
        lat[i], done_at[i] = l, arrivals[i] + l
        outs.give(k, buf)
        return True

    def wait_oldest(k):
        for e in list(outstanding):
            if e[1] == k:
                finish(e, True)
                outstanding.remove(e)
                return

    g0 = srv.stats()
    t0 = time.perf_counter() + 0.005
    for i in range(total):
        if i == n_warm:
            g0 = srv.stats()
        target = t0 + arrivals[i]
        while True:
            # harvest completions while waiting for the next arrival
            while outstanding and finish(outstanding[0], False):
                outstanding.popleft()
            now = time.perf_counter()
            if now >= target:
                break
            if target - now > 2e-3:
                time.sleep(min(target - now - 1e-3, 1e-3))
        k = int(which[i])
        buf = outs.take(k, wait_oldest)
        left, right = pool[k]
        req = dict(left=left, right=right, out=buf, max_disp=specs[k]["max_disp"], n_paths=specs[k]["n_paths"],
                   median=True, lrcheck=True, lr_threshold=1)
        try:
            outstanding.append((i, k, srv.submit(req), buf))
        except SGMError as e:
            if e.code != SGM_EBUSY:
                raise
            rejected += i >= n_warm
            outs.give(k, buf)
    while outstanding:
        finish(outstanding.popleft(), True)
    g1 = srv.stats()
    meas = [i for i in range(n_warm, total) if i in lat]
    l = np.array([lat[i] for i in meas])
    span = max(done_at[i] for i in meas) - arrivals[n_warm]
    return {"p50_ms": round(float(np.percentile(l, 50)) * 1e3, 3), "p99_ms": round(float(np.percentile(l, 99)) * 1e3, 3),
            "frames_per_s": round(len(meas) / span, 1),
            "gcells_per_s": round(sum(cells[which[i]] for i in meas) / span / 1e9, 1),
            "rejected": rejected, "requests": n_req, "warmup": n_warm,
            "mean_group": round((g1["grouped_requests"] - g0["grouped_requests"]) / max(1, g1["groups"] - g0["groups"]),
                                2)}, arrivals[n_warm:] - arrivals[n_warm], which[n_warm:]


def _plain_level(ctxs, specs, pool, outs, arrivals, which, st):
    """The same arrival times through plain per-request launches: one context
    per kind, one stream, each request synchronised before the next starts."""
    import numpy as np
    cells = np.array([k["w"] * k["h"] * k["max_disp"] * k["n_paths"] for k in specs], dtype=np.float64)
    t0 = time.perf_counter() + 0.005
    plat = []
    for i in range(len(arrivals)):
        target = t0 + arrivals[i]
        while time.perf_counter() < target:
            pass
        k = int(which[i])
        buf = outs.take(k, lambda _: None)
        ctxs[k].compute(pool[k][0], pool[k][1], buf, stream=st)
        st.synchronize()
        outs.give(k, buf)
        plat.append(time.perf_counter() - target)
    span = (t0 + arrivals[-1] + plat[-1]) - t0
    return {"p50_ms": round(float(np.percentile(plat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(plat, 99)) * 1e3, 3),
            "frames_per_s": round(len(plat) / span, 1),
            "gcells_per_s": round(float(cells[which].sum()) / span / 1e9, 1)}


def bench_serve_small(dev, qps: float = 80000.0, seconds: float = 1.5, warmup: int = 100, slots: int = 4,
                      streams: int = 4, overlap_queue: int = 3, seed: int = 1610041215):
    """Grouping where it can pay: Poisson arrivals of small requests (4 paths,
    median + LR, 160x120 to 320x240, D 32 or 64, the road scene scaled to
    D), offered past what ungrouped serving sustains, with groups of up to
    1, 8 and 32 requests (no cell limit) and with the server's default
    policy; frames/s and latency per policy."""
    import numpy as np
    import torch

    from paper_1610_04121_amd import synth
    from paper_1610_04121_amd.sgm import Server
    specs = []
    for k, ((w, h), d) in enumerate((s_, d_) for s_ in ((320, 240), (256, 192), (160, 120)) for d_ in (32, 64)):
        specs.append(dict(w=w, h=h, max_disp=d, n_paths=4, scene="K", scale_to_d=True, seed=seed * 100 + k))
    pool = []
    for k in specs:
        pr = synth.spec_pair(k)
        pool.append((torch.from_numpy(pr.left).to(dev), torch.from_numpy(pr.right).to(dev)))
    outs = _OutPool(dev, specs, per_kind=4096)
    trials = {}
    for name in ("1", "8", "32", "default"):
        if name == "default":
            srv = Server(16 << 30, slots=slots, streams=streams, max_pending=1 << 16, overlap_queue=overlap_queue)
        else:
            srv = Server(16 << 30, slots=slots, streams=streams, max_group=int(name), max_pending=1 << 16,
                         max_group_cells=1 << 62, overlap_queue=overlap_queue)
        res, _, _ = _serve_level(srv, specs, pool, outs, qps, int(seconds * qps), warmup,
                                 np.random.default_rng(seed + 1))
        srv.close()
        trials[name] = res
        print(f"bench: small-request serve max_group={name} at {qps}/s: {res['frames_per_s']} frames/s, "
              f"p99 {res['p99_ms']} ms, mean group {res['mean_group']}", file=sys.stderr, flush=True)
    return {"offered_qps": qps, "requests": int(seconds * qps), "by_max_group": trials,
            "default_policy": {"max_group": 32, "max_group_cells": 1 << 28},
            "mix": "Poisson arrivals; sizes from {320x240, 256x192, 160x120}, D from {32, 64}, 4 paths, median + "
                   "LR check, road scene scaled to D", "slots": slots, "streams": streams}


def bench_serve(dev, qps_levels, min_requests: int = 1000, per_qps_s: float = 10.0, warmup: int = 100,
                slots: int = 4, streams: int = 4, overlap_queue: int = 3, group_trial_s: float = 3.0,
                seed: int = 1610041214):
    """Poisson arrivals of 8-path median + LR requests of mixed sizes and
    disparity ranges (the road scene scaled to each range), served by the
    continuous-batching server and, on the same arrival times, by plain
    per-request launches.  Each level runs max(min_requests, per_qps_s * qps)
    requests after `warmup` warm-up requests.  First, at the highest level
    (past saturation), the server runs with and without grouping (groups of
    up to 2, 4, 8 requests against groups of one) for group_trial_s seconds
    of arrivals each; the sweep uses the policy with the highest throughput."""
    import numpy as np
    import torch

    from paper_1610_04121_amd import SGM, synth
    from paper_1610_04121_amd.sgm import Server

    specs, pool = _serve_setup(dev, seed)
    budget = 64 << 30
    top = max(qps_levels)
    outs = _OutPool(dev, specs, per_kind=1024)
    rng = np.random.default_rng(seed)
    # grouping: measured at saturation
    trials = {}
    for mg in (1, 2, 4, 8):
        srv = Server(budget, slots=slots, streams=streams, max_group=mg, max_pending=1 << 16,
                     max_group_cells=1 << 62, overlap_queue=overlap_queue)
        res, _, _ = _serve_level(srv, specs, pool, outs, top, int(group_trial_s * top), warmup,
                                 np.random.default_rng(seed + 1))
        srv.close()
        trials[str(mg)] = res
        print(f"bench: serve grouping max_group={mg} at {top}/s: {res['frames_per_s']} frames/s, "
              f"p99 {res['p99_ms']} ms, mean group {res['mean_group']}", file=sys.stderr, flush=True)
    best = max(trials, key=lambda g: trials[g]["frames_per_s"])
    max_group = int(best)
    srv = Server(budget, slots=slots, streams=streams, max_group=max_group, max_pending=1 << 16,
                 max_group_cells=1 << 62, overlap_queue=overlap_queue)
    ctxs = [SGM(k["w"], k["h"], k["max_disp"], synth.P1_DEFAULT, synth.P2_DEFAULT, 8, median=True, lrcheck=True)
            for k in specs]
    st = torch.cuda.current_stream()
    for k in range(len(specs)):  # warm the plain path's contexts
        buf = outs.take(k, lambda _: None)
        ctxs[k].compute(pool[k][0], pool[k][1], buf, stream=st)
        outs.give(k, buf)
    torch.cuda.synchronize()
    levels = []
    for qps in qps_levels:
        n_req = max(min_requests, int(per_qps_s * qps))
        server_res, arr, which = _serve_level(srv, specs, pool, outs, qps, n_req, warmup, rng)
        plain_res = _plain_level(ctxs, specs, pool, outs, arr, which, st)
        print(f"bench: serve qps={qps} ({n_req} requests) server p99={server_res['p99_ms']} ms "
              f"plain p99={plain_res['p99_ms']} ms", file=sys.stderr, flush=True)
        levels.append({"offered_qps": qps, "requests": n_req, "server": server_res, "plain": plain_res})
    stats = srv.stats()
    srv.close()
    for c in ctxs:
        c.close()
    return {"levels": levels, "budget_bytes": budget, "slots": slots, "streams": streams, "max_group": max_group,
            "max_group_cells": None, "overlap_queue": overlap_queue, "peak_bytes": stats["peak_bytes"],
            "grouping_at_saturation": {"offered_qps": top, "requests": int(group_trial_s * top), "by_max_group": trials,
                                       "chosen_max_group": max_group},
            "mix": "Poisson arrivals; sizes from {640x480, 1242x375, 1280x720, 1920x1080}, D from {128, 256}, "
                   "8 paths, median + LR check, road scene scaled to D; latency = submission to observed completion; "
                   f"max(1000, 10 qps) requests per level after {warmup} warm-up"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--inflight", type=int, default=1, help="frames in flight in the timed region")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="single-pair workload of synth.WORKLOADS to time (profiler runs of the other "
                         "workloads; the default is the headline workload)")
    ap.add_argument("--profile-every", type=int, default=32,
                    help="record stage events on every n-th frame of each context")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="also time the CPU oracle on every workload (single-pair latencies, the 64-pair "
                         "batch over all cores, the served mix); takes a few minutes")
    ap.add_argument("--tuning", default="", help="fixed kernel shape 'lanes_h,lanes_v,fused,census_cost[,final_pass[,post_in_wta]]' "
                                                   "instead of autotuning (for profiler runs)")
    ap.add_argument("--no-extras", action="store_true", help="skip serialized/latency/copy measurements")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-pair batched measurement")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-requests measurement")
    ap.add_argument("--serve-qps", default="50,500,1000,1500,2000")
    ap.add_argument("--serve-min-requests", type=int, default=1000,
                    help="requests per level: max(this, --serve-seconds * qps), after 100 warm-up")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-overlap-queue", type=int, default=3)
    ap.add_argument("--latency-samples", type=int, default=300)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a device-to-device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--read-calibration-mb", type=int, default=0,
                    help="also run a read-only reduction (torch.sum of int64 words) over this many MiB: a second "
                         "known-size reference for the byte counters, with another access pattern than the copy")
    ap.add_argument("--counters-from", default="",
                    help="FETCH_CSV,WRITE_CSV: summarize rocprofv3 --pmc output (with --copy-calibration-mb "
                         "and --tuning as in the profiled run) as JSON and exit")
    ap.add_argument("--graph", action="store_true",
                    help="time the frames as graph replays (SGM_GRAPH; no stage events in the timed region)")
    ap.add_argument("--trace-from", default="",
                    help="KERNEL_TRACE_CSV: summarize a rocprofv3 --kernel-trace run of whole frames (frame span, "
                         "kernel time, gaps between kernels) as JSON and exit")
    ap.add_argument("--trace-frames", default="", help="FIRST:END frames (launch order) for --trace-from")
    args = ap.parse_args()
    if args.trace_from:
        rng = tuple(int(v) for v in args.trace_frames.split(":")) if args.trace_frames else None
        print(json.dumps(summarize_trace(args.trace_from, frames_range=rng), indent=1))
        return
    if args.counters_from:
        fcsv, wcsv = args.counters_from.split(",")
        print(json.dumps(summarize_counters(fcsv, wcsv, args.copy_calibration_mb, args.tuning.split(",")), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent frames shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1610_04121_amd import SGM, synth

    workload = args.workload
    if workload not in synth.WORKLOADS:
        print(f"unknown workload {workload}; choose from {sorted(synth.WORKLOADS)}", file=sys.stderr)
        sys.exit(2)
    cfg = synth.WORKLOADS[workload]
    W, H, D, P = cfg["w"], cfg["h"], cfg["max_disp"], cfg["n_paths"]
    pair = synth.workload_pair(workload)
    dev = torch.device("cuda:0")
    left = torch.from_numpy(pair.left).to(dev)
    right = torch.from_numpy(pair.right).to(dev)
    F = max(1, args.inflight)

    def make_ctx(graph=False, tuning=None):
        c = SGM(W, H, D, synth.P1_DEFAULT, synth.P2_DEFAULT, P, median=cfg["median"],
                lrcheck=cfg["lr"], graph=graph)
        if tuning:
            c.set_tuning(*tuning)
        return c

    # kernel shape: measured on this device for this workload (results do not depend on it)
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")] + [0, 0]
        gh, gv, f, cc, fp, pw = vals[:6]
        choice = (gh, gv, bool(f), bool(cc), bool(fp), bool(pw))
        tuned = {"candidates": None}
    else:
        probe = make_ctx()
        tuned = probe.autotune(left, right, use_cache=False)
        probe.close()
        choice = tuple(tuned["choice"])
    print(f"bench: autotuned kernel shape {choice}", file=sys.stderr, flush=True)
    ctxs = [make_ctx(graph=args.graph, tuning=choice) for _ in range(F)]
    streams = [torch.cuda.Stream() for _ in range(F)]
    outs = [torch.empty((H, W), dtype=torch.uint16, device=dev) for _ in range(F)]
    print(f"bench: {workload} inflight={F} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)

    def run(n):
        for k in range(n):
            j = k % F
            ctxs[j].compute(left, right, outs[j], stream=streams[j])

    run(args.warmup)
    torch.cuda.synchronize()
    for c in ctxs:
        if not args.graph:  # (stage events would turn replays into direct launches)
            c.profile(True, every=args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ncalls, stage_ms = 0, {}
    for c in ctxs:
        n, st = c.profile_read()
        c.profile(False)
        ncalls += n
        for k, v in st.items():
            stage_ms[k] = stage_ms.get(k, 0.0) + v
    elapsed = t1 - t0
    fps = args.steps / elapsed
    tuning = ctxs[0].tuning()
    if args.graph:
        # the stage events need direct launches: an untimed pass of the same
        # frames on a direct-launch context gives the per-kernel times
        pc = make_ctx(tuning=choice)
        pc.profile(True, every=1)
        for _ in range(min(args.steps, 400)):
            pc.compute(left, right, outs[0], stream=streams[0])
        torch.cuda.synchronize()
        ncalls, stage_ms = pc.profile_read()
        pc.profile(False)
        pc.close()

    extras = {}
    if not args.no_extras:
        # one frame at a time on one stream: eager, then graph replay
        s0 = ctxs[0]
        st0 = torch.cuda.current_stream()
        for mode in ("eager", "graph"):
            c = s0 if mode == "eager" else make_ctx(graph=True, tuning=choice)
            for _ in range(args.warmup):
                c.compute(left, right, outs[0], stream=st0)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(args.steps // 2):
                c.compute(left, right, outs[0], stream=st0)
            torch.cuda.synchronize()
            extras[mode] = round((args.steps // 2) / (time.perf_counter() - ta), 2)
            # single frames between two events, each waited for (the events
            # themselves leave the device idle a few microseconds)
            lat = []
            for _ in range(args.latency_samples):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st0)
                c.compute(left, right, outs[0], stream=st0)
                e1.record(st0)
                e1.synchronize()
                lat.append(e0.elapsed_time(e1))
            lat = np.array(lat)
            extras["latency_ms" if mode == "graph" else "latency_ms_eager"] = {
                "p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                "mode": ("graph replay" if mode == "graph" else "direct launches") + ", one frame in flight",
                "samples": len(lat)}
            if mode == "graph":
                c.close()
        # the packed-u16 VALU rate the aggregation is compared with: the probe
        # issues 16 VALU instructions per wave per round (4 waves per block)
        from paper_1610_04121_amd.sgm import valu_probe
        pb, pit = 8192, 2048
        sink = torch.zeros(pb * 256, dtype=torch.int32, device=dev)
        for _ in range(2):
            valu_probe(pb, pit, sink)
        pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pe0.record()
        for _ in range(5):
            valu_probe(pb, pit, sink)
        pe1.record()
        pe1.synchronize()
        inst_s = 5 * pb * 4 * pit * 16 / (pe0.elapsed_time(pe1) * 1e-3)
        nominal = 1024 * 2.4e9 / 4  # one wave64 instruction per SIMD per 4 cycles at 2.4 GHz
        extras["valu_probe"] = {"wave_instr_per_s": round(inst_s / 1e9, 1), "unit": "G wave64 VALU instr/s",
                                "nominal_peak": round(nominal / 1e9, 1), "frac_of_nominal": round(inst_s / nominal, 4),
                                "packed_u16_tops": round(inst_s * 64 * 2 / 1e12, 1),
                                "kernel": "valu_probe_kernel: 8 independent v_pk_add_u16 + v_pk_min_u16 pairs per round"}
        # dependent chains, one wave per SIMD (256 blocks of 4 waves): clock
        # cycles per link at the 2.4 GHz peak clock
        lat = {}
        for mode, name in ((1, "pk_add_then_pk_min"), (2, "dpp_row_mirror_min_then_add"),
                           (3, "permlane16_swap_min_add")):
            lit = 4096
            valu_probe(256, 64, sink[:256 * 256], mode=mode)
            pe0.record()
            valu_probe(256, lit, sink[:256 * 256], mode=mode)
            pe1.record()
            pe1.synchronize()
            lat[name] = round(pe0.elapsed_time(pe1) * 1e-3 * 2.4e9 / (lit * 8), 2)
        extras["valu_probe"]["dependent_link_cycles"] = lat
        del sink
        # achievable HBM bandwidth: a timed device-to-device copy of 512 MiB
        nb = 512 << 20
        csrc = torch.empty(nb, dtype=torch.uint8, device=dev)
        cdst = torch.empty_like(csrc)
        cdst.copy_(csrc)
        ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ce0.record()
        for _ in range(10):
            cdst.copy_(csrc)
        ce1.record()
        ce1.synchronize()
        extras["copy_gbs"] = round(2 * nb * 10 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9, 1)
        del csrc, cdst

    # the aggregation kernel reads the cost volume (u8) and writes one L_r
    # plane (u8: Cmax + P2 = 148 < 256) per direction it runs: all of them,
    # or all but the last with the final pass
    Dp = 64 if D <= 64 else (128 if D <= 128 else 256)
    final_pass = bool(tuning[4]) and not tuning[2]
    if tuning[2]:  # fused: census words of both views in, L_r out
        agg_bytes = P * W * H * (Dp + 2 * 8)
    else:  # cost volume in, L_r out
        agg_bytes = (P - 1 if final_pass else P) * W * H * Dp * (1 + 1)
    agg_ms = stage_ms["aggregate"] / max(ncalls, 1)
    achieved = agg_bytes / (agg_ms * 1e-3) / 1e9
    roof = {"kernel": "aggregate_kernel", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _traffic(tuning) if workload == WORKLOAD else None, "alg_bytes_per_launch": agg_bytes, "mean_launch_ms": round(agg_ms, 5)}
    if "copy_gbs" in extras:
        roof["measured_copy_gbs"] = extras["copy_gbs"]
        roof["frac_of_measured_copy"] = round(achieved / extras["copy_gbs"], 4)
    # the winner-take-all stage: the WTA kernel (P planes in, two maps out),
    # or the final pass (cost volume and P - 1 planes in, two maps out)
    wta_ms = stage_ms["wta"] / max(ncalls, 1)
    wta_bytes = P * W * H * Dp + 4 * W * H  # P planes, or the cost volume and P - 1 planes
    wta_gbs = wta_bytes / (wta_ms * 1e-3) / 1e9
    wta_stage = {"kernel": "final_pass_kernel" if final_pass else "wta_kernel", "alg_bytes_per_launch": wta_bytes,
                 "mean_launch_ms": round(wta_ms, 5), "achieved": round(wta_gbs, 1), "unit": "GB/s",
                 "frac": round(wta_gbs / HBM_PEAK_GBS, 4)}

    # the whole path from the first census launch to the end of the WTA
    # (median and LR excluded), event-timed like the stages it spans
    pipe_ms = sum(stage_ms[k] for k in ("census_cost", "aggregate", "wta")) / max(ncalls, 1)
    pipe_bytes = pipeline_bytes(W, H, Dp, P, tuning)
    pipe_gbs = pipe_bytes / (pipe_ms * 1e-3) / 1e9
    pipe = {"stages": "census..wta", "ms_per_frame": round(pipe_ms, 5), "alg_bytes": pipe_bytes,
            "achieved": round(pipe_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(pipe_gbs / HBM_PEAK_GBS, 4)}
    if "copy_gbs" in extras:
        pipe["frac_of_measured_copy"] = round(pipe_gbs / extras["copy_gbs"], 4)
    # the same span against the byte count of the schedule with u16 partial
    # sums and costs recomputed in every pass (images in, (4P - 4) sweeps of
    # W * H * D u16 partial-sum bytes, the two raw maps out), the usual
    # yardstick for "fraction of the HBM roofline" of this path
    u16_bytes = 2 * W * H + (4 * P - 4) * W * H * D + 2 * W * H * (2 if cfg["lr"] else 1)
    pipe["alg_bytes_u16_partial_sum_schedule"] = u16_bytes
    pipe["frac_u16_partial_sum_schedule"] = round(u16_bytes / (pipe_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    line = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": workload, "width": W, "height": H, "max_disp": D, "n_paths": P,
                   "census": "9x7 full", "P1": synth.P1_DEFAULT, "P2": synth.P2_DEFAULT,
                   "median": cfg["median"], "lr_check": cfg["lr"], "scene": cfg["scene"],
                   "seed": cfg["seed"], "frames_in_flight": F, "graph_replay": bool(args.graph),
                   "lanes_h": tuning[0], "lanes_v": tuning[1], "fused_cost": tuning[2],
                   "fused_census_cost": tuning[3], "final_pass": final_pass,
                   "autotune_ms_per_frame": tuned["candidates"]},
        "gcells_per_s": round(W * H * D * P * fps / 1e9, 2),
        "stage_ms": {k: round(v / max(ncalls, 1), 5) for k, v in stage_ms.items()},
        "roofline": roof,
        "wta_stage": wta_stage,
        "pipeline": pipe,
    }
    if extras:
        line["serialized_fps"] = {"eager": extras["eager"], "graph": extras["graph"]}
        line["valu_probe"] = extras["valu_probe"]
        line["latency_ms"] = extras["latency_ms"]
        line["latency_ms_eager"] = extras["latency_ms_eager"]
        line["paths_sweep"] = bench_paths(left, right, cfg, max(200, args.steps // 4))
        line["lr_full"] = bench_variant(left, right, cfg, choice, max(200, args.steps // 4), lr_full=True)
        line["subpixel"] = bench_variant(left, right, cfg, choice, max(200, args.steps // 4), subpixel=True)
        line["adaptive_p2"] = bench_variant(left, right, cfg, choice, max(200, args.steps // 4), adaptive_p2=True)
    for c in ctxs:
        c.close()
    if args.copy_calibration_mb:
        n = args.copy_calibration_mb << 20
        src = torch.empty(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = n
    if args.read_calibration_mb:
        n = args.read_calibration_mb << 20
        src = torch.ones(n // 8, dtype=torch.int64, device=dev)
        for _ in range(3):
            total = int(src.sum().item())
        assert total == n // 8
        line["read_calibration_bytes"] = n
    if not args.no_batch:
        print("bench: 64-pair batch vs sequential launches", file=sys.stderr, flush=True)
        line["batched"] = bench_batch(dev, args.batch_steps)
        line["batched_median_lr"] = bench_batch(dev, args.batch_steps, post=True)
        line["batched_small"] = bench_batch_small(dev)
    if not args.no_serve:
        print("bench: served requests", file=sys.stderr, flush=True)
        line["served"] = bench_serve(dev, [float(q) for q in args.serve_qps.split(",")], args.serve_min_requests,
                                     args.serve_seconds, slots=args.serve_slots, streams=args.serve_streams,
                                     overlap_queue=args.serve_overlap_queue)
        line["served_small_grouping"] = bench_serve_small(dev, slots=args.serve_slots, streams=args.serve_streams,
                                                          overlap_queue=args.serve_overlap_queue)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(pair, cfg)
    if args.oracle_timing:
        print("bench: timing the CPU oracle on every workload", file=sys.stderr, flush=True)
        line["oracle_timing"] = oracle_timing()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the red-rec solve + batching hot path on one MI355X.

A step is one pass of the whole path over one batch of shots already resident in HBM:
rr_solve_many (red-rec on every shot) -> rr_plan_many (device-side arena layout from the step
counts) -> rr_batch_moves_many (Alg. 3 on every shot), all on one stream with no host sync.
Workload: 8192 shots of a 64x64 trap grid loaded i.i.d. Bernoulli(0.55), centred 44x44 target.

Reported in one JSON line: batched shots/s (value), the roofline of the dominant kernel, and
the other forms of the same path: one shot per launch (rr_solve + rr_batch_moves) with p50/p99
latency; the single-instance 32 x 32 and 128 x 128 configurations on the one-instance path;
the paper's own benchmark geometry, per launch and batched; the uneven-size batch as one
graph-captured chain per size class; a served Poisson stream with continuous batching (p50/p99
overall and per class); the serial order of red-rec and bird on the batched workload; exact 1D
on chains in the paper's 1-D geometry.  The CPU leg, run before the GPU is touched, times the
oracle on the host cores and computes the oracle results the bit-exact samples are checked
against.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The served form runs one stream per size-class wave in flight; streams sharing a hardware queue
# run in submission order, so give HIP (read once, when it starts) a queue per pooled stream: at
# least 32 (HIP's default is 4).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 32:
    os.environ["GPU_MAX_HW_QUEUES"] = "32"

METRIC = "red-rec shots/s batched vs 1-per-launch at 1 GPU; p50/p99 µs per shot (bit-exact)"
WORKLOAD = "batch64"
HBM_PEAK_GBS = 8000.0
STEP_BOUND_PER_SHOT = 48000      # pool sizing bound for a 64x64 shot (observed ~19k steps)


def _cpu_worker(rng):
    """Oracle solve + batching for shots [lo, hi) of the workload (CPU baseline leg)."""
    lo, hi = rng
    import oracle
    import rr_inputs as ri
    shots = ri.config_shots(WORKLOAD, n=hi - lo, first=lo)
    grids = [ri.shot_grid(d) for d in shots]
    t0 = time.perf_counter()
    for d, g in zip(shots, grids):
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        r = oracle.solve(shape, g)
        if r["status"] == 0:
            oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"])
    return time.perf_counter() - t0


def cpu_baseline(seconds: float, max_workers: int):
    import oracle
    oracle.build()
    cores = max(1, min(max_workers, os.cpu_count() or 1))
    calib = _cpu_worker((0, 8)) / 8.0                       # seconds per shot on one core
    per_worker = max(1, int(seconds / calib))
    n = min(8192, per_worker * cores)
    chunk = (n + cores - 1) // cores
    ranges = [(i, min(n, i + chunk)) for i in range(0, n, chunk)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(ranges)) as pool:
        pool.map(_cpu_worker, ranges)
    wall = time.perf_counter() - t0
    return {"value": round(n / wall, 2), "unit": "shots/s", "cores": len(ranges), "kind": "oracle",
            "sample": f"shots 0..{n - 1} of the same 8192-shot workload, solve + batching, "
                      f"{len(ranges)} single-threaded oracle processes; 1-core latency {calib * 1e3:.2f} ms/shot"}


def oracle_references(verify_shots: int, paper_shots: int, flags: int):
    """Part of the CPU baseline leg, run before the GPU is touched: the oracle's solve and batching
    results for the sampled shots of the 8192-shot workload, of the paper's geometry and of the
    two single-instance configurations whose GPU results the run checks bit for bit afterwards,
    the oracle's chain results for a sample of the paper's chain geometry, and the pair-loop
    iterations of the sampled 64 x 64 shots (a dependency floor of the solve)."""
    import numpy as np

    import oracle
    import rr_inputs as ri
    oracle.build()
    refs = {}
    for name, idx in ((WORKLOAD, np.linspace(0, 8191, verify_shots).astype(int) if verify_shots > 0 else []),
                      ("paper32", range(min(8, paper_shots))), ("single32", [0]), ("single128", [0])):
        out = {}
        for i in idx:
            d = ri.config_shots(name, n=1, first=int(i))[0]
            shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
            r = oracle.solve(shape, ri.shot_grid(d), trace=True)
            rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags & 0xFF, indexed=True) \
                if r["status"] == 0 else None
            out[int(i)] = (r, rb)
        refs[name] = out
    refs["pair_loop_iterations"] = [len(r["events"]) for r, _ in refs[WORKLOAD].values()]
    chains = {}
    for i in range(8):
        d = ri.config_shots("chain1024", n=1, first=i)[0]
        chains[i] = oracle.solve_chain(d["w"], ri.shot_grid(d)[0], d["x0"], d["x1"] - d["x0"])
    refs["chain1024"] = chains
    return refs


BATCH_SOURCES = ("rr_batch.hip", "rr_batch_graph.hpp", "rr_batch_loop.hpp", "rr_batch_generic.hpp", "rr_device.hpp",
                 "rr_batch_common.hpp", "rr_batch_loop_kernels.hpp", "rr_batch_loop2.hip")
PROFILE = os.path.join(ROOT, "profiles", "k_loop_many_batch64.md")


def measured_traffic(flags):
    """HBM bytes of one k_loop_many launch from the committed rocprofv3 PMC summary (FETCH_SIZE +
    WRITE_SIZE scaled by a plain copy), or None when that summary was taken on other kernel
    sources, or under another launch schedule (flags), than the ones run now."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in BATCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_06182_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()[:16]
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch k_loop_many<2,0> (\d+) sources_sha256 ([0-9a-f]+) flags (\d+)", text)
    if not m or m.group(2) != sha or int(m.group(3)) != int(flags):
        return None
    return float(m.group(1))


def mixed_step_bound(shape):
    """Pool-sizing estimate of one shot's step count (about 0.07 * side**3 for these loadings);
    the device planner reports exact totals and the pools grow once when the estimate is short."""
    side = max(shape[0], shape[1])
    return int(0.08 * side ** 3) + 1024


def mixed_graph_form(args, dev, replays):
    """Uneven batch: 4096 shots, sides uniform over {32..256}, p ~ U[0.5, 0.65], target
    floor(0.7 n), split by size class (one solve -> plan -> batch chain per class, each class on
    its own stream), captured once in a HIP graph and replayed; every replay is checked against
    the eager pass."""
    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd.pipeline import ClassedBuffers
    shots = ri.config_shots("mixed")
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    cb = ClassedBuffers(shapes, mixed_step_bound, device=dev).load(grids)
    streams = [torch.cuda.Stream() for _ in cb.parts]
    cb.run(args.flags, streams)
    torch.cuda.synchronize()
    if cb.fit_pools():
        cb.run(args.flags, streams)
        torch.cuda.synchronize()
    cb.poison_outputs()                        # unwritten output bytes show up in the comparisons
    cb.run(args.flags, streams)
    torch.cuda.synchronize()
    ref = cb.outputs()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cb.run(args.flags, streams)
    torch.cuda.synchronize()
    same = True
    for _ in range(2):                         # replays over poisoned outputs, eager work between them
        cb.poison_outputs()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        same = same and cb.same_outputs(cb.outputs(), ref)
    t0 = time.perf_counter()
    for _ in range(replays):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / replays
    same = same and cb.same_outputs(cb.outputs(), ref)
    del ref
    s_, b_ = cb.infos()
    sst = s_[:, 0].view(np.int32)
    assert np.all((sst == 0) | (sst == 1)) and np.all(b_[:, 0].view(np.int32) == 0), "a mixed shot failed"
    ws_words = np.array([s[1] * ((s[0] + 63) // 64) for s in shapes], np.int64)
    nm, ng, ns = s_[:, 1].astype(np.int64), s_[:, 2].astype(np.int64), s_[:, 3].astype(np.int64)
    nbt = b_[:, 1].astype(np.int64)
    alg = int((16 * ws_words + 8 * nm + 4 * (ng + 1) + 24 + 80).sum() +
              (8 * nm + 4 * (ng + 1) + 24 + 80 + 4 * ns + 4 * (nbt + 1) + 20).sum())
    return {"graph_shots_per_s": round(len(shots) / dt, 1), "graph_ms_per_replay": round(dt * 1e3, 3),
            "graph_algorithmic_GBps": round(alg / dt / 1e9, 2), "graph_replays_equal_eager": bool(same),
            "shots": len(shots), "infeasible": int((sst == 1).sum()),
            "classes": {str(c): int(len(idx)) for c, idx, _ in cb.parts},
            "workload": "4096 shots, side uniform over {32,48,64,96,128,192,256}, p ~ U[0.5,0.65], centred "
                        "floor(0.7 n) target; one solve+plan+batch chain per size class on its own stream, "
                        "captured in one HIP graph"}



def paper_geometry_form(args, dev, n_single, refs):
    """The paper's benchmark geometry (32 x 54 traps, full-width 32 x 32 target, exactly 1036 atoms
    per shot, 1000 shots): per-shot latency of one synchronised rr_solve launch -- the paper
    reports red-rec time per instance -- and of solve + batching, and the per-shot cost when all
    1000 shots go in one launch of each."""
    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd.pipeline import BatchBuffers, ManyBuffers, SolveBuffers
    from paper_2504_06182_amd.tune import flags_for

    shots = ri.config_shots("paper32")
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    stream = torch.cuda.current_stream()
    sbs = [SolveBuffers(shapes[i], device=dev).load(grids[i]) for i in range(n_single)]
    for sb in sbs:
        sb.run(stream)
    torch.cuda.synchronize()
    steps = [max(sb.host()["n_steps"], 1) for sb in sbs]
    bbs = [BatchBuffers(sb, step_cap=st, device=dev) for sb, st in zip(sbs, steps)]
    for sb, bb in zip(sbs[:4], bbs[:4]):
        sb.run(stream); bb.run(args.flags, stream)
    torch.cuda.synchronize()
    lat_s, lat_b = [], []
    for sb in sbs:
        a = time.perf_counter()
        sb.run(stream)
        torch.cuda.synchronize()
        lat_s.append((time.perf_counter() - a) * 1e6)
    for sb, bb in zip(sbs, bbs):
        a = time.perf_counter()
        sb.run(stream)
        bb.run(args.flags, stream)
        torch.cuda.synchronize()
        lat_b.append((time.perf_counter() - a) * 1e6)
    exact = None
    if refs:
        exact = 0
        for i, (r, rb) in refs.items():
            g, gb = sbs[i].host(), bbs[i].host()
            exact += int(g["status"] == r["status"] == 0 and np.array_equal(g["moves"], r["moves"])
                         and np.array_equal(g["final"], r["final"]) and np.array_equal(gb["steps"], rb["steps"])
                         and np.array_equal(gb["batch_off"], rb["batch_off"]))

    mb = ManyBuffers(shapes, device=dev).load(grids).solve(stream)
    torch.cuda.synchronize()
    mb.plan_batches([max(int(i[3]), 1) for i in mb.solve_infos()])
    bflags = flags_for(64, args.flags)
    ts, tb = [], []
    for _ in range(6):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        mb.solve(stream)
        e[1].record(stream)
        mb.batch(bflags, stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        ts.append(e[0].elapsed_time(e[1]))
        tb.append(e[1].elapsed_time(e[2]))
    n = len(shots)
    infeasible = int((mb.solve_infos()[:, 0].view(np.int32) == 1).sum())
    ts, tb = float(np.median(ts[1:])), float(np.median(tb[1:]))
    return {"workload": "the paper's geometry: 32 x 54 traps, full-width centred 32 x 32 target, exactly 1036 atoms "
                        "per shot drawn uniformly, 1000 shots",
            "shots": n, "infeasible": infeasible,
            "per_launch_solve_p50_us": round(float(np.percentile(lat_s, 50)), 1),
            "per_launch_solve_p99_us": round(float(np.percentile(lat_s, 99)), 1),
            "per_launch_solve_batch_p50_us": round(float(np.percentile(lat_b, 50)), 1),
            "per_launch_solve_batch_p99_us": round(float(np.percentile(lat_b, 99)), 1),
            "per_launch_sample": n_single,
            "batched_solve_us_per_shot": round(ts * 1e3 / n, 3),
            "batched_solve_batch_us_per_shot": round((ts + tb) * 1e3 / n, 3),
            "batched_launch_ms": {"solve": round(ts, 3), "batch": round(tb, 3)},
            "bit_exact_sample": f"{exact}/{len(refs)}" if refs else "not checked (--no-cpu)",
            "paper_context": {"red_rec_serial_cpu_us": 106, "red_rec_gpu_us": 197,
                              "hardware": "AMD Threadripper 2950X (CPU) / Nvidia Quadro RTX 4000 (GPU)",
                              "note": "mean time per instance over 1000 instances; batching not timed there"}}


def _same(g, r):
    import numpy as np
    ok = g["status"] == r["status"] and np.array_equal(np.asarray(g["final"]).reshape(-1),
                                                        np.asarray(r["final"]).reshape(-1))
    if ok and r["status"] == 0:
        ok = np.array_equal(g["moves"], r["moves"]) and np.array_equal(g["group_off"], r["group_off"])
    return ok


def single_instance_form(args, dev, refs):
    """The two single-instance configurations (32 x 32 grid, p 0.5, centred 16 x 16 target; 128 x
    128, p 0.6, centred 90 x 90), each on the plain one-instance path: --single-launches
    synchronised launches of rr_solve, and of rr_solve + rr_batch_moves (host clock, p50/p99),
    plus the device time of each kernel chain from HIP events."""
    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd.pipeline import BatchBuffers, SolveBuffers
    out = {}
    stream = torch.cuda.current_stream()
    for name in ("single32", "single128"):
        d = ri.config_shots(name)[0]
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        sb = SolveBuffers(shape, device=dev).load(ri.shot_grid(d))
        sb.run(stream)
        torch.cuda.synchronize()
        g = sb.host()
        bb = BatchBuffers(sb, step_cap=max(g["n_steps"], 1), device=dev)
        for _ in range(5):
            sb.run(stream); bb.run(args.flags, stream)
        torch.cuda.synchronize()
        lat_s, lat_b, dev_s, dev_b = [], [], [], []
        for _ in range(args.single_launches):
            a = time.perf_counter()
            sb.run(stream)
            torch.cuda.synchronize()
            lat_s.append((time.perf_counter() - a) * 1e6)
        for _ in range(args.single_launches):
            a = time.perf_counter()
            sb.run(stream)
            bb.run(args.flags, stream)
            torch.cuda.synchronize()
            lat_b.append((time.perf_counter() - a) * 1e6)
        for _ in range(20):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream); sb.run(stream); e[1].record(stream); bb.run(args.flags, stream); e[2].record(stream)
            torch.cuda.synchronize()
            dev_s.append(e[0].elapsed_time(e[1]) * 1e3); dev_b.append(e[1].elapsed_time(e[2]) * 1e3)
        exact = None
        if name in refs:
            r, rb = refs[name][0]
            gb = bb.host()
            exact = bool(_same(sb.host(), r) and (rb is None or (np.array_equal(gb["steps"], rb["steps"])
                                                                and np.array_equal(gb["batch_off"], rb["batch_off"]))))
        out[name] = {"grid": [d["w"], d["h"]], "target": [d["x1"] - d["x0"], d["y1"] - d["y0"]], "p": d["p"],
                     "moves": g["n_moves"], "steps": g["n_steps"], "batches": bb.host()["n_batches"],
                     "solve_p50_us": round(float(np.percentile(lat_s, 50)), 1),
                     "solve_p99_us": round(float(np.percentile(lat_s, 99)), 1),
                     "solve_batch_p50_us": round(float(np.percentile(lat_b, 50)), 1),
                     "solve_batch_p99_us": round(float(np.percentile(lat_b, 99)), 1),
                     "device_solve_us": round(float(np.median(dev_s)), 1),
                     "device_batch_us": round(float(np.median(dev_b)), 1),
                     "launches": args.single_launches, "bit_exact": exact}
    return out


def variants_form(args, dev):
    """The solver variants on the 8192-shot 64 x 64 workload, each as a batched step (solve ->
    plan -> batch): red-rec in the parallel order of §III.D (the default), red-rec in the serial
    order of Alg. 1, and bird (Alg. 2); device times from HIP events (median of 3) and the mean
    moves, unit steps and batches per shot (the operational side: fewer steps, fewer batches)."""
    import numpy as np
    import torch

    import rr_inputs as ri
    import paper_2504_06182_amd as rr
    from paper_2504_06182_amd.pipeline import ManyBuffers
    from paper_2504_06182_amd.tune import flags_for, solve_flags_for
    shots = ri.config_shots(WORKLOAD)
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    stream = torch.cuda.current_stream()
    bflags = flags_for(64, args.flags)
    ws_one = rr.rr_batch_workspace_bytes(shapes[0], 2 * 44 * 44, STEP_BOUND_PER_SHOT)
    out = {}
    for name, algo in (("redrec_parallel", 0), ("redrec_serial", 1), ("bird", 2)):
        mb = ManyBuffers(shapes, device=dev, solve_flags=solve_flags_for(64, algo)).load(grids)
        n = mb.n
        mb.alloc_pools(n * STEP_BOUND_PER_SHOT, n * (STEP_BOUND_PER_SHOT + 1), n * ((ws_one + 255) // 256 * 256))
        ts, tb = [], []
        for rep in range(4):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream); mb.solve(stream); e[1].record(stream)
            mb.plan_device(stream); mb.batch(bflags, stream); e[2].record(stream)
            torch.cuda.synchronize()
            if rep:
                ts.append(e[0].elapsed_time(e[1])); tb.append(e[1].elapsed_time(e[2]))
        sinf, binf = mb.solve_infos(), mb.batch_infos()
        ok = sinf[:, 0].view(np.int32) == 0
        assert np.all(binf[:, 0].view(np.int32) == 0)
        out[name] = {"solve_ms": round(float(np.median(ts)), 3), "plan_batch_ms": round(float(np.median(tb)), 3),
                     "shots_per_s": round(n / ((np.median(ts) + np.median(tb)) / 1e3), 1),
                     "mean_moves": round(float(sinf[ok, 1].mean()), 1), "mean_steps": round(float(sinf[ok, 3].mean()), 1),
                     "mean_batches": round(float(binf[ok, 1].mean()), 1)}
        del mb
    return out


def chain_form(args, dev, refs):
    """Exact 1D on chains (§III.A-B) in the paper's chain geometry: 1024 traps, centre-compact
    target of 512, exactly 614 atoms (1000 chains).  One chain per synchronised launch (host
    clock p50/p99; the paper: 22 us on one CPU core for the serial form), all 1000 in one launch
    (device time per chain), and 16 chains of 65535 traps in one launch."""
    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd.pipeline import ChainBuffers
    stream = torch.cuda.current_stream()
    shots = ri.config_shots("chain1024")
    chains = [(d["w"], d["x0"], d["x1"] - d["x0"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    one = [ChainBuffers([chains[i]], device=dev).load([grids[i]]) for i in range(args.single_launches)]
    for cb in one[:5]:
        cb.solve(stream)
    torch.cuda.synchronize()
    lat = []
    for cb in one:
        a = time.perf_counter()
        cb.solve(stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e6)
    allc = ChainBuffers(chains, device=dev).load(grids)

    def timed(cb, reps=5):
        ts = []
        for _ in range(reps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record(stream); cb.solve(stream); e[1].record(stream)
            torch.cuda.synchronize()
            ts.append(e[0].elapsed_time(e[1]))
        return float(np.median(ts[1:]))

    t_all = timed(allc)
    sinf = allc.solve_infos()
    exact = None
    if "chain1024" in refs:
        exact = sum(int(_same(allc.host_solve(i, sinf), r)) for i, r in refs["chain1024"].items())
        exact = f"{exact}/{len(refs['chain1024'])}"
    long_shots = ri.config_shots("chain65535")
    longc = ChainBuffers([(d["w"], d["x0"], d["x1"] - d["x0"]) for d in long_shots], device=dev)
    longc.load([ri.shot_grid(d) for d in long_shots])
    t_long = timed(longc)
    return {"workload": "chains of 1024 traps, centre-compact target of 512, exactly 614 atoms placed uniformly "
                        "(the paper's 1-D geometry), 1000 chains",
            "per_launch_p50_us": round(float(np.percentile(lat, 50)), 1),
            "per_launch_p99_us": round(float(np.percentile(lat, 99)), 1), "per_launch_sample": len(lat),
            "batched_launch_ms": round(t_all, 3), "batched_us_per_chain": round(t_all * 1e3 / len(chains), 4),
            "mean_moves": round(float(sinf[:, 1].mean()), 1), "mean_steps": round(float(sinf[:, 3].mean()), 1),
            "bit_exact_sample": exact or "not checked (--no-cpu)",
            "long_chains": {"chains": len(long_shots), "traps": 65535, "target": 32767, "atoms": 39321,
                            "launch_ms": round(t_long, 3)},
            "paper_context": {"exact_1d_serial_cpu_us_at_1024": 22,
                              "hardware": "AMD Threadripper 2950X (CPU); the paper's GPU form stops at 1024 traps"}}


def large_form(args, dev):
    """The served stream's large class alone: 1024 x 1024 shots (p 0.6, centred 780 x 780
    target) on the wide kernels -- one shot solved and batched a launch at a time (HIP events
    around each call), then --large-shots shots in one many-instance launch each for solve and
    batching."""
    import gc

    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd.pipeline import BatchBuffers, ManyBuffers, SolveBuffers
    shots = ri.config_shots("big1024", n=args.large_shots)
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    sb = SolveBuffers(shapes[0], device=dev).load(grids[0])
    solve_ms = [timed(lambda: sb.run()) for _ in range(3)]
    h = sb.host()
    bb = BatchBuffers(sb, step_cap=max(h["n_steps"], 1), device=dev)
    per_flags = {}
    for f in [int(v) for v in args.large_flags.split(",")] if args.large_flags else [args.flags]:
        t = timed(lambda: bb.run(f))
        hb = bb.host()
        per_flags[str(f)] = {"batch_ms": round(t, 1), "batch_status": hb["status"], "batches": hb.get("n_batches")}
    first = next(iter(per_flags.values()))
    out = {"single": {"solve_ms": round(float(np.median(solve_ms)), 2), "batch_ms": first["batch_ms"],
                      "solve_status": h["status"], "batch_status": first["batch_status"], "moves": h["n_moves"],
                      "steps": h["n_steps"], "batches": first["batches"], "per_constraint": per_flags}}
    del sb, bb
    mb = ManyBuffers(shapes, device=dev).load(grids)
    t_solve = timed(lambda: mb.solve())
    sinf = mb.solve_infos()
    mb.plan_batches([max(int(x[3]), 1) for x in sinf])
    t_batch = timed(lambda: mb.batch(flags=args.flags))
    binf = mb.batch_infos()
    out["many"] = {"shots": len(shots), "solve_ms": round(t_solve, 2), "batch_ms": round(t_batch, 1),
                   "shots_per_s": round(len(shots) / ((t_solve + t_batch) / 1e3), 2),
                   "all_ok": bool(np.all(sinf[:, 0] == 0) and np.all(binf[:, 0] == 0))}
    out["workload"] = ("1024 x 1024 grid, i.i.d. Bernoulli(0.6) loading, centred 780 x 780 target; "
                       f"batching constraint flags {args.flags}")
    del mb
    gc.collect()
    torch.cuda.empty_cache()
    return out


def served_form(args, dev, rate):
    """Served stream: Poisson arrivals at ``rate`` shots/s for --serve-seconds of the uneven
    mix (grid side uniform over {32..256}) plus, with probability 1/--serve-big-every per
    arrival, a 1024 x 1024 shot (p 0.6, 780 x 780 target), fed to the continuous-batching
    server; per-shot latency = completion seen by the host - arrival."""
    import gc

    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd.serve import Server, poisson_arrivals, serve_stream
    pool = ri.config_shots("mixed", n=args.serve_pool)
    big = ri.config_shots("big1024", n=4) if args.serve_big_every > 0 else []
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in pool + big]
    grids = [ri.shot_grid(d) for d in pool + big]
    arrivals = poisson_arrivals(rate, args.serve_seconds, seed=50)
    order = np.arange(len(arrivals)) % len(pool)
    if big:
        pick = np.random.default_rng(51).random(len(arrivals)) < 1.0 / args.serve_big_every
        order[pick] = len(pool) + np.arange(int(pick.sum())) % len(big)
    share = {64: 0.04, 128: 0.12, 256: 0.64, 1024: 0.20} if big else None
    srv = Server(budget_bytes=args.serve_budget_gib << 30, class_share=share, max_wave=args.serve_max_wave,
                 flags=args.flags)
    warm = Server(budget_bytes=6 << 30, class_share={64: 0.1, 128: 0.15, 256: 0.35, 1024: 0.4} if big else
                  {64: 0.2, 128: 0.3, 256: 0.5}, flags=args.flags)
    for j in list(range(16)) + ([len(pool)] if big else []):   # first-launch costs outside the measurement
        warm.submit(shapes[j], grids[j])
    warm.drain()
    del warm
    gc.collect()
    torch.cuda.empty_cache()
    wall = serve_stream(srv, shapes, grids, arrivals, order)
    lat = srv.latencies_us()
    in_window = sum(1 for sh in srv.shots if sh["t_done"] is not None and sh["t_done"] - srv.t0 <= args.serve_seconds)
    per = {}
    for side in srv.classes:
        l_ = srv.latencies_us(side)
        if l_.size:
            per[str(side)] = {"n": int(l_.size), "p50_us": round(float(np.percentile(l_, 50)), 1),
                              "p99_us": round(float(np.percentile(l_, 99)), 1)}
    out = {"served_shots_per_s": round(len(arrivals) / wall, 1), "offered_rate": rate,
            "completed_in_window_per_s": round(in_window / args.serve_seconds, 1), "wall_s": round(wall, 2),
            "shots": int(len(arrivals)), "big_shots": int((order >= len(pool)).sum()),
            "p50_us": round(float(np.percentile(lat, 50)), 1),
            "p99_us": round(float(np.percentile(lat, 99)), 1), "per_class": per, "waves": srv.waves,
            "rerun_alone": srv.overflow, "slots": {str(k): v for k, v in srv.slots().items()},
            "workload": f"Poisson arrivals at {rate:g}/s for {args.serve_seconds:g} s, shots cycling "
                        f"through {len(pool)} shots of the uneven mix"
                        + (f", a 1024 x 1024 shot (p 0.6, 780 x 780 target) with probability "
                           f"1/{args.serve_big_every} per arrival" if big else "")
                        + f"; continuous batching, {args.serve_budget_gib} GiB of slot arenas, "
                          f"streams per class {srv.streams_per_class}"}
    del srv
    gc.collect()                                     # the server's arenas go before the next one
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--per-launch-shots", type=int, default=64)
    ap.add_argument("--verify-shots", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--flags", type=int, default=0, help="batching constraint (0 line-or-column, 1 along, 2 none)")
    ap.add_argument("--traffic-gb", type=float, default=None, help="HBM bytes of one batching launch from PMC")
    ap.add_argument("--mixed-replays", type=int, default=3, help="graph replays of the uneven batch (0: skip)")
    ap.add_argument("--paper-shots", type=int, default=200,
                    help="shots of the paper's geometry timed one launch at a time (0: skip the form)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="served stream length (0: skip)")
    ap.add_argument("--serve-rates", type=str, default="20000,10000",
                    help="offered rates of the served stream, one run each (shots/s, comma separated)")
    ap.add_argument("--serve-pool", type=int, default=1024)
    ap.add_argument("--large-shots", type=int, default=16,
                    help="1024 x 1024 shots of the large-class form's many-instance launch (0: skip the form)")
    ap.add_argument("--large-flags", type=str, default="",
                    help="batching constraints (comma separated) of the large-class form's single shot (default --flags)")
    ap.add_argument("--serve-big-every", type=int, default=4096,
                    help="a 1024 x 1024 shot with probability 1/N per arrival of the served stream (0: none)")
    ap.add_argument("--serve-budget-gib", type=int, default=176)
    ap.add_argument("--serve-max-wave", type=int, default=1024)
    ap.add_argument("--single-launches", type=int, default=200,
                    help="synchronised launches per single-instance configuration and chain (0: skip those forms)")
    ap.add_argument("--no-variants", action="store_true", help="skip the serial-order and bird forms")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, run one plain device copy of this many MiB (a known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters of a --pmc run)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build measures the single-GPU kernel "
              "(multi-GPU shot sharding is design-only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    cpu, refs = None, {}
    if not args.no_cpu:                               # the CPU leg, before the GPU is touched
        cpu = cpu_baseline(args.cpu_seconds, args.cpu_workers)
        refs = oracle_references(args.verify_shots, args.paper_shots, args.flags)

    import numpy as np
    import torch

    import rr_inputs as ri
    from paper_2504_06182_amd import build as rrbuild
    if not os.path.exists(rrbuild.LIB):
        rrbuild.build()
    import paper_2504_06182_amd as rr
    from paper_2504_06182_amd.pipeline import BatchBuffers, ManyBuffers, SolveBuffers
    from paper_2504_06182_amd.tune import flags_for, solve_flags_for
    rr.lib()
    torch.cuda.set_device(0)
    dev = "cuda:0"

    shots = ri.config_shots(WORKLOAD)
    n = len(shots)
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    mb = ManyBuffers(shapes, device=dev, solve_flags=solve_flags_for(64)).load(grids)
    ws_one = rr.rr_batch_workspace_bytes(shapes[0], 2 * 44 * 44, STEP_BOUND_PER_SHOT)
    mb.alloc_pools(n * STEP_BOUND_PER_SHOT, n * (STEP_BOUND_PER_SHOT + 1), n * ((ws_one + 255) // 256 * 256))
    stream = torch.cuda.current_stream()

    bflags = flags_for(64, args.flags)          # the tuned launch schedule of the 64 class

    def step(ev=None):
        if ev: ev[0].record(stream)
        mb.solve(stream)
        if ev: ev[1].record(stream)
        mb.plan_device(stream)
        if ev: ev[2].record(stream)
        if ev:
            mb.batch(bflags, stream, graph_done_event=ev[3], loop_done_event=ev[4])
            ev[5].record(stream)
        else:
            mb.batch(bflags, stream)

    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    tot = mb.totals.cpu().numpy()
    assert tot[0] <= mb.step_pool and tot[2] <= mb.ws_pool, "pool bound too small for this workload"

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    for e in evs:                              # create the events the library records into
        for x in e:
            x.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    k_solve = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    k_plan = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    k_batch = float(np.mean([e[2].elapsed_time(e[5]) for e in evs]))
    k_graph = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    k_loop = float(np.mean([e[3].elapsed_time(e[4]) for e in evs]))
    k_generic = float(np.mean([e[4].elapsed_time(e[5]) for e in evs]))

    # results of the last timed step
    mb.refresh_desc()
    sinf, binf = mb.solve_infos(), mb.batch_infos()
    sstat = sinf[:, 0].view(np.int32)
    bstat = binf[:, 0].view(np.int32)
    assert np.all((sstat == 0) | (sstat == 1)) and np.all(bstat == 0), "a shot failed on the GPU"
    n_ok = int((sstat == 0).sum())
    n_moves, n_groups, n_steps = sinf[:, 1].astype(np.int64), sinf[:, 2].astype(np.int64), sinf[:, 3].astype(np.int64)
    n_batches = binf[:, 1].astype(np.int64)
    ws_words = np.array([s[1] * ((s[0] + 63) // 64) for s in shapes], np.int64)
    bytes_solve = int((16 * ws_words + 8 * n_moves + 4 * (n_groups + 1) + 24 + 80).sum())
    bytes_batch = int((8 * n_moves + 4 * (n_groups + 1) + 24 + 80 + 4 * n_steps + 4 * (n_batches + 1) + 20).sum())

    # bit-exact sample against the oracle's results computed in the CPU leg
    ref64 = refs.get(WORKLOAD, {})
    mv = mb.moves.cpu().numpy(); gr = mb.groups.cpu().numpy().view(np.uint32); fi = mb.final.cpu().numpy()
    st = mb.steps.cpu().numpy().view(np.uint32); bo = mb.batches.cpu().numpy().view(np.uint32)
    exact = 0
    for i, (r, rb) in ref64.items():
        g = mb.host_solve(i, sinf, mv, gr, fi)
        good = g["status"] == r["status"] and np.array_equal(g["final"], r["final"])
        if good and r["status"] == 0:
            good = np.array_equal(g["moves"], r["moves"]) and np.array_equal(g["group_off"], r["group_off"])
            gb = mb.host_batch(i, binf, st, bo)
            good = good and np.array_equal(gb["batch_off"], rb["batch_off"]) and np.array_equal(gb["steps"], rb["steps"])
        exact += int(good)

    # 1-per-launch form: rr_solve + rr_batch_moves per shot, one shot at a time
    lat = []
    per = []
    for i in range(min(args.per_launch_shots, n)):
        sb = SolveBuffers(shapes[i], device=dev).load(grids[i])
        bb = BatchBuffers(sb, step_cap=STEP_BOUND_PER_SHOT, device=dev)
        per.append((sb, bb))
    for sb, bb in per[:4]:
        sb.run(stream); bb.run(args.flags, stream)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for sb, bb in per:
        a = time.perf_counter()
        sb.run(stream)
        bb.run(args.flags, stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e6)
    tp1 = time.perf_counter()
    per_launch_sps = len(per) / (tp1 - tp0)
    lat = np.array(lat)

    single = single_instance_form(args, dev, refs) if args.single_launches > 0 else None
    chains = chain_form(args, dev, refs) if args.single_launches > 0 else None
    variants = variants_form(args, dev) if not args.no_variants else None
    paper = paper_geometry_form(args, dev, args.paper_shots, refs.get("paper32")) if args.paper_shots > 0 else None
    mixed = mixed_graph_form(args, dev, args.mixed_replays) if args.mixed_replays > 0 else None
    large = large_form(args, dev) if args.large_shots > 0 else None
    served = None
    if args.serve_seconds > 0:
        runs = [served_form(args, dev, float(r)) for r in args.serve_rates.split(",") if r.strip()]
        served = dict(runs[0])
        served["other_rates"] = runs[1:]

    value = n / (ms_per_step / 1e3)
    achieved = bytes_batch / (k_loop / 1e3) / 1e9
    traffic = measured_traffic(bflags) if args.traffic_gb is None else args.traffic_gb * 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "8192 shots, 64x64 trap grid, i.i.d. Bernoulli(0.55) loading, centred 44x44 "
                               "target; solve + batching (line-or-column constraint) per shot",
                   "shots": n, "grid": [64, 64], "target": [44, 44], "p": 0.55, "flags": bflags,
                   "schedule": {"solve_waves_per_instance": (mb.solve_flags >> 8) & 0xF or 4,
                                "graph_lds_kib": (bflags >> 24) & 0xFF, "loop_lds_kib": (bflags >> 8) & 0xFF}},
        "kernels_ms": {"solve_many": round(k_solve, 3), "plan_many": round(k_plan, 3), "batch_many": round(k_batch, 3),
                       "batch_graph": round(k_graph, 3), "batch_loop": round(k_loop, 3),
                       "batch_generic": round(k_generic, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": traffic, "kernel": "k_loop_many<2,0>",
                     "algorithmic_bytes_per_launch": bytes_batch},
        "solve_roofline": {"achieved": round(bytes_solve / (k_solve / 1e3) / 1e9, 2), "unit": "GB/s",
                           "algorithmic_bytes_per_launch": bytes_solve},
        "forms": {"batched_shots_per_s": round(value, 1),
                  "per_launch_shots_per_s": round(per_launch_sps, 1),
                  "batched_over_per_launch": round(value / per_launch_sps, 2),
                  "per_launch_p50_us": round(float(np.percentile(lat, 50)), 1),
                  "per_launch_p99_us": round(float(np.percentile(lat, 99)), 1),
                  "per_launch_sample": len(lat),
                  "batched_step_latency_us": round(ms_per_step * 1e3, 1),
                  "single_instance": single, "paper_geometry": paper, "mixed_graph": mixed,
                  "served": served, "variants": variants, "chains": chains, "large": large},
        "workload_stats": {"solved": n_ok, "infeasible": n - n_ok,
                           "mean_moves": round(float(n_moves.mean()), 1), "mean_steps": round(float(n_steps.mean()), 1),
                           "mean_batches": round(float(n_batches.mean()), 1),
                           "mean_pair_loop_iterations": (round(float(np.mean(refs["pair_loop_iterations"])), 1)
                                                         if refs.get("pair_loop_iterations") else None)},
        "bit_exact_sample": f"{exact}/{len(ref64)}" if ref64 else "not checked (--no-cpu)",
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

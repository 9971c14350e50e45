"""Launch-schedule autotuner for the solve and batching kernels.

A solve call carries one schedule knob in its flags word (include/rr.h): bits 8..11, the
wavefronts per instance (1, 2 or 4; at least one thread per grid side), i.e. how many waves
work one shot and how many shots a CU holds.  A batching call carries three:
  * bits 24..31 -- the graph kernel's LDS tile budget in KiB: how much of a grid's per-trap
    lists one workgroup holds at a time, hence workgroups per CU and, for large grids, the
    number of row ranges of the tiled build;
  * bits 20..23 -- the graph kernel's wavefronts per instance, over four (4, 8 or 16 waves);
  * bits 8..15 -- the loop kernel's LDS budget in KiB: the loop data of an instance in LDS or
    in the workspace, hence how many instance wavefronts one SIMD holds.
Neither changes a single result bit (the batches are Alg. 3's, whatever the schedule).  The
tuner times every candidate per grid size class on device-resident shots -- graph and loop
kernel apart, through the staged events of rr_batch_moves_many_staged -- keeps the fastest,
and checks on the way that every candidate's outputs equal the default schedule's.

The chosen schedules live in a small JSON table beside this file (``schedules.json``), keyed
by size class; ``flags_for`` merges them into a caller's flags.  Rerun on new hardware with
``python -m paper_2504_06182_amd.tune --write``.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "schedules.json")

SOLVE_WAVES = {64: (1, 2, 4), 128: (2, 4), 192: (4,), 256: (4,)}   # wavefronts per instance per class
DEFAULT_SOLVE_WAVES = 4
GRAPH_KIB = (24, 32, 48, 64, 96, 128, 150)
LOOP_KIB = (1, 4, 8, 16, 32, 64)
DEFAULT_GRAPH_KIB, DEFAULT_LOOP_KIB = 64, 1    # the library's own many-instance budgets
MARGIN = 0.03                                  # a candidate must beat the default by this much
GRAPH_WAVES = (4, 8, 16)                       # graph kernel wavefronts per instance
DEFAULT_GRAPH_WAVES = 8
_SCHED_MASK = (0xFF << 24) | (0xF << 20) | (0xFF << 8)


def schedule_bits(graph_kib: int, loop_kib: int, graph_waves: int = 0) -> int:
    """Flags bits of one schedule (both budgets in KiB, 1..255; graph wavefronts per instance
    4, 8 or 16, 0 for the library's default)."""
    if not (1 <= graph_kib <= 255 and 1 <= loop_kib <= 255):
        raise ValueError("LDS budgets are 1..255 KiB")
    if graph_waves not in (0, 4, 8, 16):
        raise ValueError("graph wavefronts per instance are 4, 8 or 16")
    return (int(graph_kib) << 24) | ((int(graph_waves) // 4) << 20) | (int(loop_kib) << 8)


def solve_flags_for(size_class: int, algo: int = 0, table: dict | None = None) -> int:
    """Solve flags for a class: the algorithm ``algo`` (bits 0..7) with the class's tuned
    wavefronts per instance (bits 8..11) -- unless ``algo`` sets them already."""
    algo = int(algo)
    if algo & (0xF << 8):
        return algo
    if table is None:
        if "t" not in _cache:
            _cache["t"] = load_table()
        table = _cache["t"]
    e = table["classes"].get(str(int(size_class)))
    w = int(e.get("solve_waves", 0)) if e else 0
    return algo | (w << 8)


def load_table(path: str = TABLE) -> dict:
    """The schedule table: {"classes": {"<side>": {"graph_kib": g, "loop_kib": l, ...}}, ...};
    empty when there is none."""
    if not os.path.exists(path):
        return {"classes": {}}
    with open(path) as f:
        t = json.load(f)
    if not isinstance(t.get("classes"), dict):
        raise ValueError(f"{path}: no 'classes' table")
    return t


_cache: dict = {}


def flags_for(size_class: int, flags: int = 0, table: dict | None = None) -> int:
    """``flags`` with the tuned schedule of ``size_class`` added -- unless the caller set a
    schedule of its own (any LDS budget bit), which always wins."""
    flags = int(flags)
    if flags & _SCHED_MASK:
        return flags
    if table is None:
        if "t" not in _cache:
            _cache["t"] = load_table()
        table = _cache["t"]
    e = table["classes"].get(str(int(size_class)))
    if not e:
        return flags
    return flags | schedule_bits(e["graph_kib"], e["loop_kib"], int(e.get("graph_waves", 0)))


def loop_lds_floor(side: int) -> int:
    """Bytes the loop kernel always keeps in LDS for a class of largest grid side ``side`` (its
    per-group counts and merge scratch: 8 B per group of at most 2 * side, 16 B per register
    position); the library raises a smaller loop budget to this, so smaller candidates are the
    same schedule."""
    slots = 2 if side <= 64 else (5 if side <= 128 else 6)
    return 8 * min(2 * side, 1024) + 16 * 64 * slots + 16


def _distinct_loop_budgets(side: int, loop_kib):
    """The loop budgets (KiB) that give distinct launches: of those at or below the floor, only
    the smallest."""
    floor = loop_lds_floor(side)
    out, seen_floor = [], False
    for k in sorted(int(v) for v in loop_kib):
        if k * 1024 <= floor:
            if seen_floor:
                continue
            seen_floor = True
        out.append(k)
    return out


def _run(mb, flags, reps):
    """Batch every instance of ``mb`` ``reps`` times; the best graph and loop kernel times (ms)
    and the outputs of the last run."""
    import torch

    g_best = l_best = float("inf")
    for _ in range(reps):
        mb.steps.zero_()
        mb.batches.zero_()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        mb.batch(flags, graph_done_event=e[1], loop_done_event=e[2])
        torch.cuda.synchronize()
        g_best = min(g_best, e[0].elapsed_time(e[1]))
        l_best = min(l_best, e[1].elapsed_time(e[2]))
    return g_best, l_best, (mb.batch_infos().copy(), mb.steps.clone(), mb.batches.clone())


def _same(a, b) -> bool:
    import torch

    return np.array_equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


def _pick(times: dict, default: int) -> int:
    """Fastest candidate, unless it is within MARGIN of the default (timing noise)."""
    best = min(times, key=times.get)
    if default in times and times[best] > (1.0 - MARGIN) * times[default]:
        return default
    return best


def _solve_run(mb, flags, reps):
    """Solve every instance of ``mb`` ``reps`` times under solve flags ``flags``; the best
    kernel time (ms) and the outputs of the last run (arenas cleared before each run)."""
    import torch

    best = float("inf")
    mb.solve_flags = int(flags)
    for _ in range(reps):
        for t in (mb.moves, mb.groups, mb.final, mb.sinfo):
            t.zero_()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        mb.solve()
        e[1].record()
        torch.cuda.synchronize()
        best = min(best, e[0].elapsed_time(e[1]))
    return best, (mb.sinfo.clone(), mb.moves.clone(), mb.groups.clone(), mb.final.clone())


def tune_solve(mb, side: int, reps: int = 3) -> dict:
    """Pick the wavefronts per instance of the solve for one size class (``mb`` loaded, the
    launch size of the workload); raises when a candidate's outputs differ from the default's."""
    import torch

    _, ref = _solve_run(mb, DEFAULT_SOLVE_WAVES << 8, 1)
    times = {}
    for w in SOLVE_WAVES[side]:
        t, out = _solve_run(mb, w << 8, reps)
        if not all(torch.equal(a, b) for a, b in zip(out, ref)):
            raise RuntimeError(f"{w} wavefronts per instance changed the solve outputs")
        times[w] = t
    mb.solve_flags = 0
    best = _pick(times, DEFAULT_SOLVE_WAVES)
    return {"solve_waves": best, "solve_ms": round(times[best], 3),
            "solve_ms_by_waves": {str(k): round(v, 3) for k, v in times.items()}}


def tune_class(mb, constraint: int = 0, graph_kib=GRAPH_KIB, loop_kib=LOOP_KIB, reps: int = 3) -> dict:
    """Pick the schedule of one size class.  ``mb``: a solved ManyBuffers of that class whose
    batching arenas are planned (plan_batches), holding as many shots as the launches to be
    tuned (the best loop budget depends on how many instance wavefronts share a SIMD).  The
    graph budget is chosen first (under the default loop budget), then the loop budget under
    it.  Raises when a candidate's outputs differ from the default schedule's."""
    constraint = int(constraint) & 0xFF
    _, _, ref = _run(mb, constraint, 1)
    gt = {}
    for g in graph_kib:
        t, _, out = _run(mb, constraint | (int(g) << 24), reps)
        if not _same(out, ref):
            raise RuntimeError(f"graph budget {g} KiB changed the batching outputs")
        gt[int(g)] = t
    best_g = _pick(gt, DEFAULT_GRAPH_KIB)
    wt = {}
    for gw in GRAPH_WAVES:
        t, _, out = _run(mb, constraint | (int(best_g) << 24) | ((int(gw) // 4) << 20), reps)
        if not _same(out, ref):
            raise RuntimeError(f"{gw} graph wavefronts per instance changed the batching outputs")
        wt[int(gw)] = t
    best_w = _pick(wt, DEFAULT_GRAPH_WAVES)
    lt = {}
    from .pipeline import size_class
    side = max(size_class(s) for s in mb.shapes)
    for lk in _distinct_loop_budgets(side, loop_kib):
        _, t, out = _run(mb, constraint | schedule_bits(best_g, lk, best_w), reps)
        if not _same(out, ref):
            raise RuntimeError(f"loop budget {lk} KiB changed the batching outputs")
        lt[int(lk)] = t
    best_l = _pick(lt, DEFAULT_LOOP_KIB)
    return {"graph_kib": best_g, "graph_waves": best_w, "loop_kib": best_l, "graph_ms": round(wt[best_w], 3),
            "graph_ms_by_waves": {str(k): round(v, 3) for k, v in wt.items()},
            "loop_ms": round(lt[best_l], 3), "graph_ms_by_kib": {str(k): round(v, 3) for k, v in gt.items()},
            "loop_ms_by_kib": {str(k): round(v, 3) for k, v in lt.items()}, "shots": mb.n}


def tune(shots_by_class: dict, constraint: int = 0, reps: int = 3, **kw) -> dict:
    """Tune every size class.  ``shots_by_class``: {side: (shapes, grids)}.  Returns a table."""
    import torch

    from .pipeline import ManyBuffers

    out = {"device": torch.cuda.get_device_name(), "constraint": int(constraint) & 0xFF, "classes": {}}
    for c, (shapes, grids) in sorted(shots_by_class.items()):
        mb = ManyBuffers(shapes).load(grids)
        sv = tune_solve(mb, int(c), reps)
        mb.solve()
        torch.cuda.synchronize()
        infos = mb.solve_infos()
        mb.plan_batches([max(int(i[3]), 1) for i in infos])
        out["classes"][str(int(c))] = {**tune_class(mb, constraint, reps=reps, **kw), **sv}
        del mb
        torch.cuda.empty_cache()
    return out


def _workload_shots(per_class: int | None):
    """The tuning sample: the 8192-shot 64 x 64 workload for the 64 class and the uneven batch's
    shots of the larger classes, as many as the workloads launch per class (or ``per_class``)."""
    import rr_inputs as ri

    from .pipeline import size_class

    by = {}
    for name in ("batch64", "mixed"):
        for d in ri.config_shots(name):
            s = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
            c = size_class(s)
            if name == "mixed" and c == 64:
                continue
            lst = by.setdefault(c, ([], []))
            if per_class is None or len(lst[0]) < per_class:
                lst[0].append(s)
                lst[1].append(ri.shot_grid(d))
    return by


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--per-class", type=int, default=None, help="shots per size class (default: the workloads')")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--constraint", type=int, default=0)
    ap.add_argument("--write", action="store_true", help=f"write the table to {TABLE}")
    ap.add_argument("--out", default=None, help="write the table to this path instead")
    a = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    t = tune(_workload_shots(a.per_class), a.constraint, a.reps)
    t["command"] = ("python -m paper_2504_06182_amd.tune" + (f" --per-class {a.per_class}" if a.per_class else "")
                    + f" --reps {a.reps} --write")
    print(json.dumps(t, indent=1), flush=True)
    path = a.out or (TABLE if a.write else None)
    if path:
        with open(path, "w") as f:
            json.dump(t, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()

"""GPU parity of the uneven batch's size classes and of its graph-captured pipeline.

Shots of the uneven workload (sides 32..256, p ~ U[0.5, 0.65], centred floor(0.7 n) target) are
run through ClassedBuffers: one solve -> device plan -> batch chain per size class, each class
under its tuned launch schedule.  Results are compared with the oracle (solve, and batching in
its indexed form, which is pinned byte for byte to the literal Alg. 3) under all three local
constraints, and the chains captured in one HIP graph are replayed over poisoned outputs and
compared in full with the eager pass.  Every case prints its name before it touches the GPU."""
import os
import sys

import numpy as np
import pytest

import oracle
import rr_inputs as ri

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_06182_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    import paper_2504_06182_amd
    paper_2504_06182_amd.lib()
    torch.cuda.set_device(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def shape_of(d):
    return (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])


def step_bound(shape):
    return int(0.11 * max(shape[0], shape[1]) ** 3) + 1024


def pick_mixed(per_side, sides, first=0):
    """The first ``per_side`` shots of each listed side in the seeded uneven workload."""
    got = {s: [] for s in sides}
    for d in ri.config_shots("mixed", n=4096 - first, first=first):
        if d["w"] in got and len(got[d["w"]]) < per_side:
            got[d["w"]].append(d)
        if all(len(v) == per_side for v in got.values()):
            break
    return [d for s in sides for d in got[s]]


def oracle_refs(shots, flags_list):
    refs = []
    for d in shots:
        shape, grid = shape_of(d), ri.shot_grid(d)
        r = oracle.solve(shape, grid)
        rbs = {}
        if r["status"] == 0:
            for f in flags_list:
                rbs[f] = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=f, indexed=True)
        refs.append((r, rbs))
    return refs


def same_solve(g, r, tag):
    assert g["status"] == r["status"], (tag, g["status"], r["status"])
    assert np.array_equal(g["final"], r["final"]), tag
    if r["status"] == 0:
        assert g["n_steps"] == r["n_steps"], tag
        assert np.array_equal(g["moves"], r["moves"]), tag
        assert np.array_equal(g["group_off"], r["group_off"]), tag


def same_batch(g, r, tag):
    assert g["status"] == r["status"], (tag, g["status"], r["status"])
    if r["status"] == 0:
        assert np.array_equal(g["batch_off"], r["batch_off"]), tag
        assert np.array_equal(g["steps"], r["steps"]), tag


def test_size_classes_against_oracle_all_constraints():
    """Two seeded uneven-batch shots at each side 96, 128, 192 and 256 (every class from 128
    up, the 128 class with both of its sides), launched through their own size-class buffers
    and tuned schedules: solve and batching equal the oracle under every constraint."""
    from paper_2504_06182_amd.pipeline import ClassedBuffers
    shots = pick_mixed(2, (96, 128, 192, 256))
    shapes = [shape_of(d) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    refs = oracle_refs(shots, (0, 1, 2))
    say("case size classes", [s[0] for s in shapes])
    cb = ClassedBuffers(shapes, step_bound).load(grids)
    assert sorted(c for c, _, _ in cb.parts) == [128, 192, 256]
    for flags in (0, 1, 2):
        say("  constraint", flags)
        cb.run(flags)
        torch.cuda.synchronize()
        assert not cb.fit_pools()
        for i, (r, rbs) in enumerate(refs):
            same_solve(cb.host_solve(i), r, f"shot {i} side {shapes[i][0]}")
            if r["status"] == 0:
                same_batch(cb.host_batch(i), rbs[flags], f"shot {i} side {shapes[i][0]} flags={flags}")


def test_graph_captured_pipeline_replays_equal_eager_and_oracle():
    """The uneven batch's per-class chains on their own streams, captured once in a HIP graph:
    three replays, each over outputs poisoned by an eager fill and with eager reads between
    them, write exactly the eager pass's bytes (infos, moves, group offsets, final grids, steps,
    batch offsets, planned descriptors); sampled shots of every class equal the oracle."""
    from paper_2504_06182_amd.pipeline import ClassedBuffers
    shots = ri.config_shots("mixed", n=96)
    shapes = [shape_of(d) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    say("case graph capture", len(shots))
    cb = ClassedBuffers(shapes, step_bound).load(grids)
    streams = [torch.cuda.Stream() for _ in cb.parts]
    cb.run(0, streams)
    torch.cuda.synchronize()
    assert not cb.fit_pools()
    cb.poison_outputs()
    cb.run(0, streams)
    torch.cuda.synchronize()
    ref = cb.outputs()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cb.run(0, streams)
    torch.cuda.synchronize()
    for rep in range(3):
        say("  replay", rep)
        cb.poison_outputs()
        torch.cuda.synchronize()
        assert not cb.same_outputs(cb.outputs(), ref)
        graph.replay()
        torch.cuda.synchronize()
        cb.infos()                                    # eager reads between replays
        assert cb.same_outputs(cb.outputs(), ref), f"replay {rep} differs from the eager pass"
    # two sampled shots per class against the oracle, from the last replay's outputs
    sample = []
    for c, idx, _ in cb.parts:
        sample += [int(i) for i in idx[:2]]
    for i in sample:
        r, rbs = oracle_refs([shots[i]], (0,))[0]
        say("  oracle shot", i, shapes[i])
        same_solve(cb.host_solve(i), r, f"graph shot {i}")
        if r["status"] == 0:
            same_batch(cb.host_batch(i), rbs[0], f"graph shot {i}")


def test_many_launch_refuses_workspace_region_out_of_bounds():
    """rr_batch_moves_many with a workspace one byte short of the last instance's region, and
    with a misaligned region: that instance reports RR_E_INVAL and none of its step or batch
    entries is written; the other instances equal the oracle."""
    from paper_2504_06182_amd import rr_batch_moves_many
    from paper_2504_06182_amd.pipeline import ManyBuffers
    shots = ri.config_shots("batch64", n=4)
    shapes = [shape_of(d) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    refs = oracle_refs(shots, (0,))
    say("case workspace bounds")
    mb = ManyBuffers(shapes).load(grids).solve()
    torch.cuda.synchronize()
    mb.plan_batches([max(int(i[3]), 1) for i in mb.solve_infos()])
    d = mb.desc_np
    last = len(shots) - 1

    def run(ws_bytes, desc_np):
        mb.desc.copy_(torch.from_numpy(desc_np.view(np.uint8).copy()).to(mb.desc.device))
        mb.steps.fill_(-1)
        mb.batches.fill_(-1)
        mb.binfo.fill_(0)
        rr_batch_moves_many(mb.n, mb.desc, mb.max_w, mb.max_h, mb.moves, mb.groups, mb.sinfo, 0, mb.batches,
                            mb.steps, mb.binfo, mb.ws, ws_bytes, None)
        torch.cuda.synchronize()
        return mb.batch_infos(), mb.steps.cpu().numpy(), mb.batches.cpu().numpy()

    short = mb.ws_bytes - 1
    assert int(d[last]["ws_off"]) < short
    binf, steps, batches = run(short, d)
    assert np.int32(binf[last][0]) == -1
    so, sc = int(d[last]["step_off"]), int(d[last]["step_cap"])
    bo = int(d[last]["batch_off"])
    assert np.all(steps[so:so + sc] == -1) and np.all(batches[bo:bo + sc + 1] == -1)
    for i in range(last):
        mb.desc_np = d
        same_batch(mb.host_batch(i, binf), refs[i][1][0], f"neighbour {i}")
    # a misaligned region (inside the workspace) is refused the same way
    d2 = d.copy()
    d2[1]["ws_off"] = int(d2[1]["ws_off"]) + 8
    binf, steps, batches = run(mb.ws_bytes, d2)
    assert np.int32(binf[1][0]) == -1
    so, sc, bo = int(d2[1]["step_off"]), int(d2[1]["step_cap"]), int(d2[1]["batch_off"])
    assert np.all(steps[so:so + sc] == -1) and np.all(batches[bo:bo + sc + 1] == -1)
    mb.desc_np = d2
    for i in (0, 2, 3):
        same_batch(mb.host_batch(i, binf), refs[i][1][0], f"aligned neighbour {i}")

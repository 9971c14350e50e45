"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle, bit for bit.

Every case prints its name before it touches the GPU.  Shapes span several 64-bit words per row
and column, ragged tails (W, H not multiples of 64), the empty/full/degenerate grids, the
full-width geometry of the paper, and the workloads' own sizes."""
import os
import sys

import numpy as np
import pytest

import oracle
import rr_inputs as ri
from checker import check_batches, check_solve

pytestmark = pytest.mark.gpu

GENERIC = 1 << 16   # RR_BATCH_GENERIC: the general batching path for every instance

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


def gpu_solve(shape, occ):
    from paper_2504_06182_amd.pipeline import SolveBuffers
    sb = SolveBuffers(shape).load(occ).run()
    torch.cuda.synchronize()
    return sb, sb.host()


def gpu_batch(sb, n_steps, flags):
    from paper_2504_06182_amd.pipeline import BatchBuffers
    bb = BatchBuffers(sb, step_cap=max(n_steps, 1)).run(flags=flags)
    torch.cuda.synchronize()
    return bb.host()


def same_solve(g, r, tag=""):
    assert g["status"] == r["status"], (tag, g["status"], r["status"])
    assert np.array_equal(g["final"], r["final"]), tag
    if r["status"] == 0:
        assert g["n_steps"] == r["n_steps"], tag
        assert np.array_equal(g["moves"], r["moves"]), tag
        assert np.array_equal(g["group_off"], r["group_off"]), tag


def same_batch(g, r, tag=""):
    assert g["status"] == r["status"], (tag, g["status"], r["status"])
    if r["status"] == 0:
        assert np.array_equal(g["batch_off"], r["batch_off"]), tag
        assert np.array_equal(g["steps"], r["steps"]), tag


def dense(w, h, fn):
    g = np.zeros((h, w), np.uint8)
    for y in range(h):
        for x in range(w):
            g[y, x] = 1 if fn(x, y) else 0
    return g


def centred(w, h, sw, sh):
    return (w, h, *ri.centred_target(w, h, sw, sh))


ADVERSARIAL = [
    ("empty", (32, 32, 8, 8, 24, 24), lambda x, y: False),
    ("full", (32, 32, 8, 8, 24, 24), lambda x, y: True),
    ("checker64", centred(64, 64, 44, 44), lambda x, y: (x + y) % 2 == 0),
    ("left_half", centred(64, 64, 30, 30), lambda x, y: x < 32),
    ("top_rows_only", centred(48, 48, 20, 20), lambda x, y: y >= 34),
    ("deep_receiver", (40, 40, 0, 10, 40, 30), lambda x, y: x != 17 and (x * 7 + y * 3) % 5 != 0),
    ("mirror", centred(50, 50, 30, 30), lambda x, y: ((min(x, 49 - x) * 13 + y * 7) % 5) < 3),
    ("ragged_65x70", centred(65, 70, 40, 47), lambda x, y: (x * 31 + y * 17) % 7 < 4),
    ("ragged_100x37", centred(100, 37, 70, 20), lambda x, y: (x * 11 + y * 5) % 9 < 6),
    ("ragged_130x129", centred(130, 129, 91, 90), lambda x, y: (x * 3 + y * 29) % 11 < 7),
    ("paper_full_width", (32, 54, 0, 11, 32, 43), lambda x, y: (x * 5 + y * 13) % 10 < 6),
    ("one_cell", (1, 1, 0, 0, 1, 1), lambda x, y: True),
    ("line_1x9", (1, 9, 0, 3, 1, 6), lambda x, y: y in (0, 1, 8)),
    ("line_9x1", (9, 1, 3, 0, 6, 1), lambda x, y: x in (0, 7, 8)),
    ("thin_target", centred(64, 64, 1, 40), lambda x, y: (x + 3 * y) % 4 == 0),
    ("corner_target", (64, 64, 0, 0, 20, 20), lambda x, y: (x * y) % 3 != 0),
    ("max_256", centred(256, 256, 179, 179), lambda x, y: (x * 7 + y * 11) % 10 < 6),
]


@pytest.mark.parametrize("name,shape,fn", ADVERSARIAL, ids=[a[0] for a in ADVERSARIAL])
def test_adversarial_solve_and_batch(name, shape, fn):
    say("case", name, shape)
    occ = ri.pack_rows(dense(shape[0], shape[1], fn))
    sb, g = gpu_solve(shape, occ)
    r = oracle.solve(shape, occ)
    same_solve(g, r, name)
    if r["status"] == 0:
        check_solve(shape, occ, g)
        big = shape[0] * shape[1] > 130 * 130
        for flags in ((0,) if big else (0, 1, 2, GENERIC, 1 | GENERIC, 2 | GENERIC, 1 << 8)):
            gb = gpu_batch(sb, g["n_steps"], flags)
            rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags & 0xFF)
            same_batch(gb, rb, f"{name} flags={flags:#x}")
            if not big:
                check_batches(shape, occ, g["moves"], g["final"], gb["batch_off"], gb["steps"], flags & 0xFF)


@pytest.mark.parametrize("seed", range(24))
def test_random_shapes(seed):
    rng = np.random.default_rng(seed)
    w, h = int(rng.integers(1, 200)), int(rng.integers(1, 200))
    sw, sh = int(rng.integers(1, w + 1)), int(rng.integers(1, h + 1))
    x0, y0 = int(rng.integers(0, w - sw + 1)), int(rng.integers(0, h - sh + 1))
    shape = (w, h, x0, y0, x0 + sw, y0 + sh)
    p = float(rng.choice([0.3, 0.5, 0.6, 0.8]))
    say("case random", seed, shape, p)
    occ = ri.pack_rows(ri.bernoulli_grid(900, seed, w, h, p))
    sb, g = gpu_solve(shape, occ)
    r = oracle.solve(shape, occ)
    same_solve(g, r, f"seed {seed}")
    if r["status"] == 0 and w * h <= 100 * 100:
        flags = seed % 3
        gb = gpu_batch(sb, g["n_steps"], flags)
        rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags)
        same_batch(gb, rb, f"seed {seed}")


@pytest.mark.parametrize("name", ["single32", "single128"])
def test_single_instance_workloads(name):
    d = ri.config_shots(name)[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    say("case", name, shape)
    occ = ri.shot_grid(d)
    sb, g = gpu_solve(shape, occ)
    r = oracle.solve(shape, occ)
    same_solve(g, r, name)
    for flags in (0, 1, 2):
        gb = gpu_batch(sb, g["n_steps"], flags)
        rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags)
        same_batch(gb, rb, f"{name} flags={flags}")


def run_many(shots, flags=0):
    from paper_2504_06182_amd.pipeline import ManyBuffers
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    mb = ManyBuffers(shapes).load(grids).solve()
    torch.cuda.synchronize()
    infos = mb.solve_infos()
    mb.plan_batches([max(int(i[3]), 1) for i in infos]).batch(flags=flags)
    torch.cuda.synchronize()
    return mb, shapes, grids


def test_batch64_full_size_sampled():
    """8192 shots of 64x64 in one launch each for solve and batching (the timed configuration);
    32 shots compared bit for bit with the oracle, every shot checked for consistency."""
    shots = ri.config_shots("batch64")
    say("case batch64 full", len(shots))
    mb, shapes, grids = run_many(shots)
    sinf, binf = mb.solve_infos(), mb.batch_infos()
    assert np.all((sinf[:, 0] == 0) | (sinf[:, 0] == 1))
    ok = sinf[:, 0] == 0
    assert np.all(binf[:, 0] == 0)
    assert np.array_equal(binf[ok, 2], sinf[ok, 3]), "batched steps differ from solved steps"
    moves = mb.moves.cpu().numpy(); groups = mb.groups.cpu().numpy().view(np.uint32)
    final = mb.final.cpu().numpy(); steps = mb.steps.cpu().numpy().view(np.uint32)
    batches = mb.batches.cpu().numpy().view(np.uint32)
    for i in np.linspace(0, len(shots) - 1, 32).astype(int):
        g = mb.host_solve(i, sinf, moves, groups, final)
        r = oracle.solve(shapes[i], grids[i])
        same_solve(g, r, f"shot {i}")
        if r["status"] == 0:
            gb = mb.host_batch(i, binf, steps, batches)
            rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"])
            same_batch(gb, rb, f"shot {i}")


def test_many_equals_one_and_mixed_sizes():
    """Uneven sizes in one launch: every instance equals its single-instance launch and the
    oracle (solve for all, batching for the smaller grids)."""
    shots = ri.config_shots("mixed", n=48)
    say("case mixed 48")
    mb, shapes, grids = run_many(shots)
    sinf, binf = mb.solve_infos(), mb.batch_infos()
    for i in range(len(shots)):
        g = mb.host_solve(i, sinf)
        r = oracle.solve(shapes[i], grids[i])
        same_solve(g, r, f"mixed {i}")
        sb, g1 = gpu_solve(shapes[i], grids[i])
        same_solve(g1, r, f"mixed single {i}")
        if r["status"] == 0 and shapes[i][0] <= 96:
            gb = mb.host_batch(i, binf)
            rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"])
            same_batch(gb, rb, f"mixed batch {i}")


def test_capacity_and_device_side_errors():
    from paper_2504_06182_amd.pipeline import BatchBuffers, SolveBuffers
    d = ri.config_shots("single32")[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    occ = ri.shot_grid(d)
    say("case capacity")
    r = oracle.solve(shape, occ)
    sb = SolveBuffers(shape, move_cap=10).load(occ).run()
    torch.cuda.synchronize()
    g = sb.host()
    assert g["status"] == -2 and g["need_moves"] == len(r["moves"]) and g["need_groups"] == len(r["group_off"]) - 1
    sb2 = SolveBuffers(shape, group_cap=3).load(occ).run()
    torch.cuda.synchronize()
    assert sb2.host()["status"] == -2
    sb3, g3 = gpu_solve(shape, occ)
    bb = BatchBuffers(sb3, step_cap=g3["n_steps"], batch_cap=5).run()
    torch.cuda.synchronize()
    rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"])
    h = bb.host()
    assert h["status"] == -2 and h["need_batches"] == len(rb["batch_off"]) - 1 and h["need_steps"] == r["n_steps"]
    bb2 = BatchBuffers(sb3, step_cap=g3["n_steps"] - 1).run()
    torch.cuda.synchronize()
    h2 = bb2.host()
    assert h2["status"] == -2 and h2["need_steps"] == r["n_steps"]
    # a malformed move list on the device: a zero-length move
    mv = sb3.moves.cpu().numpy().view(np.uint16).reshape(-1, 4).copy()
    mv[0, 2], mv[0, 3] = mv[0, 0], mv[0, 1]
    sb3.moves.copy_(torch.from_numpy(mv.reshape(-1).view(np.int64)).cuda())
    bb3 = BatchBuffers(sb3, step_cap=g3["n_steps"]).run()
    torch.cuda.synchronize()
    assert bb3.host()["status"] == -1


def test_repeat_runs_are_identical():
    shots = ri.config_shots("batch64", n=64)
    say("case determinism")
    a, _, _ = run_many(shots)
    b, _, _ = run_many(shots)
    assert np.array_equal(a.solve_infos(), b.solve_infos())
    assert np.array_equal(a.batch_infos(), b.batch_infos())
    for i in range(len(shots)):
        sa, sb_ = a.host_solve(i), b.host_solve(i)
        same_solve(sa, sb_, f"repeat {i}")
        same_batch(a.host_batch(i), b.host_batch(i), f"repeat {i}")


def test_device_planner_matches_host_plan_and_reports_overflow():
    """rr_plan_many lays out the arenas on the device; results equal the host-planned launch, and
    instances beyond a too-small pool report RR_E_CAPACITY with their exact step count."""
    from paper_2504_06182_amd.pipeline import ManyBuffers
    shots = ri.config_shots("mixed", n=40)
    say("case device planner")
    ref, shapes, grids = run_many(shots)
    sinf = ref.solve_infos()
    import paper_2504_06182_amd as rr
    caps = [max(int(i[3]), 1) if i[0] == 0 else 1 for i in sinf]
    ws_need = sum((rr.rr_batch_workspace_bytes(s, 2 * (s[4] - s[2]) * (s[5] - s[3]), c) + 255) // 256 * 256
                  for s, c in zip(shapes, caps))
    mb = ManyBuffers(shapes).load(grids).solve()
    mb.alloc_pools(sum(caps), sum(caps) + len(caps), ws_need).plan_device().batch()
    torch.cuda.synchronize()
    mb.refresh_desc()
    tot = mb.totals.cpu().numpy()
    assert tot[0] == sum(caps) and tot[1] == sum(caps) + len(caps) and tot[2] == ws_need
    for i in range(len(shots)):
        same_batch(mb.host_batch(i), ref.host_batch(i), f"planned {i}")
    # a pool that holds only the first few instances
    small = ManyBuffers(shapes).load(grids).solve()
    cut = int(sum(caps[:5]))
    small.alloc_pools(cut, sum(caps) + len(caps), ws_need).plan_device().batch()
    torch.cuda.synchronize()
    small.refresh_desc()
    binf = small.batch_infos()
    for i in range(len(shots)):
        if i < 5:
            same_batch(small.host_batch(i, binf), ref.host_batch(i), f"small {i}")
        elif sinf[i][0] == 0:
            assert np.int32(binf[i][0]) == -2 and binf[i][4] == sinf[i][3]


def test_fast_path_equals_general_path_and_lds_budgets():
    """The batching paths agree byte for byte, on uneven sizes and the bench grid, for every
    constraint: the default launch (graph in LDS, or in LDS row tiles for grids beyond 64 KiB;
    loop data in the workspace) against the general path, the loop data in LDS (64 KiB loop
    budget), the graph in many small row tiles (12 KiB graph budget) and the graph in the
    workspace (2 KiB: below one tile); the smaller grids also against the oracle."""
    shots = ri.config_shots("mixed", n=21) + ri.config_shots("batch64", n=6)
    variants = {"general": GENERIC, "loop in LDS": 64 << 8, "graph in 12 KiB tiles": 12 << 24,
                "graph in the workspace": 2 << 24, "graph on 4 wavefronts per instance": (64 << 24) | (1 << 20),
                "graph on 16 wavefronts per instance": (64 << 24) | (4 << 20)}
    for flags in (0, 1, 2):
        say("case paths flags", flags)
        ref, shapes, grids = run_many(shots, flags)
        binf = ref.batch_infos()
        for name, extra in variants.items():
            say("  variant", name)
            other, _, _ = run_many(shots, flags | extra)
            for i in range(len(shots)):
                same_batch(other.host_batch(i), ref.host_batch(i, binf), f"{name} {i} flags={flags}")
        for i in range(len(shots)):
            if shapes[i][0] <= 64:
                r = oracle.solve(shapes[i], grids[i])
                if r["status"] == 0:
                    rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"], flags=flags)
                    same_batch(ref.host_batch(i, binf), rb, f"oracle {i} flags={flags}")


def _load_crafted(sb, mv, goff, n_steps):
    """Put a hand-made move list into a SolveBuffers as if the solve had emitted it."""
    assert len(mv) <= sb.move_cap and len(goff) - 1 <= sb.group_cap
    m = np.zeros(sb.move_cap * 4, np.uint16)
    m[:mv.size] = mv.reshape(-1)
    sb.moves.copy_(torch.from_numpy(m.view(np.int64)).cuda())
    g = np.zeros(sb.group_cap + 1, np.uint32)
    g[:len(goff)] = goff
    sb.group_off.copy_(torch.from_numpy(g.view(np.int32)).cuda())
    info = np.zeros(sb.info.numel(), np.uint32)
    info[:6] = (0, len(mv), len(goff) - 1, n_steps, len(mv), len(goff) - 1)
    sb.info.copy_(torch.from_numpy(info.view(np.int32)).cuda())


def test_ready_set_overflow_hands_over_to_general_path():
    """A ready set that outgrows the loop's registers mid-run (hand-made wide release: 4 ready
    moves, then 240 at once on a 64 x 64 grid, whose loop holds 128): the instance is redone on
    the general path, with the oracle's batches, in one-instance and many-instance launches and
    with the loop data in LDS and in the workspace."""
    from crafted import wide_release
    from paper_2504_06182_amd.pipeline import SolveBuffers, ManyBuffers
    shape, mv, goff, n_steps = wide_release()
    say("case overflow single", shape)
    sb = SolveBuffers(shape)
    _load_crafted(sb, mv, goff, n_steps)
    torch.cuda.synchronize()
    for flags in (0, 1, 2, 1 << 8):
        rb = oracle.batch(shape, mv, goff, n_steps, flags=flags & 0xFF)
        same_batch(gpu_batch(sb, n_steps, flags), rb, f"overflow single flags={flags}")
    say("case overflow many")
    shots = ri.config_shots("batch64", n=3)
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    mb = ManyBuffers(shapes).load([ri.shot_grid(d) for d in shots]).solve()
    torch.cuda.synchronize()
    # instance 1 takes the hand-made moves (same 64 x 64 grid; its target is not read here)
    d1 = mb.desc_np[1]
    mo, go = int(d1["move_off"]), int(d1["group_off"])
    assert len(mv) <= int(d1["move_cap"]) and len(goff) - 1 <= int(d1["group_cap"])
    moves = mb.moves.cpu().numpy().copy()
    moves[mo:mo + len(mv)] = np.ascontiguousarray(mv).reshape(-1).view(np.int64)
    mb.moves.copy_(torch.from_numpy(moves).cuda())
    groups = mb.groups.cpu().numpy().copy()
    groups[go:go + len(goff)] = goff.view(np.int32)
    mb.groups.copy_(torch.from_numpy(groups).cuda())
    sinf = mb.solve_infos().copy()
    sinf[1, :6] = (0, len(mv), len(goff) - 1, n_steps, len(mv), len(goff) - 1)
    mb.sinfo.copy_(torch.from_numpy(sinf.reshape(-1).view(np.int32)).cuda())
    torch.cuda.synchronize()
    mb.plan_batches([max(int(i[3]), 1) for i in sinf])
    for flags in (0, 1, 2, 1 << 8):
        mb.batch(flags=flags)
        torch.cuda.synchronize()
        binf = mb.batch_infos()
        rb = oracle.batch(shape, mv, goff, n_steps, flags=flags & 0xFF)
        same_batch(mb.host_batch(1, binf), rb, f"overflow many flags={flags}")
        for i in (0, 2):
            r = oracle.solve(shapes[i], ri.shot_grid(shots[i]))
            rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"], flags=flags & 0xFF)
            same_batch(mb.host_batch(i, binf), rb, f"overflow neighbour {i} flags={flags}")


def test_paper_geometry_many_and_single():
    """The paper's benchmark geometry (32 x 54 traps, full-width 32 x 32 target, exactly 1036
    atoms): 64 shots in one launch and 4 one at a time, solve and batching against the oracle."""
    shots = ri.config_shots("paper32", n=64)
    say("case paper32 many", len(shots))
    mb, shapes, grids = run_many(shots)
    sinf, binf = mb.solve_infos(), mb.batch_infos()
    for i in range(len(shots)):
        r = oracle.solve(shapes[i], grids[i])
        same_solve(mb.host_solve(i, sinf), r, f"paper32 {i}")
        rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"])
        same_batch(mb.host_batch(i, binf), rb, f"paper32 batch {i}")
    for i in range(4):
        say("case paper32 single", i)
        sb, g = gpu_solve(shapes[i], grids[i])
        r = oracle.solve(shapes[i], grids[i])
        same_solve(g, r, f"paper32 single {i}")
        for flags in (0, 1, 2):
            rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"], flags=flags)
            same_batch(gpu_batch(sb, g["n_steps"], flags), rb, f"paper32 single {i} flags={flags}")


def test_tiled_graph_with_queue_overflow():
    """A hand-made instance whose touch lists exceed the graph budget (tiled build) and whose
    one row carries 600 long horizontal legs (more than the per-range wave queue holds): its
    batches equal the oracle's in a many-instance launch and, with a 32 KiB graph budget, in a
    one-instance launch."""
    from crafted import long_row
    from paper_2504_06182_amd.pipeline import SolveBuffers, ManyBuffers
    shape, mv, goff, n_steps = long_row()
    rb = oracle.batch(shape, mv, goff, n_steps)
    say("case long row single")
    sb = SolveBuffers(shape)
    _load_crafted(sb, mv, goff, n_steps)
    torch.cuda.synchronize()
    same_batch(gpu_batch(sb, n_steps, 32 << 24), rb, "long row single")
    say("case long row many")
    shots = ri.config_shots("batch64", n=3)
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    mb = ManyBuffers(shapes).load([ri.shot_grid(d) for d in shots]).solve()
    torch.cuda.synchronize()
    d1 = mb.desc_np[1]
    mo, go = int(d1["move_off"]), int(d1["group_off"])
    moves = mb.moves.cpu().numpy().copy()
    moves[mo:mo + len(mv)] = np.ascontiguousarray(mv).reshape(-1).view(np.int64)
    mb.moves.copy_(torch.from_numpy(moves).cuda())
    groups = mb.groups.cpu().numpy().copy()
    groups[go:go + len(goff)] = goff.view(np.int32)
    mb.groups.copy_(torch.from_numpy(groups).cuda())
    sinf = mb.solve_infos().copy()
    sinf[1, :6] = (0, len(mv), len(goff) - 1, n_steps, len(mv), len(goff) - 1)
    mb.sinfo.copy_(torch.from_numpy(sinf.reshape(-1).view(np.int32)).cuda())
    torch.cuda.synchronize()
    mb.plan_batches([max(int(i[3]), 1) for i in sinf])
    mb.batch(0)
    torch.cuda.synchronize()
    binf = mb.batch_infos()
    same_batch(mb.host_batch(1, binf), rb, "long row many")
    for i in (0, 2):
        r = oracle.solve(shapes[i], ri.shot_grid(shots[i]))
        same_batch(mb.host_batch(i, binf), oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"]),
                   f"long row neighbour {i}")

"""GPU parity of the grids beyond 256 per side (the wide kernels) through the C ABI, against the
oracle bit for bit: the solve (state in the caller's workspace, 16 wavefronts) for all three
algorithms, and the wide batching path (graph from path meetings and a per-trap last-group
sweep, one-wave loop with the ready set in LDS) under all three constraints, compared with the
oracle's indexed form.  Wide but short grids (W just past 256, a few to 40 rows) give many
quick instances with ragged tails; 512 x 512 and the seeded 1024 x 1024 shot of the served
stream's large class run at full size.  Every case prints its name before it touches the GPU."""
import os
import random
import sys

import numpy as np
import pytest

import oracle
import rr_inputs as ri

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SERIAL, BIRD = 1, 2


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


def gpu_solve(shape, occ, algo=0):
    from paper_2504_06182_amd.pipeline import SolveBuffers
    sb = SolveBuffers(shape, flags=algo).load(occ).run()
    torch.cuda.synchronize()
    return sb, sb.host()


def gpu_batch(sb, n_steps, flags, step_cap=None, batch_cap=None):
    from paper_2504_06182_amd.pipeline import BatchBuffers
    bb = BatchBuffers(sb, step_cap=max(n_steps, 1) if step_cap is None else step_cap, batch_cap=batch_cap)
    bb.run(flags=flags)
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


def oracle_solve(shape, occ, algo=0):
    return oracle.solve(shape, occ, serial=algo == SERIAL, bird=algo == BIRD)


def random_wide(rng, i):
    """A grid just past 256 columns (or rows), 4..40 in the other direction, random target."""
    long_, short = rng.randint(257, 330), rng.randint(4, 40)
    w, h = (long_, short) if rng.random() < 0.6 else (short, long_)
    if rng.random() < 0.4:
        x0, x1 = 0, w
    else:
        sw = rng.randint(1, w)
        x0 = rng.randint(0, w - sw)
        x1 = x0 + sw
    sh = rng.randint(1, h)
    y0 = rng.randint(0, h - sh)
    p = rng.choice([0.45, 0.6, 0.75, 0.9])
    return (w, h, x0, y0, x1, y0 + sh), ri.pack_rows(ri.bernoulli_grid(900, i, w, h, p))


def test_wide_solve_every_algorithm():
    """Grids of 257 to 1024 per side, square and not, full-width and side-column targets, a
    refused instance: each algorithm equals the oracle."""
    cases = [((257, 257, 0, 38, 257, 219), 0.6), ((300, 300, 45, 45, 255, 255), 0.55),
             ((400, 280, 60, 40, 340, 240), 0.6), ((270, 33, 20, 5, 250, 28), 0.7),
             ((33, 290, 3, 20, 30, 270), 0.7), ((512, 512, 77, 77, 435, 435), 0.6),
             ((300, 300, 0, 0, 300, 300), 0.3)]
    for k, (shape, p) in enumerate(cases):
        occ = ri.pack_rows(ri.bernoulli_grid(901, k, shape[0], shape[1], p))
        for algo in (0, SERIAL, BIRD):
            say("case wide solve", shape, algo)
            r = oracle_solve(shape, occ, algo)
            _, g = gpu_solve(shape, occ, algo)
            same_solve(g, r, f"{shape} algo {algo}")
    assert r["status"] == 1


def test_wide_batch_random_short_grids():
    """60 random grids just past 256 per side: solve and batching under every constraint equal
    the oracle (batching: its indexed form)."""
    rng = random.Random(257)
    n_batched = 0
    for i in range(60):
        shape, occ = random_wide(rng, i)
        say("case wide random", i, shape)
        r = oracle.solve(shape, occ)
        sb, g = gpu_solve(shape, occ)
        same_solve(g, r, f"random {i}")
        if r["status"] != 0:
            continue
        n_batched += 1
        for flags in (0, 1, 2):
            rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags, indexed=True)
            gb = gpu_batch(sb, r["n_steps"], flags)
            same_batch(gb, rb, f"random {i} {shape} flags {flags}")
    assert n_batched >= 30


@pytest.mark.parametrize("algo", [0, SERIAL, BIRD], ids=["parallel", "serial", "bird"])
def test_wide_batch_512(algo):
    """A 512 x 512 shot (p 0.6, centred 358 x 358 target): every constraint equals the oracle."""
    side, s = 512, 358
    x0 = (side - s) // 2
    shape = (side, side, x0, x0, x0 + s, x0 + s)
    occ = ri.pack_rows(ri.bernoulli_grid(902, algo, side, side, 0.6))
    say("case wide 512", algo)
    r = oracle_solve(shape, occ, algo)
    sb, g = gpu_solve(shape, occ, algo)
    same_solve(g, r, "512")
    assert r["status"] == 0
    for flags in (0, 1, 2):
        rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags, indexed=True)
        same_batch(gpu_batch(sb, r["n_steps"], flags), rb, f"512 flags {flags}")


def test_wide_seeded_1024_shot():
    """The served stream's large class at full size: the seeded 1024 x 1024 shot (p 0.6, 780 x 780
    target; 639,731 moves, 95,164,481 unit steps): solve and line-or-column batching equal the
    oracle."""
    d = ri.config_shots("big1024")[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    occ = ri.shot_grid(d)
    say("case wide 1024 solve")
    r = oracle.solve(shape, occ)
    sb, g = gpu_solve(shape, occ)
    same_solve(g, r, "1024")
    say("case wide 1024 batch")
    gb = gpu_batch(sb, r["n_steps"], 0)
    rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=0, indexed=True)
    same_batch(gb, rb, "1024")


def test_wide_and_small_instances_in_one_launch():
    """Small and wide grids in one many-instance launch (solve and batching run both kernel
    families, each skipping the other's instances): every instance equals the oracle and its
    single-instance launch."""
    from paper_2504_06182_amd.pipeline import ManyBuffers
    rng = random.Random(258)
    shapes, grids = [], []
    for i in range(12):
        if i % 3 == 0:
            d = ri.config_shots("mixed", n=12)[i]
            shapes.append((d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]))
            grids.append(ri.shot_grid(d))
        else:
            s, occ = random_wide(rng, 100 + i)
            shapes.append(s)
            grids.append(occ)
    say("case wide many", len(shapes))
    mb = ManyBuffers(shapes).load(grids).solve()
    torch.cuda.synchronize()
    sinf = mb.solve_infos()
    mb.plan_batches([max(int(x[3]), 1) for x in sinf]).batch(flags=0)
    torch.cuda.synchronize()
    binf = mb.batch_infos()
    for i, (shape, occ) in enumerate(zip(shapes, grids)):
        r = oracle.solve(shape, occ)
        same_solve(mb.host_solve(i, sinf), r, f"many {i} {shape}")
        if r["status"] == 0:
            rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=0, indexed=True)
            same_batch(mb.host_batch(i, binf), rb, f"many batch {i} {shape}")


def test_wide_capacity_and_status():
    """Wide path statuses: steps one short and batches one short give RR_E_CAPACITY with the
    exact needs; a refused solve batches to nothing; a solve workspace one byte short and a
    nonzero wavefront field are refused before launch."""
    import paper_2504_06182_amd as rr
    from paper_2504_06182_amd.pipeline import SolveBuffers
    shape, occ = (300, 24, 10, 4, 290, 20), ri.pack_rows(ri.bernoulli_grid(903, 0, 300, 24, 0.7))
    say("case wide capacity")
    r = oracle.solve(shape, occ)
    assert r["status"] == 0
    rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=0, indexed=True)
    nb = len(rb["batch_off"]) - 1
    sb, g = gpu_solve(shape, occ)
    h = gpu_batch(sb, r["n_steps"], 0, step_cap=r["n_steps"] - 1)
    assert h["status"] == -2 and h["need_steps"] == r["n_steps"]
    h = gpu_batch(sb, r["n_steps"], 0, batch_cap=nb - 1)
    assert h["status"] == -2 and h["need_batches"] == nb and h["need_steps"] == r["n_steps"]
    refused = ri.pack_rows(ri.bernoulli_grid(903, 1, 300, 24, 0.1))
    sb2, g2 = gpu_solve(shape, refused)
    assert g2["status"] == 1
    h2 = gpu_batch(sb2, 0, 0)
    assert h2["status"] == 0 and h2["n_batches"] == 0
    s3 = SolveBuffers(shape)
    rc = rr.rr_solve(shape, s3.occ, s3.moves, s3.move_cap, s3.group_off, s3.group_cap, s3.final, s3.info, 0,
                     s3.ws, s3.ws_bytes - 1, stream=None, check=False)
    assert rc == rr.RR_E_NOMEM
    rc = rr.rr_solve(shape, s3.occ, s3.moves, s3.move_cap, s3.group_off, s3.group_cap, s3.final, s3.info, 4 << 8,
                     s3.ws, s3.ws_bytes, stream=None, check=False)
    assert rc == rr.RR_E_INVAL


def test_wide_degenerate_shapes():
    """Thin and extreme wide grids: one row or one column of 1024 traps, two rows of 700, 1024 x 3
    and 3 x 1024 with side-column targets, a full target on a 300 x 300 grid loaded at 0.95, a
    single-trap target: solve and line-or-column batching equal the oracle (a refused instance
    batches to nothing)."""
    cases = [((1024, 1, 100, 0, 900, 1), 0.8), ((1, 1024, 0, 100, 1, 900), 0.8), ((700, 2, 50, 0, 650, 2), 0.9),
             ((1024, 3, 10, 1, 1000, 2), 0.5), ((3, 1024, 1, 10, 2, 1000), 0.5), ((300, 300, 0, 0, 300, 300), 0.95),
             ((400, 300, 200, 150, 201, 151), 0.3)]
    for k, (shape, p) in enumerate(cases):
        occ = ri.pack_rows(ri.bernoulli_grid(904, k, shape[0], shape[1], p))
        say("case wide degenerate", shape)
        r = oracle.solve(shape, occ)
        sb, g = gpu_solve(shape, occ)
        same_solve(g, r, f"degenerate {shape}")
        if r["status"] == 0:
            rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=0, indexed=True)
            same_batch(gpu_batch(sb, r["n_steps"], 0), rb, f"degenerate batch {shape}")
        else:
            h = gpu_batch(sb, 0, 0)
            assert h["status"] == 0 and h["n_batches"] == 0

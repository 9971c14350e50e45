"""GPU parity of the solver variants, through the C ABI, against the oracle's same variant, bit
for bit: the serial order of Alg. 1 (RR_REDREC_SERIAL) and bird (Alg. 2, RR_BIRD).  Moves, group
offsets, final grids, step counts, and the batches of the variant's moves.  Every case prints
its name before it touches the GPU."""
import glob
import json
import os
import sys

import numpy as np
import pytest

import oracle
import rr_inputs as ri
from checker import check_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SERIAL, BIRD = 1, 2          # RR_REDREC_SERIAL, RR_BIRD
VARIANTS = [SERIAL, BIRD]
NAMES = {SERIAL: "serial", BIRD: "bird"}


def oracle_solve(shape, occ, algo):
    return oracle.solve(shape, occ, serial=(algo == SERIAL), bird=(algo == BIRD))


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


def gpu_solve(shape, occ, flags):
    from paper_2504_06182_amd.pipeline import SolveBuffers
    sb = SolveBuffers(shape, flags=flags).load(occ).run()
    torch.cuda.synchronize()
    return sb, sb.host()


def gpu_batch(sb, n_steps, flags=0):
    from paper_2504_06182_amd.pipeline import BatchBuffers
    bb = BatchBuffers(sb, step_cap=max(n_steps, 1)).run(flags=flags)
    torch.cuda.synchronize()
    return bb.host()


def check_one(shape, occ, tag, algo, batch_flags=(0,)):
    sb, g = gpu_solve(shape, occ, algo)
    r = oracle_solve(shape, occ, algo)
    same_solve(g, r, tag)
    if r["status"] == 0:
        check_solve(shape, occ, g)
        for f in batch_flags:
            rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=f, indexed=True)
            same_batch(gpu_batch(sb, g["n_steps"], f), rb, f"{tag} batch flags={f}")
    return r


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
    ("ragged_130x129", centred(130, 129, 91, 90), lambda x, y: (x * 3 + y * 29) % 11 < 7),
    ("paper_full_width", (32, 54, 0, 11, 32, 43), lambda x, y: (x * 5 + y * 13) % 10 < 6),
    ("one_cell", (1, 1, 0, 0, 1, 1), lambda x, y: True),
    ("line_1x9", (1, 9, 0, 3, 1, 6), lambda x, y: y in (0, 1, 8)),
    ("thin_target", centred(64, 64, 1, 40), lambda x, y: (x + 3 * y) % 4 == 0),
    ("corner_target", (64, 64, 0, 0, 20, 20), lambda x, y: (x * y) % 3 != 0),
    ("max_256", centred(256, 256, 179, 179), lambda x, y: (x * 7 + y * 11) % 10 < 6),
]


@pytest.mark.parametrize("algo", VARIANTS, ids=[NAMES[a] for a in VARIANTS])
@pytest.mark.parametrize("name,shape,fn", ADVERSARIAL, ids=[a[0] for a in ADVERSARIAL])
def test_variant_adversarial(name, shape, fn, algo):
    say("case", NAMES[algo], name, shape)
    occ = ri.pack_rows(dense(shape[0], shape[1], fn))
    check_one(shape, occ, name, algo, batch_flags=(0,) if shape[0] * shape[1] > 130 * 130 else (0, 1, 2))


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FIXTURES = ([(p, (("serial", SERIAL), ("parallel", 0))) for p in sorted(glob.glob(os.path.join(GOLDEN, "serial", "*.json")))]
            + [(p, (("bird", BIRD), ("redrec", 0))) for p in sorted(glob.glob(os.path.join(GOLDEN, "bird", "*.json")))])


@pytest.mark.parametrize("path,orders", FIXTURES, ids=[os.path.basename(f[0]) for f in FIXTURES])
def test_variant_fixtures_on_gpu(path, orders):
    """The hand-worked fixtures of both variants: groups and step counts of the variant and of
    the default red-rec, as worked out by hand."""
    g = json.load(open(path))
    shape = tuple(g["shape"])
    say("case fixture", os.path.basename(path))
    d = np.zeros((shape[1], shape[0]), np.uint8)
    for x, y in g["tokens"]:
        d[y, x] = 1
    for order, flags in orders:
        _, r = gpu_solve(shape, ri.pack_rows(d), flags)
        goff = r["group_off"]
        groups = [[list(map(int, m)) for m in r["moves"][goff[k]:goff[k + 1]]] for k in range(len(goff) - 1)]
        assert groups == g[order]["groups"] and r["n_steps"] == g[order]["n_steps"], order


@pytest.mark.parametrize("algo", VARIANTS, ids=[NAMES[a] for a in VARIANTS])
@pytest.mark.parametrize("seed", range(16))
def test_variant_random_shapes(seed, algo):
    rng = np.random.default_rng(1000 + seed)
    w, h = int(rng.integers(1, 200)), int(rng.integers(2, 200))
    sw, sh = int(rng.integers(1, w + 1)), int(rng.integers(1, h))
    x0, y0 = int(rng.integers(0, w - sw + 1)), int(rng.integers(0, h - sh + 1))
    if seed % 4 == 0:
        x0, sw = 0, w                             # full-width band
    shape = (w, h, x0, y0, x0 + sw, y0 + sh)
    p = float(rng.choice([0.5, 0.6, 0.7, 0.8]))
    say("case", NAMES[algo], "random", seed, shape, p)
    occ = ri.pack_rows(ri.bernoulli_grid(901, seed, w, h, p))
    check_one(shape, occ, f"seed {seed}", algo, batch_flags=(seed % 3,) if w * h <= 120 * 120 else ())


@pytest.mark.parametrize("algo", VARIANTS, ids=[NAMES[a] for a in VARIANTS])
@pytest.mark.parametrize("name", ["single32", "single128", "paper32"])
def test_variant_single_workloads(name, algo):
    d = ri.config_shots(name)[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    say("case", NAMES[algo], name, shape)
    check_one(shape, ri.shot_grid(d), name, algo, batch_flags=(0, 1, 2))


@pytest.mark.parametrize("algo", VARIANTS, ids=[NAMES[a] for a in VARIANTS])
def test_variant_many_instances_batch64_and_mixed(algo):
    """The variant on 1024 shots of the 64 x 64 workload and 48 uneven shots in many-instance
    launches: 24 sampled 64 x 64 shots and every uneven shot equal the oracle's same variant,
    every uneven shot equals its one-instance launch; batching of the sampled shots equals the
    oracle's."""
    from paper_2504_06182_amd.pipeline import ManyBuffers
    for name, n, sample in (("batch64", 1024, 24), ("mixed", 48, 48)):
        shots = ri.config_shots(name, n=n)
        shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
        grids = [ri.shot_grid(d) for d in shots]
        say("case", NAMES[algo], "many", name, n)
        mb = ManyBuffers(shapes, solve_flags=algo).load(grids).solve()
        torch.cuda.synchronize()
        sinf = mb.solve_infos()
        mb.plan_batches([max(int(i[3]), 1) for i in sinf]).batch(0)
        torch.cuda.synchronize()
        binf = mb.batch_infos()
        for i in np.linspace(0, n - 1, sample).astype(int):
            r = oracle_solve(shapes[i], grids[i], algo)
            g = mb.host_solve(i, sinf)
            same_solve(g, r, f"{name} {i}")
            if name == "mixed":
                _, g1 = gpu_solve(shapes[i], grids[i], algo)
                same_solve(g1, r, f"{name} single {i}")
            if r["status"] == 0 and shapes[i][0] <= 128:
                rb = oracle.batch(shapes[i], r["moves"], r["group_off"], r["n_steps"], indexed=True)
                same_batch(mb.host_batch(i, binf), rb, f"{name} batch {i}")


@pytest.mark.parametrize("algo", [0, SERIAL, BIRD], ids=["parallel", "serial", "bird"])
def test_solve_wavefronts_per_instance_do_not_change_results(algo):
    """Every size class solved with each wavefront count it can take (64: 1, 2, 4; 128: 2, 4;
    256: 4) in one-instance and many-instance launches: the same bytes."""
    from paper_2504_06182_amd.pipeline import ManyBuffers, SolveBuffers
    shots = [d for d in ri.config_shots("mixed", n=80) if d["w"] <= 128][:36]
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    for cls, waves in ((64, (1, 2, 4)), (128, (2, 4))):
        idx = [i for i, s in enumerate(shapes) if (s[0] <= 64) == (cls == 64)]
        say("case waves", NAMES.get(algo, "parallel"), cls, waves, len(idx))
        ref = None
        for w in waves:
            mb = ManyBuffers([shapes[i] for i in idx], solve_flags=algo | (w << 8)).load([grids[i] for i in idx])
            mb.solve()
            torch.cuda.synchronize()
            inf = mb.solve_infos()
            outs = [mb.host_solve(k, inf) for k in range(mb.n)]
            if ref is None:
                ref = outs
            for k in range(mb.n):
                same_solve(outs[k], ref[k], f"class {cls} waves {w} shot {k}")
            sb = SolveBuffers(shapes[idx[0]], flags=algo | (w << 8)).load(grids[idx[0]]).run()
            torch.cuda.synchronize()
            same_solve(sb.host(), ref[0], f"one-instance class {cls} waves {w}")

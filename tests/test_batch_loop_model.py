"""The lane-level CPU model of the fast batching path (tests/batch_loop_model.py) reproduces the
oracle's batches bit for bit under every constraint, and its ready set stays within the bound the
graph reports -- the logic the GPU kernels run, checked without a GPU."""
import numpy as np
import pytest

import batch_loop_model as M
import oracle
import rr_inputs as ri


def _cases():
    out = []
    for name, n in (("single32", 2), ("batch64", 2), ("mixed", 12)):
        for d in ri.config_shots(name, n=n):
            if d["w"] <= 64:
                out.append((name, d))
    out += [("bird", d) for d in ri.config_shots("batch64", n=2)]
    return out


@pytest.mark.parametrize("name,d", _cases(), ids=lambda v: v if isinstance(v, str) else f"shot{v['shot']}")
def test_model_matches_oracle(name, d):
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    r = oracle.solve(shape, ri.shot_grid(d), bird=(name == "bird"))
    assert r["status"] == 0
    g = M.graph(shape, r["moves"], r["group_off"])
    S = 3
    assert g["bound"] <= 64 * S
    for flags in (0, 1, 2):
        b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags)
        pb, ps, st = M.loop(g, S, flags)
        assert np.array_equal(pb, b["batch_off"]), (name, flags)
        assert np.array_equal(ps, b["steps"]), (name, flags)
        if flags == 0:
            assert st["repeats"] > 0 and st["inplace"] > 0


def test_model_compaction_path():
    """With few register slots the ready set fills up and the model compacts it (merge path);
    results stay the oracle's."""
    d = ri.config_shots("single32", n=1)[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    r = oracle.solve(shape, ri.shot_grid(d))
    g = M.graph(shape, r["moves"], r["group_off"])
    S = 1
    assert g["bound"] <= 64 * S
    b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=2)
    pb, ps, st = M.loop(g, S, 2)
    assert np.array_equal(pb, b["batch_off"]) and np.array_equal(ps, b["steps"])


def test_ready_set_overflow_fixture():
    """The hand-made wide release outgrows 3 register slots (192 positions) after the first
    group finishes -- the case where the loop kernel hands the instance to the general path --
    while its static bound says so too; with 4 slots the model gives the oracle's batches."""
    from crafted import wide_release
    shape, mv, goff, n_steps = wide_release()
    g = M.graph(shape, mv, goff)
    assert g["bound"] > 192
    with pytest.raises(RuntimeError, match="overflow"):
        M.loop(g, 3, 0)
    for flags in (0, 1, 2):
        b = oracle.batch(shape, mv, goff, n_steps, flags=flags)
        pb, ps, _ = M.loop(g, 4, flags)
        assert np.array_equal(pb, b["batch_off"]) and np.array_equal(ps, b["steps"]), flags


def ancestors(preds):
    """In-group ancestors of every move through the predecessor sets (moves in index order)."""
    anc = []
    for b, ps in enumerate(preds):
        s = set()
        for a in ps:
            assert a < b
            s |= anc[a] | {a}
        anc.append(s)
    return anc


def preds_of(g):
    want = [set() for _ in range(g["K"])]
    for a, ss in enumerate(g["succ"]):
        for b in ss:
            want[b].add(a)
    return want


@pytest.mark.parametrize("tile_kib", [60, 12, 3])
@pytest.mark.parametrize("bird", [False, True], ids=["redrec", "bird"])
def test_tiled_graph_equals_one_piece(tile_kib, bird):
    """The tiled graph build (row ranges in LDS, per-move predecessor sets accumulated over the
    ranges) gives the one-piece build's group bit matrix and, through its predecessor sets, the
    same in-group ancestors as the one-piece build and as the unreduced sets (the reduced sets
    may differ in which redundant member they keep, with ranges arriving in another order), with
    few or many ranges; a budget below one row falls back."""
    shots = [d for d in ri.config_shots("mixed", n=12) if d["w"] <= 96][:4] + ri.config_shots("batch64", n=1)
    most = 0
    for d in shots:
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        r = oracle.solve(shape, ri.shot_grid(d), bird=bird)
        if r["status"] != 0 or len(r["moves"]) == 0:
            continue
        g = M.graph(shape, r["moves"], r["group_off"])
        t = M.graph_tiled(shape, r["moves"], r["group_off"], tile_kib * 1024)
        if t is None:
            assert tile_kib == 3
            continue
        preds, gbits, R = t
        want = preds_of(g)
        full = preds_of(M.graph(shape, r["moves"], r["group_off"], reduce=False))
        assert ancestors(preds) == ancestors(want) == ancestors(full)
        if tile_kib == 60:
            full_t, _, _ = M.graph_tiled(shape, r["moves"], r["group_off"], tile_kib * 1024, reduce=False)
            assert full_t == full
        wantg = {}
        for h, ws in enumerate(g["gw"]):
            for x in ws:
                wantg.setdefault(x, set()).add(h)
        assert {k: v for k, v in gbits.items() if v} == wantg
        most = max(most, R)
    if tile_kib < 60:
        assert most > 1


def test_tiled_graph_long_row_fixture():
    """The long-row fixture (600 identical 40-trap horizontal moves): the tiled build's
    predecessor sets are the one-piece build's (each move waits on the one before it)."""
    from crafted import long_row
    shape, mv, goff, n_steps = long_row()
    g = M.graph(shape, mv, goff)
    preds, gbits, R = M.graph_tiled(shape, mv, goff, 60 * 1024)
    assert R > 1 and gbits == {}
    assert preds == [set()] + [{b - 1} for b in range(1, len(mv))]
    assert [len(s) for s in g["succ"]] == [1] * (len(mv) - 1) + [0]


def test_paths_meet_is_trap_intersection():
    """paths_meet (the O(1) test the graph build reduces predecessor sets with) says whether two
    H-then-V paths share a trap, checked against the traps of both paths on random moves, short
    and degenerate ones included."""
    rng = np.random.default_rng(11)

    def traps(m):
        sx, sy, dx, dy = m
        st = 1 if dx >= sx else -1
        out = {(x, sy) for x in range(sx, dx + st, st)}
        st = 1 if dy >= sy else -1
        return out | {(dx, y) for y in range(sy, dy + st, st)}

    n_meet = 0
    for _ in range(20000):
        p, q = (tuple(int(v) for v in rng.integers(0, 9, 4)) for _ in range(2))
        want = bool(traps(p) & traps(q))
        assert M.paths_meet(p, q) == want == M.paths_meet(q, p), (p, q)
        n_meet += want
    assert 2000 < n_meet < 18000


def test_reduced_sets_keep_bird_within_register_sets():
    """Bird's moves have more distinct in-group previous touchers than the 8 a set holds; after
    the reduction no member's path meets another's and at most one remains on these shots, while
    readiness (in-group ancestors) is that of the unreduced sets."""
    most_full = 0
    for d in ri.config_shots("batch64", n=3):
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        r = oracle.solve(shape, ri.shot_grid(d), bird=True)
        mv = [tuple(int(v) for v in m) for m in r["moves"]]
        red = preds_of(M.graph(shape, r["moves"], r["group_off"]))
        full = preds_of(M.graph(shape, r["moves"], r["group_off"], reduce=False))
        most_full = max(most_full, max(len(p) for p in full))
        assert max(len(p) for p in red) <= 1
        assert ancestors(red) == ancestors(full)
        for ps in red:
            assert not any(M.paths_meet(mv[a], mv[b]) for a in ps for b in ps if a < b)
    assert most_full > 8


@pytest.mark.parametrize("algo", ["redrec", "bird"])
def test_wide_graph_gives_the_oracle_batches(algo):
    """The wide path's graph build (in-group sets from path meetings, group edges from a per-trap
    last-group sweep) drives the loop model to the oracle's batches under every constraint, on
    64 x 64 shots and on uneven shots up to 96 per side; its readiness (in-group ancestors)
    equals that of the per-trap previous-toucher sets."""
    shots = ri.config_shots("batch64", n=2) + [d for d in ri.config_shots("mixed", n=12) if d["w"] <= 96][:3]
    for d in shots:
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        r = oracle.solve(shape, ri.shot_grid(d), bird=(algo == "bird"))
        if r["status"] != 0 or len(r["moves"]) == 0:
            continue
        g = M.wide_graph(shape, r["moves"], r["group_off"])
        full = preds_of(M.graph(shape, r["moves"], r["group_off"], reduce=False))
        assert ancestors([set(p) for p in g["preds"]]) == ancestors(full)
        S = 8
        assert g["bound"] <= 64 * S
        for flags in (0, 1, 2):
            b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags)
            pb, ps, _ = M.loop(g, S, flags)
            assert np.array_equal(pb, b["batch_off"]), (algo, d["shot"], flags)
            assert np.array_equal(ps, b["steps"]), (algo, d["shot"], flags)

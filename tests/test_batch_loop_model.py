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
    return out


@pytest.mark.parametrize("name,d", _cases(), ids=lambda v: v if isinstance(v, str) else f"shot{v['shot']}")
def test_model_matches_oracle(name, d):
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    r = oracle.solve(shape, ri.shot_grid(d))
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


@pytest.mark.parametrize("tile_kib", [60, 12, 3])
def test_tiled_graph_equals_one_piece(tile_kib):
    """The tiled graph build (row ranges in LDS, per-move predecessor sets accumulated over the
    ranges) gives the one-piece build's predecessor sets and group bit matrix, with few or many
    ranges; a budget below one row falls back."""
    shots = [d for d in ri.config_shots("mixed", n=12) if d["w"] <= 96][:4] + ri.config_shots("batch64", n=1)
    most = 0
    for d in shots:
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        r = oracle.solve(shape, ri.shot_grid(d))
        if r["status"] != 0 or len(r["moves"]) == 0:
            continue
        g = M.graph(shape, r["moves"], r["group_off"])
        t = M.graph_tiled(shape, r["moves"], r["group_off"], tile_kib * 1024)
        if t is None:
            assert tile_kib == 3
            continue
        preds, gbits, R = t
        want = [set() for _ in range(g["K"])]
        for a, ss in enumerate(g["succ"]):
            for b in ss:
                want[b].add(a)
        assert preds == want
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

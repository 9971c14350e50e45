"""Pins for the oracle's batching routine (Alg. 3, §IV): step-by-step replay, closed cases and
the hand-worked fixtures."""
import glob
import json
import os
import random

import numpy as np
import pytest

import oracle
from checker import check_batches
from rr_inputs import pack_rows, bernoulli_grid, config_shots, shot_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FLAG = {"line_or_col": 0, "along": 1, "none": 2}


def dense_from_tokens(w, h, tokens):
    g = np.zeros((h, w), np.uint8)
    for x, y in tokens:
        g[y, x] = 1
    return g


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.json"))))
def test_golden_batches(path):
    g = json.load(open(path))
    shape = tuple(g["shape"])
    occ = pack_rows(dense_from_tokens(shape[0], shape[1], g["tokens"]))
    r = oracle.solve(shape, occ)
    for name, expect in g["batches"].items():
        b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], status=r["status"], flags=FLAG[name])
        assert b["status"] == 0
        got = []
        off = b["batch_off"]
        for k in range(len(off) - 1):
            got.append([[s >> 30, (s >> 15) & 0x7FFF, s & 0x7FFF] for s in b["steps"][off[k]:off[k + 1]].tolist()])
        assert got == expect, name


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_random_solves_batch_replay(flags):
    rng = random.Random(51 + flags)
    for i in range(120):
        w, h = rng.randint(1, 24), rng.randint(1, 24)
        x0 = rng.randint(0, w - 1); x1 = rng.randint(x0 + 1, w)
        y0 = rng.randint(0, h - 1); y1 = rng.randint(y0 + 1, h)
        shape = (w, h, x0, y0, x1, y1)
        occ = pack_rows(bernoulli_grid(300, i, w, h, rng.choice([0.5, 0.7, 0.9])))
        r = oracle.solve(shape, occ)
        if r["status"] != 0:
            continue
        b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags)
        assert b["status"] == 0
        assert len(b["steps"]) == r["n_steps"]
        check_batches(shape, occ, r["moves"], r["final"], b["batch_off"], b["steps"], flags)


@pytest.mark.parametrize("name", ["single32", "batch64"])
def test_workload_batch_replay(name):
    for d in config_shots(name, n=2):
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        occ = shot_grid(d)
        r = oracle.solve(shape, occ)
        b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"])
        check_batches(shape, occ, r["moves"], r["final"], b["batch_off"], b["steps"], 0)


def test_single_path_takes_its_length():
    """One path of length L: every batch holds its one next step, so L batches."""
    shape = (10, 10, 0, 0, 10, 10)
    mv = np.array([[1, 2, 8, 9]], np.uint16)
    b = oracle.batch(shape, mv, [0, 1], 14)
    assert len(b["batch_off"]) - 1 == 14
    assert np.all(np.diff(b["batch_off"]) == 1)


def test_parallel_column_paths_share_batches():
    """k independent paths in one column moving the same way, with gaps: each batch advances
    all of them, so the batch count equals the common length."""
    shape = (6, 20, 0, 0, 6, 20)
    mv = np.array([[2, 0, 2, 3], [2, 6, 2, 9], [2, 12, 2, 15]], np.uint16)
    b = oracle.batch(shape, mv, [0, 1, 2, 3], 9)
    assert len(b["batch_off"]) - 1 == 3
    assert np.all(np.diff(b["batch_off"]) == 3)


def test_overlapping_paths_in_one_group_serialise():
    """Two paths of one group sharing traps: the later waits until the earlier has finished."""
    shape = (10, 1, 0, 0, 10, 1)
    mv = np.array([[5, 0, 8, 0], [2, 0, 6, 0]], np.uint16)
    b = oracle.batch(shape, mv, [0, 2], 7)
    assert len(b["batch_off"]) - 1 == 7


def test_group_precedence_blocks_a_later_group():
    """Paths of different groups that share a trap: the later group waits for the whole earlier
    group, even for its moves far away (§IV: later column solves wait for earlier ones)."""
    shape = (10, 10, 0, 0, 10, 10)
    # group 0: a long path in row 0 and a short one leaving (1,5); group 1 crosses (1,5) only
    mv = np.array([[0, 0, 9, 0], [1, 5, 2, 5], [1, 7, 1, 4]], np.uint16)
    b = oracle.batch(shape, mv, [0, 2, 3], 9 + 1 + 3, flags=2)
    # without constraints group 0 runs in 9 batches, then group 1 needs 3 more
    assert len(b["batch_off"]) - 1 == 12


def test_invalid_input_rejected():
    shape = (4, 4, 0, 0, 4, 4)
    assert oracle.batch(shape, np.array([[1, 1, 1, 1]], np.uint16), [0, 1], 0)["status"] == -1
    assert oracle.batch(shape, np.array([[1, 1, 9, 1]], np.uint16), [0, 1], 8)["status"] == -1
    assert oracle.batch(shape, np.array([[1, 1, 2, 1]], np.uint16), [0, 0], 1)["status"] == -1


def test_capacity_reporting():
    d = config_shots("single32")[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    r = oracle.solve(shape, shot_grid(d))
    full = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"])
    small = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], batch_cap=3)
    assert small["status"] == -2
    assert small["need_batches"] == len(full["batch_off"]) - 1
    assert small["need_steps"] == r["n_steps"]


# ---- the indexed form (reduced dependency graph, bucketed ready set) against the literal form

def _both(shape, r, flags):
    a = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], status=r["status"], flags=flags)
    b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], status=r["status"], flags=flags, indexed=True)
    return a, b


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.json"))))
def test_indexed_equals_literal_on_fixtures(path):
    g = json.load(open(path))
    shape = tuple(g["shape"])
    occ = pack_rows(dense_from_tokens(shape[0], shape[1], g["tokens"]))
    r = oracle.solve(shape, occ)
    for flags in (0, 1, 2):
        a, b = _both(shape, r, flags)
        assert a["status"] == b["status"] == 0
        assert np.array_equal(a["batch_off"], b["batch_off"]) and np.array_equal(a["steps"], b["steps"])


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_indexed_equals_literal_random(flags):
    """Random grids up to 64 x 64 (full-width and side-column targets), every constraint:
    batch ends and steps identical, byte for byte."""
    rng = random.Random(77 + flags)
    n = 0
    for i in range(300):
        w, h = rng.randint(1, 64), rng.randint(1, 64)
        if rng.random() < 0.3:
            x0, x1 = 0, w
        else:
            sw = rng.randint(1, w); x0 = rng.randint(0, w - sw); x1 = x0 + sw
        sh = rng.randint(1, h); y0 = rng.randint(0, h - sh)
        shape = (w, h, x0, y0, x1, y0 + sh)
        occ = pack_rows(bernoulli_grid(500, i, w, h, rng.uniform(0.45, 0.95)))
        r = oracle.solve(shape, occ)
        if r["status"] != 0:
            continue
        a, b = _both(shape, r, flags)
        assert a["status"] == b["status"] == 0, (i, shape)
        assert np.array_equal(a["batch_off"], b["batch_off"]), (i, shape)
        assert np.array_equal(a["steps"], b["steps"]), (i, shape)
        n += 1
    assert n >= 200


@pytest.mark.parametrize("name", ["single32", "batch64", "single128", "mixed"])
def test_indexed_equals_literal_workloads(name):
    for d in config_shots(name, n=2):
        if d["w"] > 128:
            continue
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        r = oracle.solve(shape, shot_grid(d))
        for flags in (0, 1, 2):
            a, b = _both(shape, r, flags)
            assert np.array_equal(a["batch_off"], b["batch_off"]) and np.array_equal(a["steps"], b["steps"])


def test_indexed_capacity_and_invalid_like_literal():
    d = config_shots("single32")[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    r = oracle.solve(shape, shot_grid(d))
    full = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], indexed=True)
    for kw in (dict(batch_cap=3), dict(step_cap=10)):
        a = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], **kw)
        b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], indexed=True, **kw)
        assert a["status"] == b["status"] == -2
        assert (a["need_batches"], a["need_steps"]) == (b["need_batches"], b["need_steps"])
    assert full["status"] == 0
    bad = np.array(r["moves"]).copy()
    bad[0, 2] = bad[0, 0]; bad[0, 3] = bad[0, 1]           # zero-length move
    assert oracle.batch(shape, bad, r["group_off"], r["n_steps"], indexed=True)["status"] == -1

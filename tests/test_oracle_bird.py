"""Pins for the oracle's bird algorithm (§III.E, Alg. 2).

* Hand-worked fixtures (``tests/golden/bird/``): the paper's own example of red-rec's drawback
  (a column missing two tokens between two donors, each with one token next to the target and
  one at the far end of the reservoir: red-rec takes both from one donor, bird one nearby token
  from each), and a run boundary inside one virtual row (two tokens at the same distance from
  the column, the left one taken).
* Each bird column's group moves the fewest unit steps any choice of tokens could: its step
  count equals a min-cost assignment (scipy's Hungarian method on Manhattan distances) of the
  tokens it may draw on -- its own and every other column's reservoir tokens -- to its target
  traps, taken on the grid as it stands when the column is solved.  The virtual-row mapping
  and the generalized exact 1D are checked through that, independently.
* Every bird solve replays legally (source occupied, path free -- the paper's claim that no
  chosen token meets an obstruction --, one token per trap, Manhattan length, target covered
  iff solved) and refuses exactly what red-rec refuses; exhaustively on 3 x 3 (every loading,
  every target) and on 4 x 4 (every loading, two targets).
* Columns of non-negative surplus are solved as in red-rec: bird's groups start with red-rec's
  row pre-pass and non-negative column groups.
"""
import glob
import json
import os
import random

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
from checker import check_solve
from rr_inputs import config_shots, pack_rows, shot_grid
from test_oracle_pairing import counts_after_row_pass, random_instance

BIRD = os.path.join(os.path.dirname(__file__), "golden", "bird")


def dense_from_tokens(w, h, tokens):
    g = np.zeros((h, w), np.uint8)
    for x, y in tokens:
        g[y, x] = 1
    return g


def groups_of(r):
    goff = r["group_off"]
    return [[list(map(int, m)) for m in r["moves"][goff[k]:goff[k + 1]]] for k in range(len(goff) - 1)]


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(BIRD, "*.json"))))
def test_bird_fixtures(path):
    g = json.load(open(path))
    shape = tuple(g["shape"])
    occ = pack_rows(dense_from_tokens(shape[0], shape[1], g["tokens"]))
    for algo in ("redrec", "bird"):
        r = oracle.solve(shape, occ, bird=(algo == "bird"))
        e = g[algo]
        assert r["rc"] == 0 and r["status"] == g["status"], algo
        assert groups_of(r) == e["groups"], algo
        assert r["n_steps"] == e["n_steps"], algo
        assert np.array_equal(r["final"], pack_rows(dense_from_tokens(shape[0], shape[1], e["final"]))), algo
        check_solve(shape, occ, r)


def bird_groups_optimal(shape, dense, r):
    """Replay group by group; each of the last n_neg groups (one per column of negative surplus,
    ascending) must cost exactly the min-cost assignment of its available tokens."""
    w, h, x0, y0, x1, y1 = shape
    sh = y1 - y0
    cols = counts_after_row_pass(shape, dense)
    neg = [x for x in range(x0, x1) if len(cols[x]) < sh]
    groups = groups_of(r)
    assert len(groups) >= len(neg)
    grid = dense.astype(np.uint8).copy()
    first_bird = len(groups) - len(neg)
    for gi, grp in enumerate(groups):
        if gi >= first_bird:
            j = neg[gi - first_bird]
            assert all(m[2] == j and y0 <= m[3] < y1 for m in grp)
            toks = [(x, y) for y in range(h) for x in range(w)
                    if grid[y, x] and (x == j or not (y0 <= y < y1))]
            cost = np.array([[abs(x - j) + abs(y - t) for t in range(y0, y1)] for x, y in toks])
            ri, ci = linear_sum_assignment(cost)
            steps = sum(abs(m[2] - m[0]) + abs(m[3] - m[1]) for m in grp)
            assert steps == int(cost[ri, ci].sum()), (gi, j)
        for sx, sy, dx, dy in grp:
            grid[sy, sx] = 0
            grid[dy, dx] = 1
    return len(neg)


def test_bird_random_instances():
    """1200 random instances (full-width and side-column targets): legal replay, same status
    as red-rec, every bird column's group at the least possible step count."""
    rng = random.Random(2505)
    n_cols = 0
    fewer = 0
    for i in range(1200):
        shape, dense = random_instance(rng, i)
        occ = pack_rows(dense)
        rb = oracle.solve(shape, occ, bird=True)
        rp = oracle.solve(shape, occ)
        assert rb["rc"] == 0 and rb["status"] == rp["status"], (i, shape)
        check_solve(shape, occ, rb)
        if rb["status"] == 0:
            n_cols += bird_groups_optimal(shape, dense, rb)
            fewer += rb["n_steps"] < rp["n_steps"]
    assert n_cols >= 1000 and fewer >= 100


@pytest.mark.parametrize("name", ["single32", "single128", "batch64", "mixed", "paper32"])
def test_bird_workload_instances(name):
    for d in config_shots(name, n=4):
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        occ = shot_grid(d)
        rb = oracle.solve(shape, occ, bird=True)
        rp = oracle.solve(shape, occ)
        assert rb["status"] == rp["status"]
        check_solve(shape, occ, rb)
        if rb["status"] == 0 and shape[0] <= 64:
            dense = np.unpackbits(occ.view(np.uint8), bitorder="little").reshape(shape[1], -1)[:, :shape[0]]
            bird_groups_optimal(shape, dense, rb)


def test_bird_starts_with_redrec_stages():
    """The row pre-pass and the non-negative columns are solved as in red-rec: bird's first
    groups are red-rec's, up to the first group red-rec emits for a receiver."""
    rng = random.Random(9)
    for i in range(300):
        shape, dense = random_instance(rng, i)
        occ = pack_rows(dense)
        rb, rp = oracle.solve(shape, occ, bird=True), oracle.solve(shape, occ, trace=True)
        if rp["status"] != 0:
            continue
        w, h, x0, y0, x1, y1 = shape
        cols = counts_after_row_pass(shape, dense)
        n_neg = sum(1 for x in range(x0, x1) if len(cols[x]) < y1 - y0)
        n_rec_groups = sum(1 for e in rp["events"] if e[2] != 3)
        gb, gp = groups_of(rb), groups_of(rp)
        head = len(gp) - n_rec_groups
        assert gb[:head] == gp[:head] and len(gb) == head + n_neg, (i, shape)


def exhaustive(w, h, targets):
    for x0, y0, x1, y1 in targets:
        shape = (w, h, x0, y0, x1, y1)
        for bits in range(1 << (w * h)):
            dense = np.array([(bits >> k) & 1 for k in range(w * h)], np.uint8).reshape(h, w)
            occ = pack_rows(dense)
            rb = oracle.solve(shape, occ, bird=True)
            rp = oracle.solve(shape, occ)
            assert rb["status"] == rp["status"], (shape, bits)
            check_solve(shape, occ, rb)


def test_bird_exhaustive_3x3():
    exhaustive(3, 3, [(x0, y0, x1, y1) for x0 in range(3) for x1 in range(x0 + 1, 4)
                      for y0 in range(3) for y1 in range(y0 + 1, 4)])


def test_bird_exhaustive_4x4():
    exhaustive(4, 4, [(0, 1, 4, 3), (1, 1, 3, 3)])

"""Pins for the oracle's serial order of Alg. 1 (§III.C as written: only the columns of zero
surplus are solved at the outset, a donor hands over tokens from its reservoir -- nearest the
band first -- and is solved when it settles or, if it never does, after the loop).

* Hand-worked fixtures (``tests/golden/serial/``) give both orders' events, groups and step
  counts; in the first the donor's innermost token goes to the receiver in the serial order
  and its excess token in the parallel one.
* The naive loop of ``test_oracle_pairing`` (written from the text, O(W^3)), in its serial mode,
  agrees with the oracle event by event, split included, and no choice of donor tokens gives
  the receiver a smaller cost than the split taken.
* Every serial solve replays legally (source occupied, path free, one token per trap, Manhattan
  length, target covered iff solved) and refuses exactly the instances the parallel order
  refuses; the two orders pair the same columns in the same cases with the same counts (the
  loop reads only surpluses); in the column stage no token moves twice (§III.C).
* With no receiver, the serial groups are the parallel ones, zero-surplus columns first.
"""
import glob
import json
import os
import random

import numpy as np
import pytest

import oracle
from checker import check_solve
from rr_inputs import bernoulli_grid, config_shots, pack_rows, shot_grid
from test_oracle_pairing import naive_pair_loop, random_instance

SERIAL = os.path.join(os.path.dirname(__file__), "golden", "serial")


def dense_from_tokens(w, h, tokens):
    g = np.zeros((h, w), np.uint8)
    for x, y in tokens:
        g[y, x] = 1
    return g


def groups_of(r):
    goff = r["group_off"]
    return [[list(map(int, m)) for m in r["moves"][goff[k]:goff[k + 1]]] for k in range(len(goff) - 1)]


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(SERIAL, "*.json"))))
def test_serial_fixtures_both_orders(path):
    g = json.load(open(path))
    shape = tuple(g["shape"])
    occ = pack_rows(dense_from_tokens(shape[0], shape[1], g["tokens"]))
    fin = pack_rows(dense_from_tokens(shape[0], shape[1], g["final"]))
    for order in ("parallel", "serial"):
        r = oracle.solve(shape, occ, trace=True, serial=(order == "serial"))
        e = g[order]
        assert r["rc"] == 0 and r["status"] == g["status"], order
        assert [list(v) for v in r["events"]] == e["events"], order
        assert groups_of(r) == e["groups"], order
        assert r["n_steps"] == e["n_steps"], order
        assert np.array_equal(r["final"], fin), order
        check_solve(shape, occ, r)
        dense = dense_from_tokens(shape[0], shape[1], g["tokens"])
        ev, splits = naive_pair_loop(shape, dense, split_check=True, serial=(order == "serial"))
        assert [list(v) for v in ev] == e["events"], order
        assert all(a == b for a, b in splits), order


def column_stage_moves(shape, r):
    """Moves after the row pre-pass's groups (one group per target row with moves, first)."""
    w, h, x0, y0, x1, y1 = shape
    goff, mv = r["group_off"], r["moves"]
    k = 0
    if x0 > 0 or x1 < w:
        while k < len(goff) - 1 and all(m[1] == m[3] for m in mv[goff[k]:goff[k + 1]]):
            k += 1
    return mv[goff[k]:]


def moves_at_most_once(moves):
    """No move starts where an earlier move of the list ended (each token moves once)."""
    ends = set()
    for sx, sy, dx, dy in moves.tolist():
        if (sx, sy) in ends:
            return False
        ends.add((dx, dy))
    return True


def test_serial_random_instances():
    """1500 random instances (full-width and side-column targets): the serial solve replays
    legally, refuses what the parallel order refuses, pairs the same columns in the same cases
    with the same counts, agrees with the naive serial loop event by event (split included,
    split optimal over every choice of donor tokens), and moves no token twice in the column
    stage."""
    rng = random.Random(2504)
    n_diff = n_events = 0
    for i in range(1500):
        shape, dense = random_instance(rng, i)
        occ = pack_rows(dense)
        rs = oracle.solve(shape, occ, trace=True, serial=True)
        rp = oracle.solve(shape, occ, trace=True)
        assert rs["rc"] == 0 and rs["status"] == rp["status"], (i, shape)
        check_solve(shape, occ, rs)
        if rs["status"] != 0:
            continue
        assert [(e[0], e[1], e[2], e[4]) for e in rs["events"]] == [(e[0], e[1], e[2], e[4]) for e in rp["events"]]
        ev, splits = naive_pair_loop(shape, dense, split_check=True, serial=True)
        assert [tuple(e) for e in rs["events"]] == ev, (i, shape)
        assert all(a == b for a, b in splits), (i, shape, splits)
        assert moves_at_most_once(column_stage_moves(shape, rs)), (i, shape)
        assert moves_at_most_once(column_stage_moves(shape, rp)), (i, shape)
        n_events += len(ev) > 0
        n_diff += not (np.array_equal(rs["moves"], rp["moves"]) and np.array_equal(rs["group_off"], rp["group_off"]))
    assert n_events >= 600 and n_diff >= 300


def test_serial_equals_parallel_groups_without_receivers():
    """Full-width bands whose every column has at least sh tokens: no pair is formed, and the
    serial order emits the parallel order's groups, zero-surplus columns first."""
    rng = random.Random(5)
    for i in range(200):
        w, h = rng.randint(1, 12), rng.randint(3, 14)
        sh = rng.randint(1, h - 2)
        y0 = (h - sh) // 2
        shape = (w, h, 0, y0, w, y0 + sh)
        dense = bernoulli_grid(302, i, w, h, 0.5)
        for x in range(w):                      # top up every column to at least sh tokens
            ys = [y for y in range(h) if not dense[y, x]]
            need = sh - int(dense[:, x].sum())
            for y in ys[:max(0, need)]:
                dense[y, x] = 1
        occ = pack_rows(dense)
        rs, rp = oracle.solve(shape, occ, serial=True, trace=True), oracle.solve(shape, occ, trace=True)
        assert rs["status"] == rp["status"] == 0 and rs["events"] == rp["events"] == []
        gp = groups_of(rp)
        col = [g[0][0] for g in gp]
        zero = [x for x in range(w) if int(dense[:, x].sum()) == sh]
        expect = [g for g, x in zip(gp, col) if x in zero] + [g for g, x in zip(gp, col) if x not in zero]
        assert groups_of(rs) == expect


@pytest.mark.parametrize("name", ["single32", "single128", "batch64", "mixed", "paper32"])
def test_serial_workload_instances(name):
    """Workload shots: legal replay, same status and pairs as the parallel order, naive loop
    agreement."""
    for d in config_shots(name, n=6):
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        occ = shot_grid(d)
        rs = oracle.solve(shape, occ, trace=True, serial=True)
        rp = oracle.solve(shape, occ, trace=True)
        assert rs["status"] == rp["status"]
        check_solve(shape, occ, rs)
        if rs["status"] == 0:
            dense = np.unpackbits(occ.view(np.uint8), bitorder="little").reshape(shape[1], -1)[:, :shape[0]]
            ev, _ = naive_pair_loop(shape, dense, serial=True)
            assert [tuple(e) for e in rs["events"]] == ev

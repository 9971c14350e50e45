"""Pins for the oracle's donor/receiver loop (Alg. 1 main loop, pairing rule of §III.C, in the
order of the parallel form §III.D).

The reference below is written from the paper's text alone and shares nothing with
``oracle/rr_oracle.c``: it derives each column's surplus from the loading (after the row
pre-pass, whose only effect on the counts is which central traps of a target row end up
filled), then runs the loop by scanning every (donor, receiver) pair of the grid, O(W^3) per
instance:

* candidates are pairs of a positive and a negative column with only settled (zero) columns
  strictly between them;
* the best pair maximises, in this order: the tokens that can be exchanged
  (min(surplus, deficit)), then the fewest columns in between, then the receiver closest to
  saturation (smallest deficit); further ties take the smaller receiver index, then the
  smaller donor index (a reading: the paper stops after the third criterion);
* case 1: donor surplus > deficit (the receiver settles), case 2: equal (both settle), case 3:
  smaller (the donor's tokens are marked for the receiver and the donor settles).

For the split of cases 1-2 it also keeps each column's token pools and checks, by trying every
subset of the donor's pool, that the split the oracle takes has the least receiver cost that
any choice of donor tokens could have (so restricting to nearest-first splits loses nothing),
and that among the nearest-first splits of that cost it is the one with most tokens from
below (the tie reading).

Hand-worked fixtures (``tests/golden/pairing/``) make each criterion decide at least once
against the next one; ``tests/golden/g6_split_tie.json`` pins the split tie.
"""
import glob
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
from rr_inputs import bernoulli_grid, pack_rows

PAIRING = os.path.join(os.path.dirname(__file__), "golden", "pairing")


def counts_after_row_pass(shape, dense):
    """Eligible rows per column after the row pre-pass.

    A target row with at least sw tokens ends with every central trap filled (its extra tokens
    are parked in side columns and never counted); a row with fewer tokens ends with a run of
    that many traps starting at x0 + (sw - a) // 2.  Reservoir rows are untouched.  Side
    columns count only their reservoir-row tokens.  Returns a list of sorted row lists."""
    w, h, x0, y0, x1, y1 = shape
    sw = x1 - x0
    side = x0 > 0 or x1 < w
    grid = np.array(dense, dtype=np.uint8).copy()
    if side:
        for y in range(y0, y1):
            a = int(grid[y].sum())
            row = np.zeros(w, np.uint8)
            if a >= sw:
                row[x0:x1] = 1
            else:
                c = x0 + (sw - a) // 2
                row[c:c + a] = 1
            grid[y] = row           # parked side tokens dropped: they never count
    cols = []
    for x in range(w):
        central = x0 <= x < x1
        cols.append([y for y in range(h) if grid[y, x] and (central or y < y0 or y >= y1)])
    return cols


def best_window(rows, b, t):
    """Start of the cheapest run of t consecutive sorted rows matched in order onto b..b+t-1
    (every start tried; equal cost -> smallest start)."""
    best = None
    for s in range(len(rows) - t + 1):
        c = sum(abs(rows[s + k] - (b + k)) for k in range(t))
        if best is None or c < best[0]:
            best = (c, s)
    return best[1]


def line_cost(rows, y0):
    """Summed distance of the sorted rows matched in order onto y0, y0+1, ..."""
    return sum(abs(r - (y0 + m)) for m, r in enumerate(sorted(rows)))


def naive_pair_loop(shape, dense, split_check=False, subset_limit=12, serial=False):
    """Events (donor, receiver, case, count) of the loop, or None when the surpluses sum below
    zero (the instance is refused before any move).

    ``serial``: Alg. 1 in its serial order -- a central donor is not solved at the outset; its
    pool is its reservoir tokens (nearest the band first), it hands tokens over from that pool,
    and it is solved when it settles (case 2 after the receiver, case 3 before its tokens are
    marked: an exact-1D window over the tokens it still holds, whose unmatched ones are then
    marked)."""
    w, h, x0, y0, x1, y1 = shape
    sh = y1 - y0
    cols = counts_after_row_pass(shape, dense)
    sig = [len(c) - (sh if x0 <= x < x1 else 0) for x, c in enumerate(cols)]
    if sum(sig) < 0:
        return None, []
    below, above, own, marked, band = {}, {}, {}, {}, {}
    for x in range(w):
        if sig[x] >= 0:
            r = cols[x]
            if serial and x0 <= x < x1 and sig[x] > 0:
                below[x] = [y for y in reversed(r) if y < y0]
                above[x] = [y for y in r if y >= y1]
                band[x] = [y for y in r if y0 <= y < y1]
            elif x0 <= x < x1:
                s = best_window(r, y0, sh)
                below[x] = list(reversed(r[:s]))          # nearest the band first
                above[x] = r[s + sh:]
            else:
                below[x] = [y for y in reversed(r) if y < y0]
                above[x] = [y for y in r if y >= y1]
        else:
            own[x] = list(cols[x])
            marked[x] = []
    sp = list(sig)
    events, splits = [], []
    while any(v < 0 for v in sp):
        best = None
        for i in range(w):
            for j in range(w):
                if sp[i] <= 0 or sp[j] >= 0:
                    continue
                lo, hi = min(i, j), max(i, j)
                if any(sp[k] != 0 for k in range(lo + 1, hi)):
                    continue
                key = (min(sp[i], -sp[j]), -(hi - lo), sp[j], -j, -i)
                if best is None or key > best[0]:
                    best = (key, i, j)
        assert best is not None, "a negative column with no candidate donor"
        _, i, j = best
        si, dj = sp[i], -sp[j]
        if si > dj or si == dj:
            kase = 1 if si > dj else 2
            cnt = dj
            fixed = own[j] + marked[j]
            pool_b, pool_u = below[i], above[i]
            lo_k, hi_k = max(0, dj - len(pool_u)), min(dj, len(pool_b))
            costs = {k: line_cost(fixed + pool_b[:k] + pool_u[:dj - k], y0) for k in range(lo_k, hi_k + 1)}
            cmin = min(costs.values())
            k_sel = max(k for k, c in costs.items() if c == cmin)
            if split_check and len(pool_b) + len(pool_u) <= subset_limit:
                pool = pool_b + pool_u
                every = min(line_cost(fixed + list(sub), y0) for sub in itertools.combinations(pool, dj))
                splits.append((cmin, every))
            below[i], above[i] = pool_b[k_sel:], pool_u[dj - k_sel:]
            sp[i] -= dj
            sp[j] = 0
            events.append((i, j, kase, k_sel, cnt))
        else:
            if i in band:                                 # serial order: solve the donor first
                r = sorted(below[i] + band.pop(i) + above[i])
                s = best_window(r, y0, sh)
                below[i], above[i] = list(reversed(r[:s])), r[s + sh:]
            marked[j] += below[i] + above[i]
            below[i], above[i] = [], []
            sp[j] += si
            sp[i] = 0
            events.append((i, j, 3, -1, si))
    return events, splits


def dense_from_columns(w, h, columns):
    g = np.zeros((h, w), np.uint8)
    for x, rows in enumerate(columns):
        for y in rows:
            g[y, x] = 1
    return g


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(PAIRING, "*.json"))))
def test_pairing_fixtures(path):
    """Each hand-worked fixture: the oracle's events and the naive loop's both equal the
    events derived by hand."""
    g = json.load(open(path))
    shape = tuple(g["shape"])
    assert len(g["columns"]) == shape[0]
    dense = dense_from_columns(shape[0], shape[1], g["columns"])
    r = oracle.solve(shape, pack_rows(dense), trace=True)
    assert r["rc"] == 0 and r["status"] == g["status"]
    assert [[e[0], e[1], e[2], e[4]] for e in r["events"]] == g["events"], g["pins"]
    ev, _ = naive_pair_loop(shape, dense)
    assert [[e[0], e[1], e[2], e[4]] for e in ev] == g["events"]


def test_split_tie_fixture_matches_naive():
    g = json.load(open(os.path.join(os.path.dirname(PAIRING), "g6_split_tie.json")))
    shape = tuple(g["shape"])
    dense = np.zeros((shape[1], shape[0]), np.uint8)
    for x, y in g["tokens"]:
        dense[y, x] = 1
    ev, splits = naive_pair_loop(shape, dense, split_check=True)
    assert [list(e) for e in ev] == g["events"]
    assert splits and all(a == b for a, b in splits)


def random_instance(rng, i):
    w = rng.randint(1, 26)
    h = rng.randint(2, 26)
    kind = rng.random()
    if kind < 0.35:                                   # full-width band, the paper's geometry
        x0, x1 = 0, w
    else:                                             # side columns on one or both sides
        sw = rng.randint(1, w)
        x0 = rng.randint(0, w - sw)
        x1 = x0 + sw
    sh = rng.randint(1, h - 1)
    y0 = rng.randint(0, h - sh) if rng.random() < 0.5 else (h - sh) // 2
    shape = (w, h, x0, y0, x1, y0 + sh)
    area = (x1 - x0) * sh
    p = min(0.95, max(0.2, area / (w * h) + rng.uniform(-0.05, 0.25)))
    return shape, bernoulli_grid(300, i, w, h, p)


def test_pair_loop_event_by_event_random():
    """1500 random instances (full-width and side-column targets, surpluses taken after the
    row pre-pass): the oracle's events equal the naive loop's one by one, donor, receiver,
    case, split and count, and refused instances are exactly those whose surpluses sum below
    zero."""
    rng = random.Random(2504)
    n_multi = n_case = 0
    seen_cases = set()
    for i in range(1500):
        shape, dense = random_instance(rng, i)
        r = oracle.solve(shape, pack_rows(dense), trace=True)
        assert r["rc"] == 0
        ev, splits = naive_pair_loop(shape, dense, split_check=True)
        if ev is None:
            assert r["status"] == 1, (i, shape)
            continue
        assert r["status"] == 0, (i, shape)
        assert [tuple(e) for e in r["events"]] == ev, (i, shape)
        assert all(a == b for a, b in splits), (i, shape, splits)
        n_multi += len(ev) >= 2
        n_case += len(ev) > 0
        seen_cases.update(e[2] for e in ev)
    assert n_multi >= 300 and n_case >= 600
    assert seen_cases == {1, 2, 3}


def test_pair_loop_on_workload_shapes():
    """The same comparison on shots of the 64 x 64 and uneven workloads' geometries (centred
    squares with side columns), where loops run for tens of iterations."""
    rng = random.Random(7)
    for i in range(40):
        n = rng.choice([32, 48, 64])
        s = (7 * n) // 10
        x0 = (n - s) // 2
        shape = (n, n, x0, x0, x0 + s, x0 + s)
        dense = bernoulli_grid(301, i, n, n, rng.uniform(0.5, 0.65))
        r = oracle.solve(shape, pack_rows(dense), trace=True)
        ev, _ = naive_pair_loop(shape, dense)
        if ev is None:
            assert r["status"] == 1
            continue
        assert [tuple(e) for e in r["events"]] == ev

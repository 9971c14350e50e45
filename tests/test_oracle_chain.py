"""Pins for the oracle's chain form of exact 1D (``oracle.solve_chain``): on chains of up to 256
traps it equals the oracle's red-rec on the same 1 x N grid (where the target row is solved by
the row pre-pass, a separate path of the oracle); on short chains its move count and step count
are those of a brute-force min-cost assignment; the paper's chain geometry (centre-compact
target of N/2 traps, 0.6 N atoms) is feasible and its replay lands on the target."""
import itertools
import random

import numpy as np

import oracle
from rr_inputs import config_shots, fixed_count_grid, pack_rows, shot_grid


def test_chain_equals_grid_solve_on_one_row():
    rng = random.Random(11)
    for i in range(400):
        n = rng.randint(1, 256)
        t = rng.randint(1, n)
        b = rng.randint(0, n - t)
        count = rng.randint(0, n)
        dense = fixed_count_grid(40, i, n, 1, count)
        occ = pack_rows(dense)
        c = oracle.solve_chain(n, occ[0], b, t)
        g = oracle.solve((n, 1, b, 0, b + t, 1), occ)
        assert c["status"] == g["status"], (n, b, t, count)
        assert np.array_equal(c["final"], g["final"])
        if g["status"] == 0:
            assert np.array_equal(c["moves"], g["moves"]) and np.array_equal(c["group_off"], g["group_off"])
            assert c["n_steps"] == g["n_steps"]


def test_chain_cost_is_min_assignment_brute_force():
    rng = random.Random(12)
    for i in range(300):
        n = rng.randint(1, 10)
        t = rng.randint(1, n)
        b = rng.randint(0, n - t)
        dense = fixed_count_grid(41, i, n, 1, rng.randint(t, n))
        p = np.nonzero(dense[0])[0]
        best = min(sum(abs(int(s) - (b + k)) for k, s in enumerate(sorted(sub)))
                   for sub in itertools.combinations(p, t))
        c = oracle.solve_chain(n, pack_rows(dense)[0], b, t)
        assert c["n_steps"] == best


def test_chain_workload_geometry_replays():
    for name in ("chain1024",):
        for d in config_shots(name, n=20):
            occ = shot_grid(d)
            assert int(np.unpackbits(occ.view(np.uint8)).sum()) == d["count"]
            c = oracle.solve_chain(d["w"], occ[0], d["x0"], d["x1"] - d["x0"])
            assert c["status"] == 0
            cells = set(np.nonzero(np.unpackbits(occ.view(np.uint8), bitorder="little")[:d["w"]])[0].tolist())
            for sx, _, dx, _ in c["moves"].tolist():          # emission order is collision free
                step = 1 if dx > sx else -1
                assert sx in cells
                for x in range(sx + step, dx + step, step):
                    assert x not in cells
                cells.remove(sx)
                cells.add(dx)
            assert set(range(d["x0"], d["x1"])) <= cells

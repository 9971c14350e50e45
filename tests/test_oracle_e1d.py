"""Pins for the oracle's exact-1D routine (§III.A) against brute force and closed forms."""
import itertools
import random

import pytest

import oracle


def brute_force(p, b, t):
    """All injective maps from the t targets to the sources; returns (min cost, optimal maps)."""
    best, maps = None, []
    for choice in itertools.permutations(range(len(p)), t):
        c = sum(abs(p[choice[k]] - (b + k)) for k in range(t))
        if best is None or c < best:
            best, maps = c, [choice]
        elif c == best:
            maps.append(choice)
    return best, maps


def window_cost(p, w, b, t):
    return sum(abs(p[w + k] - (b + k)) for k in range(t))


def test_window_cost_is_the_minimum_assignment_cost():
    rng = random.Random(11)
    for _ in range(400):
        n = rng.randint(1, 12)
        a = rng.randint(1, min(n, 7))
        t = rng.randint(0, a)
        p = sorted(rng.sample(range(n), a))
        b = rng.randint(0, n - t) if t <= n else 0
        w = oracle.e1d_window(p, b, t)
        best, maps = brute_force(p, b, t)
        assert window_cost(p, w, b, t) == best
        # the chosen run is an order-preserving optimum ...
        assert tuple(range(w, w + t)) in maps
        # ... and, among optimal order-preserving runs, the leftmost (tie reading)
        runs = [m[0] for m in maps if t > 0 and list(m) == list(range(m[0], m[0] + t))]
        if runs:
            assert w == min(runs)


def test_every_source_inside_the_target_is_matched():
    rng = random.Random(12)
    for _ in range(300):
        n = rng.randint(2, 30)
        a = rng.randint(1, n)
        t = rng.randint(1, a)
        p = sorted(rng.sample(range(n), a))
        b = rng.randint(0, n - t)
        w = oracle.e1d_window(p, b, t)
        matched = set(p[w:w + t])
        for q in p:
            if b <= q < b + t:
                assert q in matched
        # unmatched sources lie on no matched path
        for q in set(p) - matched:
            for k in range(t):
                lo, hi = sorted((p[w + k], b + k))
                assert not (lo <= q <= hi)


def test_equal_counts_is_the_sorted_matching():
    """|S| = |T|: the only order-preserving matching pairs sorted sources with sorted targets."""
    rng = random.Random(13)
    for _ in range(100):
        n = rng.randint(1, 40)
        t = rng.randint(1, n)
        p = sorted(rng.sample(range(n), t))
        assert oracle.e1d_window(p, rng.randint(0, n - t), t) == 0


@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_quadratic_worst_case(n):
    """§III.A complexity: n tokens on the first n of 2n traps, target the last n: n^2 steps."""
    mv = oracle.e1d_moves(list(range(n)), n, n)
    assert len(mv) == n
    assert sum(abs(s - d) for s, d in mv) == n * n


def test_emission_order_is_collision_free_on_a_line():
    """Right-oriented paths first (largest target first), then left-oriented (smallest target
    first): replaying the moves in order never crosses an occupied trap (§III.A)."""
    rng = random.Random(14)
    for _ in range(300):
        n = rng.randint(2, 40)
        a = rng.randint(1, n)
        t = rng.randint(1, a)
        p = sorted(rng.sample(range(n), a))
        b = rng.randint(0, n - t)
        occ = set(p)
        mv = oracle.e1d_moves(p, b, t)
        seen_left = False
        last_right, last_left = None, None
        for s, d in mv:
            assert s in occ
            step = 1 if d > s else -1
            for x in range(s + step, d + step, step):
                assert x not in occ
            occ.remove(s)
            occ.add(d)
            if d > s:
                assert not seen_left
                assert last_right is None or d < last_right
                last_right = d
            else:
                seen_left = True
                assert last_left is None or d > last_left
                last_left = d
        assert set(range(b, b + t)) <= occ

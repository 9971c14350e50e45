"""Independent replay checker for solve and batch outputs.

Written from the problem statement (§II.B-C: tokens on a grid graph, one token per trap after
every elementary step, a move follows a shortest path free of other tokens; §IV: a batch is a
set of simultaneous elementary steps that pairwise share no trap).  It shares no code with the
oracle or with the HIP library: it only replays what they output.
"""
from __future__ import annotations

import numpy as np

from rr_inputs import unpack_rows

DIRS = {0: (1, 0), 1: (-1, 0), 2: (0, 1), 3: (0, -1)}


def feasibility_margin(shape, dense):
    """F = N - D - |T|, D = band-row tokens beyond the target width when side columns exist."""
    w, h, x0, y0, x1, y1 = shape
    sw, sh = x1 - x0, y1 - y0
    n = int(dense.sum())
    d = 0
    if x0 > 0 or x1 < w:
        for y in range(y0, y1):
            d += max(0, int(dense[y].sum()) - sw)
    return n - d - sw * sh


def path_cells(m):
    """Trap sequence of move (sx, sy, dx, dy): along row sy to column dx, then along column dx."""
    sx, sy, dx, dy = (int(v) for v in m)
    cells = [(sx, sy)]
    x, y = sx, sy
    while x != dx:
        x += 1 if dx > x else -1
        cells.append((x, y))
    while y != dy:
        y += 1 if dy > y else -1
        cells.append((x, y))
    return cells


def check_solve(shape, occ, res):
    """Validate one solve result against the problem statement.  Raises AssertionError."""
    w, h, x0, y0, x1, y1 = shape
    grid = unpack_rows(occ, w).copy()          # grid[y][x]
    n0 = int(grid.sum())
    margin = feasibility_margin(shape, grid)
    status = res["status"]
    moves = np.asarray(res["moves"]).reshape(-1, 4)
    goff = np.asarray(res["group_off"])
    final = unpack_rows(res["final"], w)
    if status == 1:
        assert margin < 0, "reported infeasible although F >= 0"
        assert len(moves) == 0
        assert np.array_equal(final, grid)
        return
    assert status == 0, f"status {status}"
    assert margin >= 0, "solved although F < 0"
    assert goff[0] == 0 and goff[-1] == len(moves)
    assert np.all(np.diff(goff.astype(np.int64)) > 0), "empty or reversed group"
    steps = 0
    for m in moves:
        cells = path_cells(m)
        assert len(cells) >= 2, "zero-length move"
        sx, sy = cells[0]
        assert grid[sy, sx] == 1, f"source {cells[0]} empty for move {m}"
        for (x, y) in cells[1:]:
            assert 0 <= x < w and 0 <= y < h
            assert grid[y, x] == 0, f"move {tuple(m)} obstructed at {(x, y)}"
        grid[sy, sx] = 0
        dx_, dy_ = cells[-1]
        grid[dy_, dx_] = 1
        steps += len(cells) - 1
    assert steps == res["n_steps"], "n_steps is not the summed path length"
    assert int(grid.sum()) == n0, "token count changed"
    assert np.array_equal(grid, final), "final grid differs from replay"
    assert grid[y0:y1, x0:x1].all(), "target not covered"


def check_batches(shape, occ, moves, final, batch_off, steps, flags=0):
    """Replay batches of unit steps.  Every step must be the next step of a path whose current
    trap is its source; a batch's steps share no trap; all sources are occupied and all
    destinations empty at the batch's start; the batch obeys the local constraint; the replay
    ends on the solve's final grid with every path complete."""
    w, h = shape[0], shape[1]
    grid = unpack_rows(occ, w).copy()
    moves = np.asarray(moves).reshape(-1, 4)
    paths = [path_cells(m) for m in moves]
    pos = [0] * len(paths)
    at = {}                                     # trap -> unfinished paths currently there
    for b, p in enumerate(paths):
        at.setdefault(p[0], []).append(b)
    batch_off = np.asarray(batch_off).astype(np.int64)
    steps = np.asarray(steps).astype(np.int64)
    assert batch_off[0] == 0 and batch_off[-1] == len(steps)
    longest = max((len(p) - 1 for p in paths), default=0)
    assert len(batch_off) - 1 >= longest
    for k in range(len(batch_off) - 1):
        seg = steps[batch_off[k]:batch_off[k + 1]]
        assert len(seg) > 0, "empty batch"
        dec = []
        for s in seg.tolist():
            d, x, y = s >> 30, (s >> 15) & 0x7FFF, s & 0x7FFF
            ddx, ddy = DIRS[d]
            dec.append((d, (x, y), (x + ddx, y + ddy)))
        used = set()
        owners = []
        for (d, u, v) in dec:
            assert u not in used and v not in used, "batch steps share a trap"
            used.add(u); used.add(v)
            assert grid[u[1], u[0]] == 1, "step from an empty trap"
            assert 0 <= v[0] < w and 0 <= v[1] < h
            assert grid[v[1], v[0]] == 0, "step into an occupied trap"
            cand = [b for b in at.get(u, []) if paths[b][pos[b] + 1] == v]
            assert cand, "step is no path's next step"
            started = [b for b in cand if pos[b] > 0]
            owners.append(min(started) if started else min(cand))
        if flags != 2:
            for a in range(len(dec)):
                for c in range(a + 1, len(dec)):
                    da, ua, _ = dec[a]
                    dc, uc, _ = dec[c]
                    assert da == dc, "mixed directions in a constrained batch"
                    if flags == 1:
                        assert (ua[0] == uc[0]) if da >= 2 else (ua[1] == uc[1]), "not along one line"
                    else:
                        assert ua[0] == uc[0] or ua[1] == uc[1], "steps share neither row nor column"
        for (d, u, v), b in zip(dec, owners):
            grid[u[1], u[0]] = 0
            at[u].remove(b)
            pos[b] += 1
            if pos[b] < len(paths[b]) - 1:
                at.setdefault(v, []).append(b)
        for (d, u, v) in dec:
            grid[v[1], v[0]] = 1
    assert all(pos[b] == len(paths[b]) - 1 for b in range(len(paths))), "a path was not completed"
    assert np.array_equal(grid, unpack_rows(final, w)), "batch replay does not end on the final grid"

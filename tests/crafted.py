"""Hand-made batching inputs (moves and groups that no solve emits) for the batching routine's
limits.  Moves are (sx, sy, dx, dy): along row sy to column dx, then along column dx (§II.C)."""
import numpy as np


def wide_release(side=64, rows=(0, 16, 32, 48), width=60):
    """Group 0 sweeps the given rows end to end; group k (k >= 1) then holds `width` one-step
    vertical moves leaving row rows[k-1], one per column.  Each such group waits on group 0
    only (it touches group 0's row) and its moves are pairwise disjoint, so when group 0
    finishes, len(rows) * width moves become ready at once (Alg. 3's ready set jumps from
    len(rows) to len(rows) * width)."""
    moves = [(0, r, side - 1, r) for r in rows]
    group_off = [0, len(moves)]
    for r in rows:
        moves += [(c, r, c, r + 1) for c in range(width)]
        group_off.append(len(moves))
    mv = np.asarray(moves, np.uint16)
    n_steps = int((np.abs(mv[:, 2].astype(int) - mv[:, 0]) + np.abs(mv[:, 3].astype(int) - mv[:, 1])).sum())
    shape = (side, side, 0, 0, side, side)
    return shape, mv, np.asarray(group_off, np.uint32), n_steps

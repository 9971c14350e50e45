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


def long_row(side=64, n=600, length=40, row=0):
    """n moves, all along row `row` from column 0 to column `length` (one group).  Every trap
    of the row's first length + 1 columns is on all n paths: the instance's touch lists
    (n * (length + 1) entries) exceed a 64 KiB graph budget, so the tiled build takes it, and
    the row's range holds n long horizontal legs -- more than the wave queue's 512."""
    moves = [(0, row, length, row)] * n
    mv = np.asarray(moves, np.uint16)
    return (side, side, 0, 0, side, side), mv, np.asarray([0, n], np.uint32), n * length

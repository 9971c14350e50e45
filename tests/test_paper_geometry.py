"""The paper's benchmark geometry (32 columns x ceil(32 / 0.6) = 54 rows, a full-width centred
32 x 32 target, exactly floor(0.6 * 32 * 54) = 1036 atoms drawn uniformly): the fixed-count
loading, and the oracle on it -- the row pre-pass is skipped for a full-width target, and every
result satisfies the problem statement and replays as legal batches."""
import numpy as np
import pytest

import oracle
import rr_inputs as ri
from checker import check_batches, check_solve


def test_fixed_count_loading():
    g = ri.fixed_count_grid(6, 0, 32, 54, 1036)
    assert g.shape == (54, 32) and int(g.sum()) == 1036
    assert int(ri.fixed_count_grid(6, 0, 5, 3, 0).sum()) == 0
    assert int(ri.fixed_count_grid(6, 0, 5, 3, 15).sum()) == 15
    with pytest.raises(ValueError):
        ri.fixed_count_grid(6, 0, 5, 3, 16)
    # another shot or seed is another draw; the same one is the same draw
    assert not np.array_equal(g, ri.fixed_count_grid(6, 1, 32, 54, 1036))
    assert not np.array_equal(g, ri.fixed_count_grid(7, 0, 32, 54, 1036))
    assert np.array_equal(g, ri.fixed_count_grid(6, 0, 32, 54, 1036))
    # uniform over cells: over 400 draws of 4 atoms in 8 cells, every cell is hit about 200 times
    hits = sum(ri.fixed_count_grid(9, s, 4, 2, 4).astype(int) for s in range(400))
    assert hits.sum() == 1600 and hits.min() > 150 and hits.max() < 250


def test_workload_shape():
    shots = ri.config_shots("paper32", n=3)
    d = shots[0]
    assert (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) == (32, 54, 0, 11, 32, 43)
    assert all(int(ri.unpack_rows(ri.shot_grid(s), 32).sum()) == 1036 for s in shots)
    assert len(ri.config_shots("paper32")) == 1000


@pytest.mark.parametrize("shot", range(6))
def test_oracle_on_paper_geometry(shot):
    d = ri.config_shots("paper32", n=1, first=shot)[0]
    shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
    occ = ri.shot_grid(d)
    r = oracle.solve(shape, occ)
    check_solve(shape, occ, r)
    assert r["status"] == 0                    # 1036 >= 1024 atoms, none parked: always feasible
    mv = np.asarray(r["moves"]).reshape(-1, 4)
    # full width: no row pre-pass, so no move changes column inside the band rows before the
    # columns are balanced -- every move of the first group is vertical
    first = mv[r["group_off"][0]:r["group_off"][1]]
    assert len(first) and np.all(first[:, 0] == first[:, 2])
    for flags in (0, 2):
        b = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags)
        check_batches(shape, occ, r["moves"], r["final"], b["batch_off"], b["steps"], flags=flags)

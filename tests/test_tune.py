"""Launch-schedule table (paper_2504_06182_amd/tune.py): host logic on the CPU; the tuner itself
on the GPU, where every schedule it tries must leave the batching outputs bit for bit the same."""
import json

import numpy as np
import pytest

from paper_2504_06182_amd import tune


def test_schedule_bits_and_merge(tmp_path):
    assert tune.schedule_bits(64, 1) == (64 << 24) | (1 << 8)
    with pytest.raises(ValueError):
        tune.schedule_bits(0, 1)
    with pytest.raises(ValueError):
        tune.schedule_bits(64, 256)
    table = {"classes": {"64": {"graph_kib": 48, "loop_kib": 4}}}
    # the constraint bits pass through, the tuned budgets are added
    assert tune.flags_for(64, 1, table) == 1 | (48 << 24) | (4 << 8)
    # a caller's own schedule wins, as does a class with no entry
    assert tune.flags_for(64, 2 | (16 << 8), table) == 2 | (16 << 8)
    assert tune.flags_for(128, 2, table) == 2
    p = tmp_path / "s.json"
    p.write_text(json.dumps(table))
    assert tune.load_table(str(p)) == table
    assert tune.load_table(str(tmp_path / "none.json")) == {"classes": {}}
    p.write_text("{}")
    with pytest.raises(ValueError):
        tune.load_table(str(p))


def test_committed_table_is_well_formed():
    t = tune.load_table()
    for c, e in t["classes"].items():
        assert int(c) in (64, 128, 192, 256)
        tune.schedule_bits(e["graph_kib"], e["loop_kib"])


@pytest.mark.gpu
def test_tuner_keeps_outputs_and_picks_a_candidate():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import rr_inputs as ri
    from paper_2504_06182_amd.pipeline import ManyBuffers
    torch.cuda.set_device(0)
    shots = [d for d in ri.config_shots("mixed", n=40) if d["w"] <= 128][:16]
    print("case tune 16 uneven shots", flush=True)
    shapes = [(d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"]) for d in shots]
    mb = ManyBuffers(shapes).load([ri.shot_grid(d) for d in shots]).solve()
    torch.cuda.synchronize()
    mb.plan_batches([max(int(i[3]), 1) for i in mb.solve_infos()])
    for constraint in (0, 2):
        e = tune.tune_class(mb, constraint, graph_kib=(16, 64, 150), loop_kib=(1, 24, 64), reps=1)
        assert e["graph_kib"] in (16, 64, 150) and e["loop_kib"] in (1, 24, 64)
        assert e["graph_ms"] > 0 and e["loop_ms"] > 0
        assert np.all(mb.batch_infos()[:, 0].view(np.int32) >= 0)


def test_loop_budgets_below_the_floor_are_one_schedule():
    # 64 class: 8*128 + 16*64*2 + 16 = 3088 B; 256 class: 8*512 + 16*64*6 + 16 = 10256 B
    assert tune.loop_lds_floor(64) == 3088 and tune.loop_lds_floor(256) == 10256
    assert tune._distinct_loop_budgets(64, (1, 2, 4, 8)) == [1, 4, 8]
    assert tune._distinct_loop_budgets(256, (1, 4, 8, 16, 32)) == [1, 16, 32]


"""rr_batch_moves_noalloc (batching with the library's own device array as workspace) against
rr_batch_moves with a caller workspace: the same bytes on two calls in a row, the second on a
smaller instance, so that the array holds the first call's contents when the second runs."""
import os
import sys

import numpy as np
import pytest

import oracle
import rr_inputs as ri

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_06182_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    import paper_2504_06182_amd
    paper_2504_06182_amd.lib()
    torch.cuda.set_device(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_caller_workspace_on_two_calls():
    import paper_2504_06182_amd as rr
    from paper_2504_06182_amd.pipeline import BatchBuffers, SolveBuffers
    for name, flags in (("single128", 0), ("single32", 1)):
        d = ri.config_shots(name)[0]
        shape = (d["w"], d["h"], d["x0"], d["y0"], d["x1"], d["y1"])
        occ = ri.shot_grid(d)
        say("case noalloc", name, shape, "flags", flags)
        sb = SolveBuffers(shape).load(occ).run()
        torch.cuda.synchronize()
        g = sb.host()
        assert g["status"] == 0
        n = g["n_steps"]
        ref = BatchBuffers(sb, step_cap=n).run(flags)
        torch.cuda.synchronize()
        out = BatchBuffers(sb, step_cap=n)
        out.batch_off.fill_(-1)
        out.steps.fill_(-1)
        out.info.fill_(-1)
        rr.rr_batch_moves_noalloc(shape, sb.moves, sb.group_off, sb.info, sb.move_cap, flags, out.batch_off,
                                  out.batch_cap, out.steps, out.step_cap, out.info)
        torch.cuda.synchronize()
        assert torch.equal(out.info, ref.info)
        assert torch.equal(out.steps, ref.steps)
        nb = ref.host()["n_batches"]
        assert torch.equal(out.batch_off[:nb + 1], ref.batch_off[:nb + 1])
        r = oracle.solve(shape, occ)
        rb = oracle.batch(shape, r["moves"], r["group_off"], r["n_steps"], flags=flags, indexed=True)
        h = out.host()
        assert h["status"] == 0
        assert np.array_equal(h["steps"], rb["steps"]) and np.array_equal(h["batch_off"], rb["batch_off"])

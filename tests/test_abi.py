"""The C-ABI library loads on a CPU-only host, exports every entry point of include/rr.h, and
rejects bad host-side arguments before any launch."""
import os
import re
import subprocess

import pytest

import paper_2504_06182_amd as rr
from paper_2504_06182_amd import build as rrbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(rrbuild.LIB):
        rrbuild.build()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rr_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rr_solve", "rr_batch_moves", "rr_solve_many", "rr_batch_moves_many",
              "rr_solve_workspace_bytes", "rr_batch_workspace_bytes", "rr_version"):
        assert n in names


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", rrbuild.LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(rr_[a-z_0-9]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = rr.lib()
    for n in declared_functions():
        assert hasattr(L, n)


def test_host_only_calls():
    assert "gfx950" in rr.rr_version()
    assert rr.rr_solve_workspace_bytes((64, 64, 10, 10, 54, 54)) == 0
    a = rr.rr_batch_workspace_bytes((64, 64, 10, 10, 54, 54), 4000, 20000)
    b = rr.rr_batch_workspace_bytes((64, 64, 10, 10, 54, 54), 4000, 40000)
    assert 0 < a < b


@pytest.mark.parametrize("shape", [(0, 4, 0, 0, 1, 1), (4, 4, 2, 0, 2, 1), (4, 4, 0, 3, 4, 5), (4, 4, 0, 0, 5, 1)])
def test_invalid_shapes_are_rejected_before_launch(shape):
    rc = rr.rr_solve(shape, 8, 8, 10, 8, 10, 8, 8, 0, None, 0, stream=0, check=False)
    assert rc == rr.RR_E_INVAL


def test_unknown_solve_order_is_rejected():
    rc = rr.rr_solve((32, 32, 8, 8, 24, 24), 8, 8, 10, 8, 10, 8, 8, 3, None, 0, stream=0, check=False)
    assert rc == rr.RR_E_INVAL
    rc = rr.rr_solve_many(1, 8, 32, 32, 8, 8, 8, 8, 8, 7, None, 0, stream=0, check=False)
    assert rc == rr.RR_E_INVAL


def test_oversized_grid_is_unsupported():
    rc = rr.rr_solve((1100, 300, 10, 10, 20, 20), 8, 8, 10, 8, 10, 8, 8, 0, None, 0, stream=0, check=False)
    assert rc == rr.RR_E_UNSUPPORTED
    rc = rr.rr_batch_moves((300, 1025, 1, 1, 2, 2), 8, 8, 8, 2, 0, 8, 8, 8, 8, 8, 8, 1 << 20, stream=0, check=False)
    assert rc == rr.RR_E_UNSUPPORTED
    rc = rr.rr_solve_many(1, 8, 1025, 32, 8, 8, 8, 8, 8, 0, None, 0, stream=0, check=False)
    assert rc == rr.RR_E_UNSUPPORTED


def test_wide_grids_need_a_solve_workspace():
    """Grids beyond RR_LDS_SIDE keep the solve's state in the caller's workspace: its size is
    reported, a missing, short or misaligned one is refused, and so is a wavefront field (the
    wide kernel runs 16 wavefronts); up to RR_LDS_SIDE none is needed."""
    assert rr.RR_MAX_SIDE == 1024 and rr.RR_LDS_SIDE == 256
    assert rr.rr_solve_workspace_bytes((256, 256, 10, 10, 200, 200)) == 0
    need = rr.rr_solve_workspace_bytes((257, 8, 10, 1, 200, 5))
    assert need > 0 and need % 256 == 0 and need == rr.rr_solve_workspace_bytes((1024, 1024, 0, 0, 1024, 1024))
    shape = (300, 300, 10, 10, 290, 290)
    assert rr.rr_solve(shape, 8, 8, 10, 8, 10, 8, 8, 0, None, 0, stream=0, check=False) == rr.RR_E_NOMEM
    assert rr.rr_solve(shape, 8, 8, 10, 8, 10, 8, 8, 0, 256, need - 1, stream=0, check=False) == rr.RR_E_NOMEM
    assert rr.rr_solve(shape, 8, 8, 10, 8, 10, 8, 8, 0, 264, need, stream=0, check=False) == rr.RR_E_NOMEM
    assert rr.rr_solve(shape, 8, 8, 10, 8, 10, 8, 8, 4 << 8, 256, need, stream=0, check=False) == rr.RR_E_INVAL
    assert rr.rr_solve_many(3, 8, 300, 300, 8, 8, 8, 8, 8, 0, 256, 3 * need - 1, stream=0,
                            check=False) == rr.RR_E_NOMEM
    # batching: the wide layout depends on the grid and the move capacity only
    a = rr.rr_batch_workspace_bytes(shape, 1000, 10)
    assert a == rr.rr_batch_workspace_bytes(shape, 1000, 10_000) and a < rr.rr_batch_workspace_bytes(shape, 2000, 10)


def test_null_outputs_and_small_workspace_rejected():
    shape = (32, 32, 8, 8, 24, 24)
    assert rr.rr_solve(shape, 8, 8, 10, None, 10, 8, 8, 0, None, 0, stream=0, check=False) == rr.RR_E_INVAL
    assert rr.rr_solve(shape, 8, 12, 10, 8, 10, 8, 8, 0, None, 0, stream=0, check=False) == rr.RR_E_INVAL  # misaligned
    need = rr.rr_batch_workspace_bytes(shape, 100, 100)
    rc = rr.rr_batch_moves(shape, 8, 8, 8, 100, 0, 8, 100, 8, 100, 8, 8, need - 1, stream=0, check=False)
    assert rc == rr.RR_E_NOMEM
    rc = rr.rr_batch_moves(shape, 8, 8, 8, 100, 7, 8, 100, 8, 100, 8, 8, need, stream=0, check=False)
    assert rc == rr.RR_E_INVAL


def test_noalloc_refuses_oversized_workspace_before_launch():
    shape = (256, 256, 38, 38, 217, 217)
    mc = 2 * 179 * 179
    fits = rr.rr_batch_workspace_bytes(shape, mc, 3_000_000)
    assert fits <= rr.RR_NOALLOC_WORKSPACE_BYTES < rr.rr_batch_workspace_bytes(shape, mc, 3_100_000)
    rc = rr.rr_batch_moves_noalloc(shape, 8, 8, 8, mc, 0, 8, 3_100_000, 8, 3_100_000, 8, stream=0, check=False)
    assert rc == rr.RR_E_NOMEM
    rc = rr.rr_batch_moves_noalloc((300, 300, 1, 1, 2, 2), 8, 8, 8, 2, 0, 8, 8, 8, 8, 8, stream=0, check=False)
    assert rc == rr.RR_E_UNSUPPORTED


def test_solve_waves_per_instance_checked_before_launch():
    """Wavefronts per instance (flags bits 8..11): 1, 2 or 4, at least one thread per grid side;
    anything else is refused before any launch."""
    for shape, waves in (((100, 100, 10, 10, 90, 90), 1), ((200, 200, 10, 10, 190, 190), 2),
                         ((32, 32, 8, 8, 24, 24), 3), ((32, 32, 8, 8, 24, 24), 8)):
        rc = rr.rr_solve(shape, 8, 8, 10, 8, 10, 8, 8, waves << 8, None, 0, stream=0, check=False)
        assert rc == rr.RR_E_INVAL, (shape, waves)
    rc = rr.rr_solve_many(1, 8, 200, 200, 8, 8, 8, 8, 8, 2 << 8, None, 0, stream=0, check=False)
    assert rc == rr.RR_E_INVAL


def test_batch_graph_waves_checked_before_launch():
    shape = (32, 32, 8, 8, 24, 24)
    need = rr.rr_batch_workspace_bytes(shape, 100, 100)
    for bad in (1 << 17, 3 << 20, 15 << 20):
        rc = rr.rr_batch_moves(shape, 8, 8, 8, 100, bad, 8, 100, 8, 100, 8, 8, need, stream=0, check=False)
        assert rc == rr.RR_E_INVAL, hex(bad)

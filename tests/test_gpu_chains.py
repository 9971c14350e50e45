"""GPU parity of exact 1D on chains (rr_solve_chains) through the C ABI: against the oracle's
chain form bit for bit, against rr_solve on the same 1 x N grid for N <= 256, in LDS and in
the workspace, for the paper's chain geometry (1024 traps) and the longest chain the move format
holds (65535 traps).  Every case prints its name before it touches the GPU."""
import os
import random
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


def run_chains(chains, grids, max_len=None):
    from paper_2504_06182_amd.pipeline import ChainBuffers
    cb = ChainBuffers(chains, max_len=max_len).load(grids).solve()
    torch.cuda.synchronize()
    return cb


def same(g, r, tag):
    assert g["status"] == r["status"], (tag, g["status"], r["status"])
    assert np.array_equal(g["final"].reshape(-1), r["final"].reshape(-1)), tag
    if r["status"] == 0:
        assert np.array_equal(g["moves"], r["moves"]), tag
        assert np.array_equal(g["group_off"], r["group_off"]), tag
        assert g["n_steps"] == r["n_steps"], tag


def random_chains(seed, count, n_lo, n_hi):
    rng = random.Random(seed)
    chains, grids = [], []
    for i in range(count):
        n = rng.randint(n_lo, n_hi)
        t = rng.randint(1, n)
        b = rng.randint(0, n - t) if rng.random() < 0.7 else (n - t) // 2
        k = rng.choice([rng.randint(0, n), min(n, t + rng.randint(0, 3)), t])   # around a = t too
        chains.append((n, b, t))
        grids.append(ri.pack_rows(ri.fixed_count_grid(50 + seed, i, n, 1, k)))
    return chains, grids


def test_short_chains_equal_grid_solve_and_oracle():
    """300 chains of 1..256 traps in one launch: each equals the oracle's chain form and
    rr_solve on its 1 x N grid (one-instance launches for the first 40)."""
    from paper_2504_06182_amd.pipeline import SolveBuffers
    chains, grids = random_chains(1, 300, 1, 256)
    say("case short chains", len(chains))
    cb = run_chains(chains, grids)
    sinf = cb.solve_infos()
    for i, ((n, b, t), g) in enumerate(zip(chains, grids)):
        r = oracle.solve_chain(n, g[0], b, t)
        same(cb.host_solve(i, sinf), r, f"chain {i} {(n, b, t)}")
        if i < 40:
            sb = SolveBuffers((n, 1, b, 0, b + t, 1)).load(g).run()
            torch.cuda.synchronize()
            same(sb.host(), r, f"grid {i}")


def test_paper_chain_geometry_all_shots():
    """The paper's chain geometry: 1000 chains of 1024 traps, centre-compact target of 512,
    exactly 614 atoms, in one launch; every chain equals the oracle."""
    shots = ri.config_shots("chain1024")
    chains = [(d["w"], d["x0"], d["x1"] - d["x0"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    say("case chain1024", len(chains))
    cb = run_chains(chains, grids)
    sinf = cb.solve_infos()
    assert np.all(sinf[:, 0] == 0)
    for i, ((n, b, t), g) in enumerate(zip(chains, grids)):
        same(cb.host_solve(i, sinf), oracle.solve_chain(n, g[0], b, t), f"chain1024 {i}")


def test_lds_and_workspace_forms_agree():
    """Chains of 4000..8192 traps solved with token positions in LDS (max_len 8192) and in the
    workspace (max_len 8193, 1024-thread workgroups above 16384): same bytes, equal to the
    oracle on a sample."""
    chains, grids = random_chains(2, 24, 4000, 8192)
    say("case lds vs workspace", len(chains))
    a = run_chains(chains, grids, max_len=8192)
    b = run_chains(chains, grids, max_len=8193)
    c = run_chains(chains, grids, max_len=20000)
    sinf = a.solve_infos()
    for x in (b, c):
        assert np.array_equal(sinf, x.solve_infos())
        xinf = x.solve_infos()
        for i in range(len(chains)):
            same(x.host_solve(i, xinf), a.host_solve(i, sinf), f"form {i}")
    for i in range(0, len(chains), 6):
        n, b_, t = chains[i]
        same(a.host_solve(i, sinf), oracle.solve_chain(n, grids[i][0], b_, t), f"long {i}")


def test_longest_chains():
    """Chains of 65535 traps (the longest the move format holds), target of 32767, exactly
    39321 atoms: 16 in one launch, four compared with the oracle."""
    shots = ri.config_shots("chain65535")
    chains = [(d["w"], d["x0"], d["x1"] - d["x0"]) for d in shots]
    grids = [ri.shot_grid(d) for d in shots]
    say("case chain65535", len(chains))
    cb = run_chains(chains, grids)
    sinf = cb.solve_infos()
    assert np.all(sinf[:, 0] == 0)
    for i in (0, 5, 10, 15):
        n, b, t = chains[i]
        same(cb.host_solve(i, sinf), oracle.solve_chain(n, grids[i][0], b, t), f"chain65535 {i}")


def test_chain_edge_cases_and_errors():
    """One trap; full chain; no token; a = t; target at either end; a chain too short for its
    target's tokens (infeasible, final = input); a move capacity one short (exact need);
    a malformed descriptor (two rows) reported as RR_E_INVAL."""
    from paper_2504_06182_amd.pipeline import ChainBuffers
    cases = [((1, 0, 1), [1]), ((1, 0, 1), [0]), ((64, 10, 20), [1] * 64), ((64, 10, 20), [0] * 64),
             ((65, 0, 30), [1 if x % 2 else 0 for x in range(65)]),
             ((65, 35, 30), [1 if x % 2 else 0 for x in range(65)]),
             ((130, 50, 30), [1 if x < 30 else 0 for x in range(130)]),
             ((130, 50, 31), [1 if x < 30 else 0 for x in range(130)])]
    chains = [c for c, _ in cases]
    grids = [ri.pack_rows(np.array([row], np.uint8)) for _, row in cases]
    say("case chain edges")
    cb = run_chains(chains, grids)
    sinf = cb.solve_infos()
    for i, ((n, b, t), g) in enumerate(zip(chains, grids)):
        same(cb.host_solve(i, sinf), oracle.solve_chain(n, g[0], b, t), f"edge {i}")
    assert np.int32(sinf[7][0]) == 1
    # capacity: one move short
    n, b, t = 130, 50, 30
    r = oracle.solve_chain(n, grids[6][0], b, t)
    short = ChainBuffers([(n, b, t)])
    short.desc_np[0]["move_cap"] = len(r["moves"]) - 1
    short.desc.copy_(torch.from_numpy(short.desc_np.view(np.uint8).copy()).cuda())
    short.load([grids[6]]).solve()
    torch.cuda.synchronize()
    inf = short.solve_infos()[0]
    assert np.int32(inf[0]) == -2 and inf[4] == len(r["moves"]) and inf[5] == 1
    # a descriptor with two rows is not a chain
    bad = ChainBuffers([(64, 10, 20)])
    bad.desc_np[0]["h"], bad.desc_np[0]["y1"] = 2, 2
    bad.desc.copy_(torch.from_numpy(bad.desc_np.view(np.uint8).copy()).cuda())
    bad.load([grids[2]]).solve()
    torch.cuda.synchronize()
    assert np.int32(bad.solve_infos()[0][0]) == -1

"""Device-buffer management around librr: sizes, arenas and descriptors, plus host readback.

Nothing here computes any part of the method: it allocates torch device tensors as raw storage,
lays out per-instance arenas, fills descriptors and calls the C entry points through the binding.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (rr_batch_moves, rr_batch_moves_many, rr_batch_moves_many_staged, rr_batch_workspace_bytes,
               rr_plan_many, rr_solve, rr_solve_chains, rr_solve_chains_workspace_bytes, rr_solve_many,
               rr_solve_workspace_bytes)
from .tune import flags_for, solve_flags_for

SOLVE_INFO_WORDS = 6   # rr_solve_info: int32 status + 5 x uint32
BATCH_INFO_WORDS = 5   # rr_batch_info: int32 status + 4 x uint32

DESC_DTYPE = np.dtype([("w", "<u2"), ("h", "<u2"), ("x0", "<u2"), ("y0", "<u2"), ("x1", "<u2"), ("y1", "<u2"),
                       ("pad0", "<u2"), ("pad1", "<u2"), ("move_cap", "<u4"), ("group_cap", "<u4"),
                       ("step_cap", "<u4"), ("batch_cap", "<u4"), ("occ_off", "<u8"), ("move_off", "<u8"),
                       ("group_off", "<u8"), ("step_off", "<u8"), ("batch_off", "<u8"), ("ws_off", "<u8")])
assert DESC_DTYPE.itemsize == 80


def words_per_row(w: int) -> int:
    return (int(w) + 63) // 64


def solve_caps(shape):
    """Output capacities that always suffice for one solve: 2*sw*sh moves, sw+sh groups."""
    w, h, x0, y0, x1, y1 = (int(v) for v in shape)
    sw, sh = x1 - x0, y1 - y0
    return 2 * sw * sh, sw + sh


def _dev(n, dtype, device):
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


def _u64_to_dev(a: np.ndarray, device) -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64).reshape(-1).copy()).to(device)


def _host_u32(t: torch.Tensor, n=None) -> np.ndarray:
    a = t.detach().cpu().numpy().view(np.uint32)
    return a if n is None else a[:n]


# ------------------------------------------------------------------------------------------
# one instance


class SolveBuffers:
    """Device buffers of one rr_solve call (capacities default to the always-sufficient ones)."""

    def __init__(self, shape, device="cuda", move_cap=None, group_cap=None, flags=0):
        self.shape = tuple(int(v) for v in shape)
        self.flags = int(flags)                  # order of Alg. 1 (RR_REDREC_*)
        mc, gc = solve_caps(shape)
        self.move_cap = mc if move_cap is None else int(move_cap)
        self.group_cap = gc if group_cap is None else int(group_cap)
        w, h = self.shape[0], self.shape[1]
        self.nwords = h * words_per_row(w)
        self.occ = _dev(self.nwords, torch.int64, device)
        self.moves = _dev(self.move_cap, torch.int64, device)            # rr_move = 8 bytes
        self.group_off = _dev(self.group_cap + 1, torch.int32, device)
        self.final = _dev(self.nwords, torch.int64, device)
        self.info = _dev(SOLVE_INFO_WORDS, torch.int32, device)
        self.ws_bytes = rr_solve_workspace_bytes(self.shape)     # grids beyond 256 per side
        self.ws = _dev((self.ws_bytes + 7) // 8, torch.int64, device) if self.ws_bytes else None

    def load(self, occ_rows: np.ndarray):
        self.occ.copy_(_u64_to_dev(occ_rows, self.occ.device))
        return self

    def run(self, stream=None):
        rr_solve(self.shape, self.occ, self.moves, self.move_cap, self.group_off, self.group_cap,
                 self.final, self.info, self.flags, self.ws, self.ws_bytes, stream)
        return self

    def host(self):
        """Read the result back: dict(status, moves uint16[n][4], group_off, final, n_steps, need_*)."""
        info = self.info.detach().cpu().numpy().view(np.uint32)
        status = int(np.int32(info[0]))
        n_moves, n_groups, n_steps, need_m, need_g = (int(v) for v in info[1:6])
        w, h = self.shape[0], self.shape[1]
        out = dict(status=status, n_steps=n_steps, need_moves=need_m, need_groups=need_g,
                   n_moves=n_moves, n_groups=n_groups)
        out["final"] = self.final.detach().cpu().numpy().view(np.uint64)[:self.nwords].reshape(h, words_per_row(w))
        if status == 0:
            mv = self.moves.detach().cpu().numpy()[:n_moves].view(np.uint16).reshape(-1, 4)
            out["moves"] = mv.copy()
            out["group_off"] = _host_u32(self.group_off, n_groups + 1).copy()
        elif status == 1:
            out["moves"] = np.zeros((0, 4), np.uint16)
            out["group_off"] = _host_u32(self.group_off, 1).copy()
        return out


class BatchBuffers:
    """Device buffers of one rr_batch_moves call for a solved SolveBuffers."""

    def __init__(self, sb: SolveBuffers, step_cap: int, batch_cap=None, device="cuda"):
        self.sb = sb
        self.step_cap = int(step_cap)
        self.batch_cap = self.step_cap if batch_cap is None else int(batch_cap)
        self.batch_off = _dev(self.batch_cap + 1, torch.int32, device)
        self.steps = _dev(self.step_cap, torch.int32, device)
        self.info = _dev(BATCH_INFO_WORDS, torch.int32, device)
        self.ws_bytes = rr_batch_workspace_bytes(sb.shape, sb.move_cap, self.step_cap)
        self.ws = _dev((self.ws_bytes + 7) // 8, torch.int64, device)

    def run(self, flags=0, stream=None):
        sb = self.sb
        rr_batch_moves(sb.shape, sb.moves, sb.group_off, sb.info, sb.move_cap, flags, self.batch_off,
                       self.batch_cap, self.steps, self.step_cap, self.info, self.ws, self.ws_bytes, stream)
        return self

    def host(self):
        info = self.info.detach().cpu().numpy().view(np.uint32)
        status = int(np.int32(info[0]))
        nb, ns, need_b, need_s = (int(v) for v in info[1:5])
        out = dict(status=status, n_batches=nb, n_steps=ns, need_batches=need_b, need_steps=need_s)
        if status == 0:
            out["batch_off"] = _host_u32(self.batch_off, nb + 1).copy()
            out["steps"] = _host_u32(self.steps, ns).copy()
        return out


# ------------------------------------------------------------------------------------------
# many instances in one launch


class ManyBuffers:
    """Arenas and descriptors for rr_solve_many / rr_batch_moves_many over a list of shots.

    ``shapes``: list of (w, h, x0, y0, x1, y1).  Solve capacities are the always-sufficient ones.
    Batching capacities are set by :meth:`plan_batches` from per-instance step counts (exact
    counts read back after the solve, or caller-chosen bounds)."""

    def __init__(self, shapes, device="cuda", solve_flags=0):
        self.device = device
        self.solve_flags = int(solve_flags)      # order of Alg. 1 (RR_REDREC_*)
        self.n = len(shapes)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        d = np.zeros(self.n, DESC_DTYPE)
        occ_off = move_off = group_off = 0
        self.max_w = max(s[0] for s in self.shapes)
        self.max_h = max(s[1] for s in self.shapes)
        for i, s in enumerate(self.shapes):
            w, h, x0, y0, x1, y1 = s
            mc, gc = solve_caps(s)
            d[i]["w"], d[i]["h"], d[i]["x0"], d[i]["y0"], d[i]["x1"], d[i]["y1"] = w, h, x0, y0, x1, y1
            d[i]["move_cap"], d[i]["group_cap"] = mc, gc
            d[i]["occ_off"], d[i]["move_off"], d[i]["group_off"] = occ_off, move_off, group_off
            occ_off += h * words_per_row(w)
            move_off += mc
            group_off += gc + 1
        self.desc_np = d
        self.occ_words = occ_off
        self.occ = _dev(occ_off, torch.int64, device)
        self.final = _dev(occ_off, torch.int64, device)
        self.moves = _dev(move_off, torch.int64, device)
        self.groups = _dev(group_off, torch.int32, device)
        self.sinfo = _dev(self.n * SOLVE_INFO_WORDS, torch.int32, device)
        self.binfo = _dev(self.n * BATCH_INFO_WORDS, torch.int32, device)
        self.desc = torch.from_numpy(d.view(np.uint8).copy()).to(device)
        self.steps = self.batches = self.ws = None
        self.ws_bytes = 0
        big = [s for s in self.shapes if max(s[0], s[1]) > 256]
        self.solve_ws_bytes = self.n * rr_solve_workspace_bytes(big[0]) if big else 0
        self.solve_ws = _dev((self.solve_ws_bytes + 7) // 8, torch.int64, device) if big else None

    def load(self, grids):
        """grids: list of packed bit-row arrays, one per shot, in order."""
        flat = np.concatenate([np.ascontiguousarray(g, dtype=np.uint64).reshape(-1) for g in grids])
        assert flat.size == self.occ_words
        self.occ.copy_(_u64_to_dev(flat, self.device))
        return self

    def solve(self, stream=None):
        rr_solve_many(self.n, self.desc, self.max_w, self.max_h, self.occ, self.moves, self.groups, self.final,
                      self.sinfo, self.solve_flags, self.solve_ws, self.solve_ws_bytes, stream)
        return self

    def solve_infos(self) -> np.ndarray:
        return self.sinfo.detach().cpu().numpy().view(np.uint32).reshape(self.n, SOLVE_INFO_WORDS)

    def plan_batches(self, step_caps):
        """Lay out step/batch arenas and workspaces for per-instance step capacities."""
        d = self.desc_np
        step_off = batch_off = ws_off = 0
        for i, s in enumerate(self.shapes):
            sc = max(int(step_caps[i]), 1)
            d[i]["step_cap"], d[i]["batch_cap"] = sc, sc
            d[i]["step_off"], d[i]["batch_off"], d[i]["ws_off"] = step_off, batch_off, ws_off
            step_off += sc
            batch_off += sc + 1
            ws = rr_batch_workspace_bytes(s, int(d[i]["move_cap"]), sc)
            ws_off += (ws + 255) // 256 * 256
        self.steps = _dev(step_off, torch.int32, self.device)
        self.batches = _dev(batch_off, torch.int32, self.device)
        self.ws_bytes = ws_off
        self.ws = _dev((ws_off + 7) // 8, torch.int64, self.device)
        self.desc = torch.from_numpy(d.view(np.uint8).copy()).to(self.device)
        return self

    def alloc_pools(self, step_pool: int, batch_pool: int, ws_pool_bytes: int):
        """Pools for the device-side planner (rr_plan_many); sizes are caller-chosen bounds."""
        self.step_pool, self.batch_pool, self.ws_pool = int(step_pool), int(batch_pool), int(ws_pool_bytes)
        self.steps = _dev(self.step_pool, torch.int32, self.device)
        self.batches = _dev(self.batch_pool, torch.int32, self.device)
        self.ws_bytes = self.ws_pool
        self.ws = _dev((self.ws_pool + 7) // 8, torch.int64, self.device)
        self.totals = torch.zeros(3, dtype=torch.int64, device=self.device)
        return self

    def plan_device(self, stream=None):
        """Lay out the batching arenas on the device from the solve's step counts (no host sync)."""
        rr_plan_many(self.n, self.desc, self.sinfo, self.step_pool, self.batch_pool, self.ws_pool, self.totals,
                     stream)
        return self

    def refresh_desc(self):
        """Copy the device descriptors (as updated by the planner) back to the host mirror."""
        self.desc_np = self.desc.cpu().numpy().view(DESC_DTYPE).copy()
        return self

    def batch(self, flags=0, stream=None, graph_done_event=None, loop_done_event=None):
        """Batch every solved instance; the optional events (torch.cuda.Event) mark the end of the
        graph kernel and of the loop kernel on the stream (rr_batch_moves_many_staged)."""
        if graph_done_event is None and loop_done_event is None:
            rr_batch_moves_many(self.n, self.desc, self.max_w, self.max_h, self.moves, self.groups, self.sinfo,
                                flags, self.batches, self.steps, self.binfo, self.ws, self.ws_bytes, stream)
        else:
            rr_batch_moves_many_staged(self.n, self.desc, self.max_w, self.max_h, self.moves, self.groups,
                                       self.sinfo, flags, self.batches, self.steps, self.binfo, self.ws,
                                       self.ws_bytes, stream, graph_done_event, loop_done_event)
        return self

    def batch_infos(self) -> np.ndarray:
        return self.binfo.detach().cpu().numpy().view(np.uint32).reshape(self.n, BATCH_INFO_WORDS)

    def host_solve(self, i, infos=None, moves=None, groups=None, final=None):
        """Result of shot i in the layout of SolveBuffers.host()."""
        infos = self.solve_infos() if infos is None else infos
        d = self.desc_np[i]
        w, h = int(d["w"]), int(d["h"])
        nw = h * words_per_row(w)
        info = infos[i]
        status = int(np.int32(info[0]))
        out = dict(status=status, n_moves=int(info[1]), n_groups=int(info[2]), n_steps=int(info[3]),
                   need_moves=int(info[4]), need_groups=int(info[5]))
        final = self.final.detach().cpu().numpy() if final is None else final
        out["final"] = final[int(d["occ_off"]):int(d["occ_off"]) + nw].view(np.uint64).reshape(h, words_per_row(w))
        if status == 0:
            moves = self.moves.detach().cpu().numpy() if moves is None else moves
            groups = self.groups.detach().cpu().numpy().view(np.uint32) if groups is None else groups
            mo, go = int(d["move_off"]), int(d["group_off"])
            out["moves"] = moves[mo:mo + out["n_moves"]].view(np.uint16).reshape(-1, 4).copy()
            out["group_off"] = groups[go:go + out["n_groups"] + 1].copy()
        return out

    def host_batch(self, i, infos=None, steps=None, batches=None):
        infos = self.batch_infos() if infos is None else infos
        d = self.desc_np[i]
        info = infos[i]
        status = int(np.int32(info[0]))
        out = dict(status=status, n_batches=int(info[1]), n_steps=int(info[2]), need_batches=int(info[3]),
                   need_steps=int(info[4]))
        if status == 0:
            steps = self.steps.detach().cpu().numpy().view(np.uint32) if steps is None else steps
            batches = self.batches.detach().cpu().numpy().view(np.uint32) if batches is None else batches
            so, bo = int(d["step_off"]), int(d["batch_off"])
            out["steps"] = steps[so:so + out["n_steps"]].copy()
            out["batch_off"] = batches[bo:bo + out["n_batches"] + 1].copy()
        return out


class ChainBuffers(ManyBuffers):
    """Arenas for rr_solve_chains: chains given as (N, b, t) -- N traps, target [b, b+t) -- laid
    out as 1 x N grids (same arenas, descriptors and readback as ManyBuffers)."""

    def __init__(self, chains, device="cuda", max_len=None):
        shapes = [(int(n), 1, int(b), 0, int(b) + int(t), 1) for n, b, t in chains]
        super().__init__(shapes, device=device)
        self.max_len = int(max_len) if max_len is not None else self.max_w
        self.chain_ws_bytes = rr_solve_chains_workspace_bytes(self.n, self.max_len)
        self.chain_ws = _dev((self.chain_ws_bytes + 7) // 8, torch.int64, device) if self.chain_ws_bytes else None

    def solve(self, stream=None):
        rr_solve_chains(self.n, self.desc, self.max_len, self.occ, self.moves, self.groups, self.final, self.sinfo,
                        self.chain_ws, self.chain_ws_bytes, stream)
        return self


# ------------------------------------------------------------------------------------------
# uneven sizes: one launch chain per grid size class

SIZE_CLASSES = (64, 128, 192, 256)


def size_class(shape) -> int:
    """Smallest class (largest grid side it holds) for a shape: the batching launch of a class
    picks its register slots and LDS budgets from that side."""
    side = max(int(shape[0]), int(shape[1]))
    for c in SIZE_CLASSES:
        if side <= c:
            return c
    raise ValueError(f"grid side {side} above {SIZE_CLASSES[-1]}")


class ClassedBuffers:
    """Shots of uneven sizes split by size class, each class a ManyBuffers with device-planned
    batching pools.  ``run`` enqueues solve -> plan -> batch for every class (on one stream, or
    one stream per class), with no host synchronisation, so the whole pass can be captured in a
    graph and replayed."""

    def __init__(self, shapes, step_bound, device="cuda", algo=0):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.n = len(self.shapes)
        self.device = device
        by = {}
        for i, s in enumerate(self.shapes):
            by.setdefault(size_class(s), []).append(i)
        self.parts = []
        for c in SIZE_CLASSES:
            if c not in by:
                continue
            idx = np.array(by[c], np.int64)
            mb = ManyBuffers([self.shapes[i] for i in idx], device=device, solve_flags=solve_flags_for(c, algo))
            self.parts.append((c, idx, mb))
        self.step_bound = step_bound
        for _, idx, mb in self.parts:
            self._alloc(mb, [self.step_bound(mb.shapes[k]) for k in range(mb.n)])

    @staticmethod
    def _alloc(mb, bounds):
        steps = int(sum(max(int(b), 1) for b in bounds))
        ws = int(sum((rr_batch_workspace_bytes(s, solve_caps(s)[0], max(int(b), 1)) + 255) // 256 * 256
                     for s, b in zip(mb.shapes, bounds)))
        mb.alloc_pools(steps, steps + mb.n, ws)

    def load(self, grids):
        for _, idx, mb in self.parts:
            mb.load([grids[i] for i in idx])
        return self

    def run(self, flags=0, streams=None):
        """Enqueue every class.  With ``streams`` the classes fork from the current stream onto
        their own streams and join back (event edges, valid under graph capture).  Each class
        batches under its tuned launch schedule unless ``flags`` sets one (tune.flags_for)."""
        if streams is None:
            for c, _, mb in self.parts:
                mb.solve()
                mb.plan_device()
                mb.batch(flags_for(c, flags))
            return self
        cur = torch.cuda.current_stream()
        for k, (c, _, mb) in enumerate(self.parts):
            st = streams[k % len(streams)]
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                mb.solve(st)
                mb.plan_device(st)
                mb.batch(flags_for(c, flags), st)
        for k in range(min(len(streams), len(self.parts))):
            cur.wait_stream(streams[k])
        return self

    def fit_pools(self):
        """After a run: grow any pool the planner found too small (host sync), to the exact
        totals it reported.  Returns True when something was reallocated (run again)."""
        grown = False
        for _, _, mb in self.parts:
            tot = mb.totals.cpu().numpy()
            if tot[0] > mb.step_pool or tot[1] > mb.batch_pool or tot[2] > mb.ws_pool:
                mb.alloc_pools(int(tot[0]), int(tot[1]), int(tot[2]))
                grown = True
        return grown

    OUTPUTS = ("sinfo", "binfo", "moves", "groups", "final", "steps", "batches", "desc")

    def outputs(self):
        """Device copies of every array a run writes, per class: solve and batching infos, moves,
        group offsets, final grids, steps, batch offsets and the planned descriptors."""
        return [{k: getattr(mb, k).clone() for k in self.OUTPUTS} for _, _, mb in self.parts]

    def poison_outputs(self, byte=0x5A):
        """Fill every output array except the descriptors with ``byte`` (a device fill), so that
        a later run that leaves something unwritten is seen when its outputs are compared."""
        for _, _, mb in self.parts:
            for k in self.OUTPUTS[:-1]:
                getattr(mb, k).view(torch.uint8).fill_(byte)
        return self

    @staticmethod
    def same_outputs(a, b) -> bool:
        """Byte equality of two ``outputs()`` snapshots (compared on the device)."""
        return len(a) == len(b) and all(torch.equal(x[k], y[k]) for x, y in zip(a, b) for k in x)

    def infos(self):
        """(solve_infos, batch_infos) in the caller's shot order."""
        s = np.zeros((self.n, SOLVE_INFO_WORDS), np.uint32)
        b = np.zeros((self.n, BATCH_INFO_WORDS), np.uint32)
        for _, idx, mb in self.parts:
            s[idx] = mb.solve_infos()
            b[idx] = mb.batch_infos()
        return s, b

    def locate(self, i):
        for _, idx, mb in self.parts:
            k = np.nonzero(idx == i)[0]
            if k.size:
                return mb, int(k[0])
        raise IndexError(i)

    def host_solve(self, i):
        mb, k = self.locate(i)
        return mb.host_solve(k)

    def host_batch(self, i):
        mb, k = self.locate(i)
        mb.refresh_desc()
        return mb.host_batch(k)

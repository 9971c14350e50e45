"""Continuous-batching server for red-rec shots on one GPU.

Shots (a grid shape and its packed occupancy bits) arrive on the host at any time.  The server
keeps device-resident arenas per grid size class, each cut into fixed-size *slots* (input and
final bits, moves, group offsets, steps, batch ends, batching workspace), and admits a waiting
shot as soon as its class has a free slot: the number of slots per class is set by a device
memory budget (admission by memory).  Every admitted group of shots becomes one *wave*: the
wave's grids go to the device in one copy from pinned staging and are scattered into their slots,
then one ``rr_solve_many`` + ``rr_batch_moves_many`` pair runs over just those slots.  Each class
has several streams and a wave is launched only on a stream of its class that is idle, so while
the class's streams are busy, arrivals gather into the next, larger wave (a wave takes every
waiting shot its free slots and ``max_wave`` allow); waves of all classes overlap on the device.
A wave retires when its completion event has fired: its infos were copied into pinned host
memory on its own stream, so the host reads them without waiting on the device; its shots are
stamped done and their slots return to the free list.

Every result is that of a single ``rr_solve`` + ``rr_batch_moves`` on the same shot: the kernels
work per instance and are deterministic, and a slot is sized so that the shot fits (a shot whose
step count exceeds its slot's bound is re-run alone with exact buffers on a stream of its own,
retired by its event like a wave, and counted).

Nothing here computes any part of the method: it schedules, copies and launches.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import (RR_E_CAPACITY, RR_LDS_SIDE, RR_OK, rr_batch_moves_many, rr_batch_workspace_bytes, rr_solve_many,
               rr_solve_workspace_bytes)
from .tune import flags_for, solve_flags_for
from .pipeline import (BATCH_INFO_WORDS, DESC_DTYPE, SOLVE_INFO_WORDS, BatchBuffers, SolveBuffers,
                       solve_caps, words_per_row)


def step_bound(side: int) -> int:
    """Steps one slot of a class holds: 0.11 * side**3, never below 4096.  The configs' loadings
    take 0.067-0.069 * side**3 steps on average and at most 0.096 * side**3 (500 uneven shots,
    sides 32..128, oracle); a shot beyond its slot is re-run alone."""
    return max(4096, int(0.11 * side ** 3))


class _Class:
    """Slot arenas of one size class (largest grid side ``side``)."""

    def __init__(self, side, n_slots, n_streams, device, step_cap=None):
        self.side = side
        self.n = n_slots
        full = (side, side, 0, 0, side, side)
        self.occ_words = side * words_per_row(side)
        self.move_cap, self.group_cap = solve_caps(full)
        self.step_cap = step_bound(side) if step_cap is None else int(step_cap)
        self.ws_bytes = (rr_batch_workspace_bytes(full, self.move_cap, self.step_cap) + 255) // 256 * 256
        n = n_slots
        self.occ = torch.zeros(n * self.occ_words, dtype=torch.int64, device=device)
        self.final = torch.zeros_like(self.occ)
        self.moves = torch.empty(n * self.move_cap, dtype=torch.int64, device=device)
        self.groups = torch.empty(n * (self.group_cap + 1), dtype=torch.int32, device=device)
        self.steps = torch.empty(n * self.step_cap, dtype=torch.int32, device=device)
        self.batches = torch.empty(n * (self.step_cap + 1), dtype=torch.int32, device=device)
        self.ws = torch.empty((n * self.ws_bytes + 7) // 8, dtype=torch.int64, device=device)
        # grids beyond RR_LDS_SIDE: the solve's per-instance state, one slice per shot of a wave
        self.solve_ws_bytes = n * rr_solve_workspace_bytes(full)
        self.solve_ws = (torch.empty((self.solve_ws_bytes + 7) // 8, dtype=torch.int64, device=device)
                         if self.solve_ws_bytes else None)
        self.free = collections.deque(range(n))
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.on_stream = [None] * n_streams          # the wave last launched on each stream

    def idle_stream(self):
        """Index of a stream whose last wave has finished (or that never ran one), else None."""
        for j, w in enumerate(self.on_stream):
            if w is None or w.event.query():
                return j
        return None

    @staticmethod
    def slot_bytes(side, step_cap=None):
        full = (side, side, 0, 0, side, side)
        mc, gc = solve_caps(full)
        sc = step_bound(side) if step_cap is None else int(step_cap)
        return (16 * side * words_per_row(side) + 8 * mc + 4 * (gc + 1) + 8 * sc + 4 +
                rr_batch_workspace_bytes(full, mc, sc) + rr_solve_workspace_bytes(full) + 256)


class _Wave:
    pass


class Server:
    """Continuous batching over device-resident slot arenas (see the module docstring).

    ``budget_bytes``: device memory for all arenas, split over the size classes by ``class_share``
    (fractions; a class's slot count is its share over its slot size).  ``max_wave``: most shots
    one wave takes.  ``streams_per_class``: waves of one class in flight at once (one number, or
    one per class).  ``flags``: batching flags.  ``keep_results``: copy every shot's outputs to
    the host when its wave retires (for checking; off when only timing).  ``slot_steps``: steps a
    slot holds, per class (default step_bound)."""

    # streams per class: one wave each of the two small classes and two of the 256 class in
    # flight (one 256 stream makes waves so large that they crowd the small classes off the CUs:
    # 64-class p99 0.7-1.9 s at 20k shots/s).  Streams that share a hardware queue run in
    # submission order, so a small class behind a 256 wave (~0.2 s) or a 1024 wave (~3 s) on the
    # same queue waits for it; HIP maps streams onto GPU_MAX_HW_QUEUES queues (4 by default) in
    # an order the caller does not control, and torch hands out pooled streams, so a process
    # serving classes this way should run with as many queues as it has streams (bench.py sets
    # 32).  With 32 queues, at 20k shots/s: 64-class p50 / p99 7 / 65 ms with the 1024 class,
    # 7 / 76 ms without.
    STREAMS = {64: 1, 128: 1, 256: 2}
    STREAMS_LARGE = {64: 1, 128: 1, 256: 2, 1024: 1}

    def __init__(self, budget_bytes, class_share=None, max_wave=256, streams_per_class=None, flags=0,
                 keep_results=False, device="cuda", slot_steps=None):
        self.device = device
        self.flags = int(flags)
        self.max_wave = int(max_wave)
        self.keep = bool(keep_results)
        share = class_share or {64: 0.04, 128: 0.12, 256: 0.84}
        if streams_per_class is None:
            table = self.STREAMS_LARGE if any(side > RR_LDS_SIDE for side in share) else self.STREAMS
            streams_per_class = {side: table.get(side, 1) for side in share}
        elif not isinstance(streams_per_class, dict):
            streams_per_class = {side: int(streams_per_class) for side in share}
        self.streams_per_class = dict(streams_per_class)
        self.classes = {}
        slot_steps = slot_steps or {}
        for side, f in share.items():
            n = int(budget_bytes * f) // _Class.slot_bytes(side, slot_steps.get(side))
            if n > 0:
                self.classes[side] = _Class(side, n, streams_per_class[side], device, slot_steps.get(side))
        self.rerun_stream = torch.cuda.Stream(device=device)
        self.waiting = {side: collections.deque() for side in self.classes}
        self.inflight = []
        self.shots = []
        self.overflow = 0
        self.waves = 0

    def class_of(self, shape):
        """The server's class for a shape: the smallest of its classes that holds the grid (the
        server's classes are the keys of class_share; fewer classes than the launch-side size
        classes keep fewer waves in flight on the GPU's four hardware queues)."""
        side = max(int(shape[0]), int(shape[1]))
        fit = [c for c in self.classes if c >= side]
        if not fit:
            raise ValueError(f"grid side {side} above every class of this server")
        return min(fit)

    def slots(self):
        return {side: c.n for side, c in self.classes.items()}

    # ---- intake
    def submit(self, shape, grid, t_arrive=None):
        """Queue one shot (shape (w, h, x0, y0, x1, y1), packed bit rows); returns its id."""
        shape = tuple(int(v) for v in shape)
        side = self.class_of(shape)
        if side not in self.classes:
            raise ValueError(f"no slots for size class {side}")
        i = len(self.shots)
        self.shots.append(dict(shape=shape, grid=np.ascontiguousarray(grid, dtype=np.uint64).reshape(-1),
                               t_arrive=time.perf_counter() if t_arrive is None else t_arrive, t_done=None))
        self.waiting[side].append(i)
        return i

    # ---- one turn of the loop: admit and launch, then retire what finished
    def pump(self):
        launched = 0
        for side, c in self.classes.items():
            q = self.waiting[side]
            while q and c.free:
                j = c.idle_stream()
                if j is None:
                    break                              # the class's streams are busy: let the wave grow
                k = min(len(q), len(c.free), self.max_wave)
                self._launch(c, j, [q.popleft() for _ in range(k)], [c.free.popleft() for _ in range(k)])
                launched += 1
        self._retire()
        return launched

    def _launch(self, c, j, ids, slots):
        n = len(ids)
        d = np.zeros(n, DESC_DTYPE)
        stage = torch.zeros((n, c.occ_words), dtype=torch.int64, pin_memory=True)
        st_np = stage.numpy().view(np.uint64)
        for k, (i, s) in enumerate(zip(ids, slots)):
            sh = self.shots[i]
            w, h, x0, y0, x1, y1 = sh["shape"]
            mc, gc = solve_caps(sh["shape"])
            d[k]["w"], d[k]["h"], d[k]["x0"], d[k]["y0"], d[k]["x1"], d[k]["y1"] = w, h, x0, y0, x1, y1
            d[k]["move_cap"], d[k]["group_cap"] = mc, gc
            d[k]["step_cap"], d[k]["batch_cap"] = c.step_cap, c.step_cap
            d[k]["occ_off"] = s * c.occ_words
            d[k]["move_off"] = s * c.move_cap
            d[k]["group_off"] = s * (c.group_cap + 1)
            d[k]["step_off"] = s * c.step_cap
            d[k]["batch_off"] = s * (c.step_cap + 1)
            d[k]["ws_off"] = s * c.ws_bytes
            st_np[k, :sh["grid"].size] = sh["grid"]
            sh["slot"] = s
        desc_h = torch.from_numpy(d.view(np.uint8).copy()).pin_memory()
        idx_h = torch.tensor(slots, dtype=torch.int64).pin_memory()
        st = c.streams[j]
        w = _Wave()
        with torch.cuda.stream(st):
            desc = desc_h.to(self.device, non_blocking=True)
            idx = idx_h.to(self.device, non_blocking=True)
            rows = stage.to(self.device, non_blocking=True)
            c.occ.view(c.n, c.occ_words).index_copy_(0, idx, rows)
            w.sinfo = torch.empty(n * SOLVE_INFO_WORDS, dtype=torch.int32, device=self.device)
            w.binfo = torch.empty(n * BATCH_INFO_WORDS, dtype=torch.int32, device=self.device)
            rr_solve_many(n, desc, c.side, c.side, c.occ, c.moves, c.groups, c.final, w.sinfo,
                          solve_flags_for(c.side), c.solve_ws, c.solve_ws_bytes, st)
            rr_batch_moves_many(n, desc, c.side, c.side, c.moves, c.groups, w.sinfo, flags_for(c.side, self.flags),
                                c.batches, c.steps,
                                w.binfo, c.ws, c.ws.numel() * 8, st)
            # the infos come back on the wave's own stream, into pinned buffers the host reads
            # once the event has fired: retiring a wave never waits on the device
            w.sinfo_h = torch.empty(w.sinfo.numel(), dtype=torch.int32, pin_memory=True)
            w.binfo_h = torch.empty(w.binfo.numel(), dtype=torch.int32, pin_memory=True)
            w.sinfo_h.copy_(w.sinfo, non_blocking=True)
            w.binfo_h.copy_(w.binfo, non_blocking=True)
            w.event = torch.cuda.Event()
            w.event.record(st)
        w.cls, w.ids, w.slots, w.launched = c, ids, slots, time.perf_counter()
        w.keep_alive = (desc, idx, rows, desc_h, idx_h, stage)   # until the wave retires
        c.on_stream[j] = w
        self.inflight.append(w)
        self.waves += 1

    def _retire(self):
        still = []
        for w in self.inflight:
            if not w.event.query():
                still.append(w)
                continue
            now = time.perf_counter()
            if w.cls is None:                          # a shot re-run alone with exact buffers
                self._retire_rerun(w, now)
                continue
            si = w.sinfo_h.numpy().view(np.uint32).reshape(-1, SOLVE_INFO_WORDS)
            bi = w.binfo_h.numpy().view(np.uint32).reshape(-1, BATCH_INFO_WORDS)
            for k, i in enumerate(w.ids):
                sh = self.shots[i]
                sh["t_launch"] = w.launched
                if np.int32(bi[k, 0]) == RR_E_CAPACITY and np.int32(si[k, 0]) == RR_OK:
                    still.append(self._launch_rerun(i, int(si[k, 3])))   # more steps than the slot holds
                    continue
                sh["sinfo"], sh["binfo"] = si[k].copy(), bi[k].copy()
                if self.keep:
                    sh["out"] = self._copy_out(w.cls, w.slots[k], sh, si[k], bi[k])
                sh["t_done"] = time.perf_counter() if self.keep else now
            for s in w.slots:
                w.cls.free.append(s)
        self.inflight = still

    def _copy_out(self, c, s, sh, si, bi):
        w, h = sh["shape"][0], sh["shape"][1]
        nw = h * words_per_row(w)
        status = int(np.int32(si[0]))
        sol = dict(status=status, n_moves=int(si[1]), n_groups=int(si[2]), n_steps=int(si[3]))
        fin = c.final[s * c.occ_words:s * c.occ_words + nw].cpu().numpy().view(np.uint64)
        sol["final"] = fin.reshape(h, words_per_row(w))
        if status == 0:
            mv = c.moves[s * c.move_cap:s * c.move_cap + sol["n_moves"]].cpu().numpy()
            sol["moves"] = mv.view(np.uint16).reshape(-1, 4).copy()
            go = c.groups[s * (c.group_cap + 1):s * (c.group_cap + 1) + sol["n_groups"] + 1].cpu().numpy()
            sol["group_off"] = go.view(np.uint32).copy()
        bst = int(np.int32(bi[0]))
        bat = dict(status=bst, n_batches=int(bi[1]), n_steps=int(bi[2]))
        if bst == 0:
            bo = c.batches[s * (c.step_cap + 1):s * (c.step_cap + 1) + bat["n_batches"] + 1].cpu().numpy()
            bat["batch_off"] = bo.view(np.uint32).copy()
            sp = c.steps[s * c.step_cap:s * c.step_cap + bat["n_steps"]].cpu().numpy()
            bat["steps"] = sp.view(np.uint32).copy()
        return sol, bat

    def _launch_rerun(self, i, n_steps):
        """Re-run shot i alone with buffers sized to its exact step count, on the re-run stream,
        as a wave of its own (retired by its event like the others; nothing waits for it)."""
        self.overflow += 1
        sh = self.shots[i]
        w = _Wave()
        w.cls, w.ids, w.slots, w.launched = None, [i], [], time.perf_counter()
        st = self.rerun_stream
        with torch.cuda.stream(st):
            w.sb = SolveBuffers(sh["shape"], device=self.device)
            w.sb.occ.copy_(torch.from_numpy(sh["grid"].view(np.int64)).to(self.device, non_blocking=False))
            w.sb.run(st)
            w.bb = BatchBuffers(w.sb, step_cap=max(n_steps, 1), device=self.device).run(self.flags, st)
            w.event = torch.cuda.Event()
            w.event.record(st)
        return w

    def _retire_rerun(self, w, now):
        i = w.ids[0]
        sh = self.shots[i]
        sol, bat = w.sb.host(), w.bb.host()
        sh["sinfo"] = np.array([sol["status"], sol["n_moves"], sol["n_groups"], sol["n_steps"], 0, 0], np.uint32)
        sh["binfo"] = np.array([bat["status"], bat["n_batches"], bat["n_steps"], 0, 0], np.uint32)
        if self.keep:
            sh["out"] = (sol, bat)
        sh["t_done"] = time.perf_counter() if self.keep else now

    def drain(self, timeout_s=120.0):
        t0 = time.perf_counter()
        while any(self.waiting.values()) or self.inflight:
            self.pump()
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("server did not drain")

    # ---- results
    def result(self, i):
        """(solve, batch) of shot i as SolveBuffers.host / BatchBuffers.host give them
        (keep_results=True)."""
        return self.shots[i]["out"]

    def latencies_us(self, side=None):
        return np.array([(s["t_done"] - s["t_arrive"]) * 1e6 for s in self.shots
                         if s["t_done"] is not None and (side is None or self.class_of(s["shape"]) == side)])


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process: i.i.d. exponential gaps, seeded."""
    rng = np.random.default_rng(seed)
    n = int(rate_hz * duration_s * 1.3) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    return t[t < duration_s]


def serve_stream(server: Server, shapes, grids, arrivals, order):
    """Feed shots into ``server`` at their arrival times (seconds from the start) and pump until
    all are done.  ``order[k]`` is the index into shapes/grids of the k-th arrival.  Returns the
    wall time from the first arrival to the last completion."""
    t0 = time.perf_counter()
    server.t0 = t0
    k = 0
    n = len(arrivals)
    while k < n or any(server.waiting.values()) or server.inflight:
        now = time.perf_counter() - t0
        while k < n and arrivals[k] <= now:
            j = order[k]
            server.submit(shapes[j], grids[j], t_arrive=t0 + arrivals[k])
            k += 1
        server.pump()
    return time.perf_counter() - t0

"""CPU oracle for red-rec + batching (arXiv 2504.06182) — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It wraps ``liboracle.so`` (plain single-threaded C, built from
``rr_oracle.c`` by :func:`build`) with numpy-in / numpy-out helpers.  It shares no code with the
HIP library in ``paper_2504_06182_amd``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, INFEASIBLE, E_INVAL, E_CAPACITY, E_NOMEM, E_INTERNAL = 0, 1, -1, -2, -4, -5
LAMBDA_LINE_OR_COL, LAMBDA_ALONG, LAMBDA_NONE = 0, 1, 2


class Shape(C.Structure):
    _fields_ = [(n, C.c_uint16) for n in ("w", "h", "x0", "y0", "x1", "y1")]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_moves", C.c_uint32), ("n_groups", C.c_uint32),
                ("n_steps", C.c_uint32), ("need_moves", C.c_uint32), ("need_groups", C.c_uint32)]


class BatchInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_batches", C.c_uint32), ("n_steps", C.c_uint32),
                ("need_batches", C.c_uint32), ("need_steps", C.c_uint32)]


class Event(C.Structure):
    _fields_ = [("donor", C.c_int32), ("receiver", C.c_int32), ("kase", C.c_int32),
                ("k_bottom", C.c_int32), ("count", C.c_int32)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, single-threaded C)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.rr_oracle_solve.argtypes = [C.POINTER(Shape), P, P, C.c_uint32, P, C.c_uint32, P, C.POINTER(SolveInfo)]
        L.rr_oracle_solve.restype = C.c_int
        L.rr_oracle_solve_trace.argtypes = [C.POINTER(Shape), P, P, C.c_uint32, P, C.c_uint32, P,
                                            C.POINTER(SolveInfo), C.c_uint32, P, C.c_uint32,
                                            C.POINTER(C.c_uint32)]
        L.rr_oracle_solve_trace.restype = C.c_int
        L.rr_oracle_batch_moves.argtypes = [C.POINTER(Shape), P, P, C.POINTER(SolveInfo), C.c_uint32,
                                            P, C.c_uint32, P, C.c_uint32, C.POINTER(BatchInfo)]
        L.rr_oracle_batch_moves.restype = C.c_int
        L.rr_oracle_batch_moves_indexed.argtypes = L.rr_oracle_batch_moves.argtypes
        L.rr_oracle_batch_moves_indexed.restype = C.c_int
        L.rr_oracle_e1d_window.argtypes = [P, C.c_int, C.c_int, C.c_int]
        L.rr_oracle_e1d_window.restype = C.c_int
        L.rr_oracle_e1d_moves.argtypes = [P, C.c_int, C.c_int, C.c_int, P, P]
        L.rr_oracle_e1d_moves.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_shape(shape) -> Shape:
    w, h, x0, y0, x1, y1 = (int(v) for v in shape)
    return Shape(w, h, x0, y0, x1, y1)


def e1d_window(p, b: int, t: int) -> int:
    arr = np.ascontiguousarray(p, dtype=np.int32)
    return lib().rr_oracle_e1d_window(_ptr(arr), len(arr), int(b), int(t))


def e1d_moves(p, b: int, t: int):
    arr = np.ascontiguousarray(p, dtype=np.int32)
    src = np.zeros(max(t, 1), np.int32)
    dst = np.zeros(max(t, 1), np.int32)
    n = lib().rr_oracle_e1d_moves(_ptr(arr), len(arr), int(b), int(t), _ptr(src), _ptr(dst))
    if n < 0:
        raise ValueError("bad exact-1D arguments")
    return list(zip(src[:n].tolist(), dst[:n].tolist()))


REDREC_PARALLEL, REDREC_SERIAL, BIRD = 0, 1, 2


def solve(shape, occ, move_cap=None, group_cap=None, trace=False, serial=False, bird=False):
    """Run the oracle solve on packed rows ``occ`` (uint64[h][ws]).

    ``serial`` selects the serial order of Alg. 1 (donors solved after they donate) instead of
    the parallel one of §III.D; ``bird`` selects the bird algorithm (Alg. 2) instead of red-rec.
    Returns a dict: rc, status, moves (uint16[n][4] = sx,sy,dx,dy),
    group_off (uint32[g+1]), final (uint64[h][ws]), n_steps, need_moves, need_groups and, with
    ``trace``, events."""
    sh = make_shape(shape)
    occ = np.ascontiguousarray(occ, dtype=np.uint64)
    w, h, x0, y0, x1, y1 = (int(v) for v in shape)
    if move_cap is None:
        move_cap = 2 * (x1 - x0) * (y1 - y0)
    if group_cap is None:
        group_cap = (x1 - x0) + (y1 - y0)
    moves = np.zeros((max(move_cap, 1), 4), np.uint16)
    goff = np.zeros(group_cap + 1, np.uint32)
    final = np.zeros_like(occ)
    info = SolveInfo()
    out = {}
    algo = BIRD if bird else (REDREC_SERIAL if serial else REDREC_PARALLEL)
    if trace or algo:
        ev = (Event * (w + 1))()
        nev = C.c_uint32(0)
        rc = lib().rr_oracle_solve_trace(C.byref(sh), _ptr(occ), _ptr(moves), move_cap, _ptr(goff), group_cap,
                                         _ptr(final), C.byref(info), algo,
                                         C.cast(ev, C.c_void_p), w + 1, C.byref(nev))
        if trace:
            out["events"] = [(e.donor, e.receiver, e.kase, e.k_bottom, e.count)
                             for e in ev[:min(nev.value, w + 1)]]
    else:
        rc = lib().rr_oracle_solve(C.byref(sh), _ptr(occ), _ptr(moves), move_cap, _ptr(goff), group_cap,
                                   _ptr(final), C.byref(info))
    out.update(rc=rc, status=info.status, n_steps=info.n_steps, need_moves=info.need_moves,
               need_groups=info.need_groups, info=info)
    if rc == 0 and info.status == OK:
        out["moves"] = moves[:info.n_moves].copy()
        out["group_off"] = goff[:info.n_groups + 1].copy()
        out["final"] = final
    elif rc == 0 and info.status == INFEASIBLE:
        out["moves"] = np.zeros((0, 4), np.uint16)
        out["group_off"] = np.zeros(1, np.uint32)
        out["final"] = final
    return out


def batch(shape, moves, group_off, n_steps, status=OK, flags=LAMBDA_LINE_OR_COL, batch_cap=None, step_cap=None,
          indexed=False):
    """Run the oracle batching routine.  Returns rc, status, batch_off (uint32[nb+1]), steps.

    ``indexed`` selects the indexed form (reduced dependency graph, bucketed ready set), which
    gives the same results as the literal form and is the one that can run large grids."""
    sh = make_shape(shape)
    moves = np.ascontiguousarray(moves, dtype=np.uint16).reshape(-1, 4)
    goff = np.ascontiguousarray(group_off, dtype=np.uint32)
    si = SolveInfo(status, len(moves), max(len(goff) - 1, 0), int(n_steps), len(moves), max(len(goff) - 1, 0))
    if step_cap is None:
        step_cap = int(n_steps)
    if batch_cap is None:
        batch_cap = int(n_steps)
    boff = np.zeros(batch_cap + 1, np.uint32)
    steps = np.zeros(max(step_cap, 1), np.uint32)
    bi = BatchInfo()
    fn = lib().rr_oracle_batch_moves_indexed if indexed else lib().rr_oracle_batch_moves
    rc = fn(C.byref(sh), _ptr(moves) if len(moves) else None, _ptr(goff), C.byref(si), flags, _ptr(boff),
            batch_cap, _ptr(steps), step_cap, C.byref(bi))
    out = dict(rc=rc, status=bi.status, need_batches=bi.need_batches, need_steps=bi.need_steps)
    if rc == 0 and bi.status == OK:
        out["batch_off"] = boff[:bi.n_batches + 1].copy()
        out["steps"] = steps[:bi.n_steps].copy()
    return out


def solve_chain(n: int, occ_row, b: int, t: int):
    """Exact 1D on a chain of n traps (a 1 x n grid; bit row ``occ_row``) with the contiguous
    target [b, b+t): the exact-1D window and emission of §III.A (``rr_oracle_e1d_moves``) over
    the sorted token positions.  Returns the layout of :func:`solve` for that 1 x n grid:
    status, moves (uint16[k][4], rows 0), group_off (one group, or none), final, n_steps."""
    row = np.ascontiguousarray(occ_row, dtype=np.uint64).reshape(-1)
    bits = np.unpackbits(row.view(np.uint8), bitorder="little")[:n]
    p = np.nonzero(bits)[0].astype(np.int32)
    if len(p) < t:
        return dict(status=INFEASIBLE, moves=np.zeros((0, 4), np.uint16), group_off=np.zeros(1, np.uint32),
                    final=row.reshape(1, -1).copy(), n_steps=0)
    pairs = e1d_moves(p, b, t)
    moves = np.zeros((len(pairs), 4), np.uint16)
    for k, (s, d) in enumerate(pairs):
        moves[k] = (s, 0, d, 0)
    w = e1d_window(p, b, t)
    fin = bits.copy()
    fin[p[w:w + t]] = 0
    fin[b:b + t] = 1
    padded = np.zeros(row.size * 64, np.uint8)
    padded[:n] = fin
    final = np.packbits(padded, bitorder="little").view(np.uint64).reshape(1, -1)
    goff = np.array([0, len(pairs)] if pairs else [0], np.uint32)
    steps = int(sum(abs(int(s) - int(d)) for s, d in pairs))
    return dict(status=OK, moves=moves, group_off=goff, final=final, n_steps=steps)

"""Python binding of librr: red-rec solve and batching on MI355X (gfx950).

Argument marshalling only.  Every function here has the name of the C entry point it calls
(declared in ``include/rr.h``); device buffers are torch tensors (or raw device addresses) and
the stream is a torch stream (default: the current one).  No step of the method runs in Python.
If ``librr.so`` is missing or cannot be loaded, :func:`lib` raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librr.so")

RR_OK, RR_INFEASIBLE = 0, 1
RR_E_INVAL, RR_E_CAPACITY, RR_E_DEVICE, RR_E_NOMEM, RR_E_INTERNAL, RR_E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
RR_LAMBDA_LINE_OR_COL, RR_LAMBDA_ALONG, RR_LAMBDA_NONE = 0, 1, 2
RR_REDREC_PARALLEL, RR_REDREC_SERIAL, RR_BIRD = 0, 1, 2
RR_BATCH_GENERIC = 1 << 16
RR_MAX_SIDE = 1024
RR_LDS_SIDE = 256
RR_MAX_CHAIN = 65535
RR_NOALLOC_WORKSPACE_BYTES = 64 << 20
STATUS_NAMES = {0: "RR_OK", 1: "RR_INFEASIBLE", -1: "RR_E_INVAL", -2: "RR_E_CAPACITY", -3: "RR_E_DEVICE",
                -4: "RR_E_NOMEM", -5: "RR_E_INTERNAL", -6: "RR_E_UNSUPPORTED"}


class rr_shape(C.Structure):
    _fields_ = [(n, C.c_uint16) for n in ("w", "h", "x0", "y0", "x1", "y1")]


class rr_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_moves", C.c_uint32), ("n_groups", C.c_uint32),
                ("n_steps", C.c_uint32), ("need_moves", C.c_uint32), ("need_groups", C.c_uint32)]


class rr_batch_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_batches", C.c_uint32), ("n_steps", C.c_uint32),
                ("need_batches", C.c_uint32), ("need_steps", C.c_uint32)]


class rr_desc(C.Structure):
    _fields_ = [("shape", rr_shape), ("pad0", C.c_uint16), ("pad1", C.c_uint16),
                ("move_cap", C.c_uint32), ("group_cap", C.c_uint32), ("step_cap", C.c_uint32),
                ("batch_cap", C.c_uint32), ("occ_off", C.c_uint64), ("move_off", C.c_uint64),
                ("group_off", C.c_uint64), ("step_off", C.c_uint64), ("batch_off", C.c_uint64),
                ("ws_off", C.c_uint64)]


assert C.sizeof(rr_desc) == 80 and C.sizeof(rr_shape) == 12


class RRError(RuntimeError):
    pass


_lib = None
_P = C.c_void_p
_U32 = C.c_uint32
_SZ = C.c_size_t

_SIGS = {
    "rr_version": ([], C.c_char_p),
    "rr_solve_workspace_bytes": ([rr_shape], _SZ),
    "rr_solve": ([rr_shape, _P, _P, _U32, _P, _U32, _P, _P, _U32, _P, _SZ, _P], C.c_int),
    "rr_batch_workspace_bytes": ([rr_shape, _U32, _U32], _SZ),
    "rr_batch_moves": ([rr_shape, _P, _P, _P, _U32, _U32, _P, _U32, _P, _U32, _P, _P, _SZ, _P], C.c_int),
    "rr_batch_moves_noalloc": ([rr_shape, _P, _P, _P, _U32, _U32, _P, _U32, _P, _U32, _P, _P], C.c_int),
    "rr_solve_chains_workspace_bytes": ([_U32, _U32], _SZ),
    "rr_solve_chains": ([_U32, _P, _U32, _P, _P, _P, _P, _P, _P, _SZ, _P], C.c_int),
    "rr_solve_many": ([_U32, _P, _U32, _U32, _P, _P, _P, _P, _P, _U32, _P, _SZ, _P], C.c_int),
    "rr_batch_moves_many": ([_U32, _P, _U32, _U32, _P, _P, _P, _U32, _P, _P, _P, _P, _SZ, _P], C.c_int),
    "rr_plan_many": ([_U32, _P, _P, C.c_uint64, C.c_uint64, C.c_uint64, _P, _P], C.c_int),
    "rr_batch_moves_many_staged": ([_U32, _P, _U32, _U32, _P, _P, _P, _U32, _P, _P, _P, _P, _SZ, _P, _P, _P],
                                   C.c_int),
}


def lib():
    """The loaded librr.so (raises if it was not built or cannot load)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RRError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _shape(s) -> rr_shape:
    if isinstance(s, rr_shape):
        return s
    w, h, x0, y0, x1, y1 = (int(v) for v in s)
    return rr_shape(w, h, x0, y0, x1, y1)


def _check(rc: int, what: str) -> int:
    if rc != RR_OK:
        raise RRError(f"{what} returned {STATUS_NAMES.get(rc, rc)}")
    return rc


def rr_version() -> str:
    return lib().rr_version().decode()


def rr_solve_workspace_bytes(shape) -> int:
    return int(lib().rr_solve_workspace_bytes(_shape(shape)))


def rr_batch_workspace_bytes(shape, move_cap: int, step_cap: int) -> int:
    return int(lib().rr_batch_workspace_bytes(_shape(shape), int(move_cap), int(step_cap)))


def rr_solve(shape, occ, moves, move_cap, group_off, group_cap, final_occ, info, flags=RR_REDREC_PARALLEL,
             workspace=None, workspace_bytes=0, stream=None, check=True) -> int:
    rc = lib().rr_solve(_shape(shape), _ptr(occ), _ptr(moves), int(move_cap), _ptr(group_off), int(group_cap),
                        _ptr(final_occ), _ptr(info), int(flags), _ptr(workspace), int(workspace_bytes),
                        _stream(stream))
    return _check(rc, "rr_solve") if check else rc


def rr_batch_moves(shape, moves, group_off, sinfo, move_cap, flags, batch_off, batch_cap, steps, step_cap,
                   binfo, workspace, workspace_bytes, stream=None, check=True) -> int:
    rc = lib().rr_batch_moves(_shape(shape), _ptr(moves), _ptr(group_off), _ptr(sinfo), int(move_cap),
                              int(flags), _ptr(batch_off), int(batch_cap), _ptr(steps), int(step_cap),
                              _ptr(binfo), _ptr(workspace), int(workspace_bytes), _stream(stream))
    return _check(rc, "rr_batch_moves") if check else rc


def rr_batch_moves_noalloc(shape, moves, group_off, sinfo, move_cap, flags, batch_off, batch_cap, steps, step_cap,
                           binfo, stream=None, check=True) -> int:
    rc = lib().rr_batch_moves_noalloc(_shape(shape), _ptr(moves), _ptr(group_off), _ptr(sinfo), int(move_cap),
                                      int(flags), _ptr(batch_off), int(batch_cap), _ptr(steps), int(step_cap),
                                      _ptr(binfo), _stream(stream))
    return _check(rc, "rr_batch_moves_noalloc") if check else rc


def rr_solve_chains_workspace_bytes(n: int, max_len: int) -> int:
    return int(lib().rr_solve_chains_workspace_bytes(int(n), int(max_len)))


def rr_solve_chains(n, desc, max_len, occ_arena, move_arena, group_arena, final_arena, infos, workspace=None,
                    workspace_bytes=0, stream=None, check=True) -> int:
    rc = lib().rr_solve_chains(int(n), _ptr(desc), int(max_len), _ptr(occ_arena), _ptr(move_arena),
                               _ptr(group_arena), _ptr(final_arena), _ptr(infos), _ptr(workspace),
                               int(workspace_bytes), _stream(stream))
    return _check(rc, "rr_solve_chains") if check else rc


def rr_solve_many(n, desc, max_w, max_h, occ_arena, move_arena, group_arena, final_arena, infos,
                  flags=RR_REDREC_PARALLEL, workspace=None, workspace_bytes=0, stream=None, check=True) -> int:
    rc = lib().rr_solve_many(int(n), _ptr(desc), int(max_w), int(max_h), _ptr(occ_arena), _ptr(move_arena),
                             _ptr(group_arena), _ptr(final_arena), _ptr(infos), int(flags), _ptr(workspace),
                             int(workspace_bytes), _stream(stream))
    return _check(rc, "rr_solve_many") if check else rc


def rr_batch_moves_many(n, desc, max_w, max_h, move_arena, group_arena, sinfos, flags, batch_arena,
                        step_arena, binfos, workspace, workspace_bytes, stream=None, check=True) -> int:
    rc = lib().rr_batch_moves_many(int(n), _ptr(desc), int(max_w), int(max_h), _ptr(move_arena),
                                   _ptr(group_arena), _ptr(sinfos), int(flags), _ptr(batch_arena),
                                   _ptr(step_arena), _ptr(binfos), _ptr(workspace), int(workspace_bytes),
                                   _stream(stream))
    return _check(rc, "rr_batch_moves_many") if check else rc


def _event(e):
    """Raw hipEvent_t of a torch.cuda.Event (created on first use), an int, or None."""
    if e is None or isinstance(e, int):
        return e
    if not e.cuda_event:
        e.record()                         # torch creates the event lazily
    return e.cuda_event


def rr_batch_moves_many_staged(n, desc, max_w, max_h, move_arena, group_arena, sinfos, flags, batch_arena,
                               step_arena, binfos, workspace, workspace_bytes, stream=None, graph_done_event=None,
                               loop_done_event=None, check=True) -> int:
    rc = lib().rr_batch_moves_many_staged(int(n), _ptr(desc), int(max_w), int(max_h), _ptr(move_arena),
                                          _ptr(group_arena), _ptr(sinfos), int(flags), _ptr(batch_arena),
                                          _ptr(step_arena), _ptr(binfos), _ptr(workspace), int(workspace_bytes),
                                          _stream(stream), _event(graph_done_event), _event(loop_done_event))
    return _check(rc, "rr_batch_moves_many_staged") if check else rc


def rr_plan_many(n, desc, infos, step_pool, batch_pool, ws_pool_bytes, totals=None, stream=None, check=True) -> int:
    rc = lib().rr_plan_many(int(n), _ptr(desc), _ptr(infos), int(step_pool), int(batch_pool), int(ws_pool_bytes),
                            _ptr(totals), _stream(stream))
    return _check(rc, "rr_plan_many") if check else rc


__all__ = [n for n in dir() if n.startswith("rr_") or n.startswith("RR_")] + ["lib", "RRError", "LIB_PATH"]

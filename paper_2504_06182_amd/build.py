"""Build librr.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("rr_batch_loop6.hip", "rr_batch_loop5.hip", "rr_batch_loop2.hip",
                                                   "rr_batch_wide.hip", "rr_batch.hip", "rr_solve.hip",
                                                   "rr_chain.hip")]
HEADERS = [os.path.join(HERE, "csrc", h) for h in ("rr_device.hpp", "rr_batch_generic.hpp", "rr_batch_graph.hpp",
                                                   "rr_batch_loop.hpp", "rr_batch_common.hpp",
                                                   "rr_batch_loop_kernels.hpp", "rr_batch_wide.hpp")] + [os.path.join(ROOT, "include", "rr.h")]
LIB = os.path.join(HERE, "librr.so")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build librr.so")
    return p


OBJ_DIR = os.path.join(ROOT, "_build")


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every HIP source for gfx950 into paper_2504_06182_amd/librr.so.

    Each source is compiled to an object in its own hipcc process (in parallel), then linked.
    By default every source is recompiled; ``incremental`` reuses an object in ``_build/`` that
    is newer than its source and every header."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = [os.path.join(OBJ_DIR, os.path.basename(src) + ".o") for src in SOURCES]
    newest_header = max(os.path.getmtime(h) for h in HEADERS)
    procs = []
    for src, obj in zip(SOURCES, objs):
        if (incremental and os.path.exists(obj)
                and os.path.getmtime(obj) > max(os.path.getmtime(src), newest_header)):
            continue
        tmp = obj + ".tmp%d" % os.getpid()
        procs.append((subprocess.Popen([hipcc(), *flags, "-c", src, "-o", tmp], stdout=subprocess.PIPE,
                                       stderr=subprocess.PIPE, text=True), tmp, obj))
    errs = []
    for p, tmp, obj in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            errs.append(out + err)
            continue
        os.replace(tmp, obj)
        if verbose and err:
            print(err)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))

"""Seeded synthetic trap-array loadings shared by the oracle-side tests and the GPU side.

This module holds no part of the reconfiguration method: it only draws occupancy grids and
packs them into the bit-row layout the C interfaces take.  Both the CPU oracle and the HIP
library consume the very same bytes produced here.

Random source: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based hash of a 64-bit key.

* cell key      = seed << 48  ^  shot << 24  ^  y << 12  ^  x          (x, y < 4096)
* shot-level key = (seed | 0x8000) << 48  ^  shot << 24  ^  j          (j = draw index)
* a cell is loaded iff (splitmix64(key) >> 32) < floor(p * 2**32)      (i.i.d. Bernoulli(p))
* fixed-count loading (exactly n atoms, uniform over the n-subsets of traps): the n cells with
  the smallest splitmix64(cell key), ties broken by cell index y*W + x

Layout of a packed grid: ``uint64[H][ws]`` with ``ws = ceil(W/64)``; bit ``x % 64`` of word
``y*ws + x//64`` is trap (x, y); columns run left to right, rows bottom to top; padding bits
beyond W are zero.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "splitmix64", "bernoulli_grid", "fixed_count_grid", "pack_rows", "unpack_rows", "words_per_row",
    "centred_target", "config_shots", "CONFIGS", "uniform01",
]

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(key):
    """SplitMix64 finaliser applied to ``key + golden gamma`` (vectorised, wraps mod 2**64)."""
    with np.errstate(over="ignore"):
        z = np.asarray(key, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def words_per_row(w: int) -> int:
    return (int(w) + 63) // 64


def bernoulli_grid(seed: int, shot: int, w: int, h: int, p: float) -> np.ndarray:
    """Dense ``uint8[h][w]`` occupancy: cell (x, y) loaded with probability p."""
    ys, xs = np.meshgrid(np.arange(h, dtype=np.uint64), np.arange(w, dtype=np.uint64), indexing="ij")
    key = (np.uint64(seed) << np.uint64(48)) ^ (np.uint64(shot) << np.uint64(24)) ^ (ys << np.uint64(12)) ^ xs
    thr = np.uint64(int(p * 4294967296.0))
    return ((splitmix64(key) >> np.uint64(32)) < thr).astype(np.uint8)


def fixed_count_grid(seed: int, shot: int, w: int, h: int, n: int) -> np.ndarray:
    """Dense ``uint8[h][w]`` occupancy with exactly n loaded cells, drawn uniformly: the n cells
    of smallest hash (cell keys as for bernoulli_grid), ties broken by cell index."""
    if not 0 <= n <= w * h:
        raise ValueError("atom count outside 0..W*H")
    ys, xs = np.meshgrid(np.arange(h, dtype=np.uint64), np.arange(w, dtype=np.uint64), indexing="ij")
    key = (np.uint64(seed) << np.uint64(48)) ^ (np.uint64(shot) << np.uint64(24)) ^ (ys << np.uint64(12)) ^ xs
    order = np.argsort(splitmix64(key).reshape(-1), kind="stable")
    dense = np.zeros(w * h, dtype=np.uint8)
    dense[order[:n]] = 1
    return dense.reshape(h, w)


def uniform01(seed: int, shot: int, j: int) -> float:
    """Shot-level uniform draw in [0, 1) (top 32 bits of the hash)."""
    key = (np.uint64(seed | 0x8000) << np.uint64(48)) ^ (np.uint64(shot) << np.uint64(24)) ^ np.uint64(j)
    return float(splitmix64(key) >> np.uint64(32)) / 4294967296.0


def pack_rows(dense: np.ndarray) -> np.ndarray:
    """``uint8[h][w]`` -> ``uint64[h][ws]`` bit rows (bit x%64 of word x//64)."""
    dense = np.asarray(dense, dtype=np.uint8)
    h, w = dense.shape
    ws = words_per_row(w)
    padded = np.zeros((h, ws * 64), dtype=np.uint8)
    padded[:, :w] = dense
    bits = padded.reshape(h, ws, 64).astype(np.uint64)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    return (bits * weights).sum(axis=2, dtype=np.uint64).astype(np.uint64)


def unpack_rows(packed: np.ndarray, w: int) -> np.ndarray:
    packed = np.asarray(packed, dtype=np.uint64)
    h, ws = packed.shape
    shifts = np.arange(64, dtype=np.uint64)
    bits = (packed[:, :, None] >> shifts) & np.uint64(1)
    return bits.reshape(h, ws * 64)[:, :w].astype(np.uint8)


def centred_target(n_w: int, n_h: int, s_w: int, s_h: int):
    """Centred target rectangle (x0, y0, x1, y1) with origin floor((n - s)/2)."""
    x0 = (n_w - s_w) // 2
    y0 = (n_h - s_h) // 2
    return (x0, y0, x0 + s_w, y0 + s_h)


# Workload recipes.  Each shot is (w, h, x0, y0, x1, y1, p, seed, shot_index).
MIX_SIDES = (32, 48, 64, 96, 128, 192, 256)

CONFIGS = {
    "single32": dict(n=1, side=32, s=16, p=0.5, seed=1),
    "single128": dict(n=1, side=128, s=90, p=0.6, seed=2),
    "batch64": dict(n=8192, side=64, s=44, p=0.55, seed=3),
    "mixed": dict(n=4096, sides=MIX_SIDES, frac=0.7, p_lo=0.5, p_hi=0.65, seed=4),
    "big1024": dict(n=1, side=1024, s=780, p=0.6, seed=5),
    # the paper's benchmark geometry: N_tx = 32 columns, N_ty = ceil(N_tx / 0.6) = 54 rows, a
    # full-width 32 x 32 target (centre-compact), exactly floor(0.6 * 32 * 54) = 1036 atoms
    "paper32": dict(n=1000, w=32, h=54, sw=32, sh=32, count=1036, seed=6),
    # the paper's chain geometry: a centre-compact target of N_t / 2 traps in a chain of N_t
    # traps, exactly floor(0.6 * N_t) atoms; N_t = 1024 as timed there, and the longest chain
    # the move format holds (coordinates are 16-bit); chains are 1 x N grids (x < 2**24 keeps
    # cell keys distinct)
    "chain1024": dict(n=1000, w=1024, h=1, sw=512, sh=1, count=614, seed=7),
    "chain65535": dict(n=16, w=65535, h=1, sw=32767, sh=1, count=39321, seed=8),
}


def config_shots(name: str, n: int | None = None, first: int = 0):
    """List of shot descriptors for a named workload (optionally a sub-range of shots)."""
    c = CONFIGS[name]
    total = c["n"] if n is None else n
    shots = []
    for i in range(first, first + total):
        if "count" in c:
            x0, y0, x1, y1 = centred_target(c["w"], c["h"], c["sw"], c["sh"])
            shots.append(dict(w=c["w"], h=c["h"], x0=x0, y0=y0, x1=x1, y1=y1, p=None, count=c["count"],
                              seed=c["seed"], shot=i))
            continue
        if name == "mixed":
            side = c["sides"][int(uniform01(c["seed"], i, 0) * 4294967296.0) % len(c["sides"])]
            p = c["p_lo"] + (c["p_hi"] - c["p_lo"]) * uniform01(c["seed"], i, 1)
            s = (7 * side) // 10
        else:
            side, s, p = c["side"], c["s"], c["p"]
        x0, y0, x1, y1 = centred_target(side, side, s, s)
        shots.append(dict(w=side, h=side, x0=x0, y0=y0, x1=x1, y1=y1, p=p, seed=c["seed"], shot=i))
    return shots


def shot_grid(desc) -> np.ndarray:
    """Packed bit rows for one shot descriptor."""
    if desc.get("count") is not None:
        return pack_rows(fixed_count_grid(desc["seed"], desc["shot"], desc["w"], desc["h"], desc["count"]))
    return pack_rows(bernoulli_grid(desc["seed"], desc["shot"], desc["w"], desc["h"], desc["p"]))

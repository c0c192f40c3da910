"""Vectorised numpy Jones-Plassmann colouring (Sec. 2.2, Algorithm 3) -- TEST
INFRASTRUCTURE ONLY.

An independent re-implementation of jp_oracle.c used to cross-check it: whole-array
operations over the arc list instead of per-vertex loops, and its own SplitMix64
(Steele, Lea and Flood, OOPSLA 2014).  Same readings: only neighbours still
uncoloured compete, ties exclude both endpoints, self-loops are ignored, and the
priority of v in round c is SplitMix64 output number c * 2^32 + v.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_np(seed: int, k: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs number k (uint64 array) for one seed."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & (2**64 - 1)) + np.asarray(k, dtype=np.uint64) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def jp_numpy(n: int, rowptr, colidx, seed: int = 0, max_rounds: int = 1 << 20):
    """Returns (colors 0-based, ncolors, rounds, wsize list)."""
    rp = np.asarray(rowptr, dtype=np.int64)
    ci = np.asarray(colidx, dtype=np.int64)
    if n == 0:
        return np.zeros(0, dtype=np.int32), 0, 0, []
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    keep = src != ci
    src, dst = src[keep], ci[keep]
    color = np.zeros(n, dtype=np.int64)
    ids = np.arange(n, dtype=np.uint64)
    wsize = []
    c = 0
    while (color == 0).any():
        c += 1
        if c > max_rounds:
            raise RuntimeError("JP did not finish")
        inW = color == 0
        wsize.append(int(inW.sum()))
        r = splitmix64_np(seed, (np.uint64(c) << np.uint64(32)) + ids)
        live = inW[src] & inW[dst]
        blocked = np.zeros(n, dtype=bool)
        blk = live & (r[src] <= r[dst])
        blocked[src[blk]] = True
        S = inW & ~blocked
        color[S] = c
    return (color - 1).astype(np.int32), c, c, wsize

"""Independent vectorised SGR oracle -- TEST INFRASTRUCTURE ONLY.

A second implementation of the same rounds as sgr_oracle.c (Sec. 3.1, Algorithm
Data-GC with FirstFit and ConflictResolve of Sec. 3), written set-at-a-time over the
arc list instead of vertex-at-a-time, so that a slip in either one shows up as a
disagreement.  Same readings: FirstFit reads the previous round's snapshot only; the
higher id of a same-colour adjacent pair is requeued and its colour cleared.
"""
from __future__ import annotations

import numpy as np


def _mex_per_vertex(verts: np.ndarray, owner: np.ndarray, col: np.ndarray) -> np.ndarray:
    """For each vertex in `verts`, the smallest positive integer not among the colours
    `col[k]` with `owner[k]` equal to it."""
    out = np.ones(len(verts), dtype=np.int64)
    if len(owner) == 0:
        return out
    pos = np.searchsorted(verts, owner)
    key = np.unique(pos * (np.int64(col.max()) + 2) + col)     # distinct (vertex, colour)
    base = np.int64(col.max()) + 2
    p = key // base
    c = key - p * base
    # rank of each colour within its vertex group, 1-based
    first = np.r_[True, p[1:] != p[:-1]]
    start = np.maximum.accumulate(np.where(first, np.arange(len(p)), 0))
    rank = np.arange(len(p)) - start + 1
    # the mex is the first rank whose colour differs from the rank; else count + 1
    gap = c != rank
    cnt = np.bincount(p, minlength=len(verts))
    mex = cnt + 1
    gp = p[gap]
    gr = rank[gap]
    # first gap per vertex: gaps are in increasing rank order inside each group
    firstgap = np.r_[True, gp[1:] != gp[:-1]] if len(gp) else np.zeros(0, bool)
    mex[gp[firstgap]] = gr[firstgap]
    out[:] = mex
    return out


def sgr_numpy(n: int, rowptr, colidx, trace: list | None = None, rule: int = 0):
    """Return (colors 0-based int32[n], ncolors, rounds, wsize list).

    If `trace` is a list, one (W, C[W] 1-based, losers) tuple per round is appended.
    rule 0: the higher id of a same-colour adjacent pair is requeued; rule 1: the
    smaller degree (row length) is requeued, the higher id on equal degree."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    if n == 0:
        return np.zeros(0, np.int32), 0, 0, []
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    dst = colidx
    keep = src != dst
    src, dst = src[keep], dst[keep]
    rowlen = np.diff(rowptr)
    if rule == 0:
        beats = dst < src                       # arc (src, dst): dst requeues src on a tie of colours
    else:
        beats = (rowlen[dst] > rowlen[src]) | ((rowlen[dst] == rowlen[src]) & (dst < src))
    S = np.zeros(n, dtype=np.int64)
    C = np.zeros(n, dtype=np.int64)
    inW = np.ones(n, dtype=bool)
    rounds = 0
    wsize = []
    while inW.any():
        rounds += 1
        W = np.flatnonzero(inW)
        wsize.append(len(W))
        # FirstFit against the snapshot: colours of coloured neighbours are forbidden
        sel = inW[src] & (S[dst] > 0)
        C[W] = _mex_per_vertex(W, src[sel], S[dst[sel]])
        # pairwise conflict test over arcs to lower ids
        bad = inW[src] & beats & (C[src] == C[dst])
        lose = np.zeros(n, dtype=bool)
        lose[src[bad]] = True
        win = inW & ~lose
        if trace is not None:
            trace.append((W.tolist(), C[W].tolist(), np.flatnonzero(lose).tolist()))
        S[win] = C[win]
        S[lose] = 0
        inW = lose
    return (S - 1).astype(np.int32), int(S.max()), rounds, wsize

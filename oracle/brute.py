"""Exhaustive colouring numbers of tiny graphs -- TEST INFRASTRUCTURE ONLY.

chromatic(G): the least k admitting a proper k-colouring (backtracking search).
grundy(G):    the most colours sequential greedy (Sec. 2.1, Algorithm 1) can use over
              all n! vertex orders (exhaustive over permutations, vectorised).
Every greedy/first-fit colouring lies between the two, which pins any oracle output.
"""
from __future__ import annotations

import itertools

import numpy as np


def _adj(n, rowptr, colidx):
    adj = [set() for _ in range(n)]
    for v in range(n):
        for e in range(int(rowptr[v]), int(rowptr[v + 1])):
            w = int(colidx[e])
            if w != v:
                adj[v].add(w)
    return adj


def chromatic(n: int, rowptr, colidx) -> int:
    if n == 0:
        return 0
    adj = _adj(n, rowptr, colidx)
    order = sorted(range(n), key=lambda v: -len(adj[v]))

    def colorable(k: int) -> bool:
        col = [-1] * n

        def go(i: int) -> bool:
            if i == n:
                return True
            v = order[i]
            used = {col[w] for w in adj[v] if col[w] >= 0}
            for c in range(k):
                if c not in used:
                    col[v] = c
                    if go(i + 1):
                        return True
                    col[v] = -1
            return False

        return go(0)

    k = 1
    while not colorable(k):
        k += 1
    return k


def grundy(n: int, rowptr, colidx) -> int:
    """Maximum over all vertex orders of the number of colours greedy uses (n <= 8)."""
    if n == 0:
        return 0
    A = np.zeros((n, n), dtype=bool)
    for v, nb in enumerate(_adj(n, rowptr, colidx)):
        for w in nb:
            A[v, w] = True
    perms = np.array(list(itertools.permutations(range(n))), dtype=np.int64)
    P = len(perms)
    col = np.zeros((P, n), dtype=np.int64)          # 0 = uncoloured
    rows = np.arange(P)
    for i in range(n):
        v = perms[:, i]
        # forbidden[p, c] for colours 1..n
        nbcol = np.where(A[v], col, 0)              # (P, n) colours of v's neighbours
        forb = np.zeros((P, n + 2), dtype=bool)
        np.put_along_axis(forb, nbcol, True, axis=1)
        forb[:, 0] = True
        c = np.argmin(forb, axis=1)                 # first False = smallest free colour
        col[rows, v] = c
    return int(col.max(axis=1).max())

"""The pins reject plausible mistakes.

A small pure-Python round loop with switches plants each mistake (on the CPU): the
lower id requeued instead of the higher one, a requeued vertex keeping its tentative
colour instead of having it cleared (Sec. 3.1 "colour clearing"), FirstFit reading
colours written earlier in the same round, and a conflict test that ignores a lower
neighbour which itself lost.  Each mutant must fail at least one pin used for the
oracle: the hand-worked traces, the K_n / cycle closed forms or the Grundy property.
"""
import os

import pytest

from paper_1606_06025_amd import graphs as gg
from tests.test_oracle_pins import _parse_trace


def _sgr_variant(n, rowptr, colidx, requeue="higher", clear=True, reads="snapshot",
                 pairwise=True):
    adj = [[int(w) for w in colidx[rowptr[v]:rowptr[v + 1]] if w != v] for v in range(n)]
    S = [0] * n
    C = [0] * n
    W = list(range(n))
    rounds = 0
    while W and rounds < 4 * n + 4:
        rounds += 1
        inW = set(W)
        for v in W:
            src = C if reads == "current" else S
            used = {src[w] for w in adj[v] if (reads != "current" or w not in inW or w < v)}
            c = 1
            while c in used:
                c += 1
            C[v] = c
            if reads == "current":
                S[v] = c
        lose = set()
        for v in (sorted(W) if not pairwise else W):
            for w in adj[v]:
                if w in inW and C[w] == C[v]:
                    if (requeue == "higher" and w < v) or (requeue == "lower" and w > v):
                        if pairwise or w not in lose:
                            lose.add(v)
                            break
        for v in W:
            if v in lose:
                S[v] = 0 if clear else C[v]
            else:
                S[v] = C[v]
        W = [v for v in W if v in lose]
    return [s - 1 for s in S], rounds


def _passes_pins(**kw):
    for fname in ("sgr_c5.txt", "sgr_c7.txt"):
        rec = _parse_trace(fname)
        g = gg.from_edges(rec["n"], rec["edges"])
        col, r = _sgr_variant(g.n, g.rowptr, g.colidx, **kw)
        if [c + 1 for c in col] != rec["final"] or r != len(rec["rounds"]):
            return False
    for n in (6, 8, 10):
        g = gg.cycle(n)
        col, _ = _sgr_variant(g.n, g.rowptr, g.colidx, **kw)
        if max(col) + 1 != 2:
            return False
    g = gg.complete(7)
    col, r = _sgr_variant(g.n, g.rowptr, g.colidx, **kw)
    if col != list(range(7)) or r != 7:
        return False
    return True


def test_unmutated_variant_passes():
    assert _passes_pins()


@pytest.mark.parametrize("kw", [dict(requeue="lower"), dict(clear=False),
                                dict(reads="current"), dict(pairwise=False)])
def test_mutant_is_caught(kw):
    assert not _passes_pins(**kw)

"""Pins of the oracles for the two other colouring methods of the paper.

Jones-Plassmann (Sec. 2.2, Algorithm 3), oracle/jp_oracle.c and oracle/jp_numpy.py:
  * the priority generator reproduces published SplitMix64 outputs (tests/golden);
  * closed forms: an edgeless graph takes colour 1 in one round; K_n needs n rounds
    (exactly one vertex of a clique can beat all others); a single edge gives its
    endpoint of larger round-1 priority colour 1;
  * a round-by-round certificate that determines the JP colouring uniquely: vertex v
    has colour c iff in round c its priority beats every neighbour still uncoloured,
    and in every earlier round some such neighbour blocked it;
  * structure fixed by Algorithm 3: every colour class is a non-empty independent
    set and the number of colours equals the number of rounds;
  * an independent vectorised implementation, and planted mistakes the pins reject.

Topology-driven SGR (Sec. 3.1, Algorithm Topo-GC), oracle_sgr_topo: the worklist of
the data-driven algorithm is the set of uncoloured vertices, so both must give the
same colouring in the same rounds; checked on all 5-vertex graphs, the hand traces
and random graphs, with every round visiting all n vertices.
"""
import itertools
import os

import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _vectors():
    out = []
    for line in open(os.path.join(GOLDEN, "splitmix64.txt")):
        if line.strip() and not line.startswith("#"):
            s, k, v = line.split()
            out.append((int(s), int(k), int(v)))
    return out


def test_splitmix64_published_outputs(oracle_mod):
    vec = _vectors()
    assert len(vec) == 5
    for seed, k, val in vec:
        assert oracle_mod.splitmix64(seed, k) == val
    from oracle.jp_numpy import splitmix64_np
    got = splitmix64_np(1234567, np.array([k for _, k, _ in vec], dtype=np.uint64))
    assert [int(x) for x in got] == [v for _, _, v in vec]


def test_jp_priority_is_the_documented_output_number(oracle_mod):
    for seed in (0, 7, 2**63 + 5):
        for c, v in ((1, 0), (1, 5), (3, 1000), (70000, 2**31 - 1)):
            assert oracle_mod.jp_priority(seed, c, v) == oracle_mod.splitmix64(seed, (c << 32) + v)


def test_jp_priorities_of_one_round_are_distinct(oracle_mod):
    # seed + k * gamma (gamma odd) and the output function are both bijections on
    # 64-bit words, so no two vertices of a round can tie
    from oracle.jp_numpy import splitmix64_np
    for seed, c in ((0, 1), (5, 2), (2**64 - 1, 77)):
        ks = (np.uint64(c) << np.uint64(32)) + np.arange(200000, dtype=np.uint64)
        pr = splitmix64_np(seed, ks)
        assert np.unique(pr).size == pr.size


def _check_certificate(oracle_mod, g, seed, colors):
    """Every vertex v with 1-based colour c_v: in round c_v its priority beats every
    neighbour w != v with c_w >= c_v, and in each round c < c_v some neighbour w with
    c_w >= c has a priority >= v's."""
    col = np.asarray(colors, dtype=np.int64) + 1
    rp, ci = g.rowptr, g.colidx
    for v in range(g.n):
        nb = [int(w) for w in ci[rp[v]:rp[v + 1]] if w != v]
        for c in range(1, col[v] + 1):
            rv = oracle_mod.jp_priority(seed, c, v)
            live = [w for w in nb if col[w] >= c]
            wins = all(rv > oracle_mod.jp_priority(seed, c, w) for w in live)
            if wins != (c == col[v]):
                return False
    return True


def _structure(g, res):
    col = res.colors.astype(np.int64)
    assert res.ncolors == res.rounds
    assert col.min() >= 0 and col.max() == res.ncolors - 1
    assert set(col.tolist()) == set(range(res.ncolors))        # no empty class
    src = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    keep = src != g.colidx
    assert not np.any(col[src[keep]] == col[g.colidx[keep]])    # independent classes
    # |W_c| = vertices of colour >= c
    ws = [int((col >= c).sum()) for c in range(res.rounds)]
    assert res.wsize.tolist() == ws


def test_jp_edgeless_and_empty(oracle_mod):
    res = oracle_mod.jp(0, np.zeros(1, np.int32), np.zeros(0, np.int32), seed=3)
    assert res.ncolors == 0 and res.rounds == 0
    g = gg.edgeless(9)
    res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=3)
    assert res.colors.tolist() == [0] * 9 and res.rounds == 1


@pytest.mark.parametrize("n", [1, 2, 3, 6, 17])
@pytest.mark.parametrize("seed", [0, 1, 99])
def test_jp_clique_one_vertex_per_round(oracle_mod, n, seed):
    g = gg.complete(n)
    res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=seed)
    assert res.rounds == n and sorted(res.colors.tolist()) == list(range(n))
    # the vertex of colour c is the priority maximum of round c among the rest
    left = set(range(n))
    for c in range(1, n + 1):
        best = max(left, key=lambda v: oracle_mod.jp_priority(seed, c, v))
        assert res.colors[best] == c - 1
        left.remove(best)


@pytest.mark.parametrize("seed", range(8))
def test_jp_single_edge(oracle_mod, seed):
    g = gg.from_edges(2, [(0, 1)])
    res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=seed)
    first = 0 if oracle_mod.jp_priority(seed, 1, 0) > oracle_mod.jp_priority(seed, 1, 1) else 1
    assert res.colors[first] == 0 and res.colors[1 - first] == 1 and res.rounds == 2


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield gg.from_edges(n, [p for i, p in enumerate(pairs) if mask >> i & 1])


def test_jp_certificate_all_5_vertex_graphs(oracle_mod):
    for i, g in enumerate(_all_graphs(5)):
        seed = i * 7919
        res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=seed)
        _structure(g, res)
        assert _check_certificate(oracle_mod, g, seed, res.colors), i


@pytest.mark.parametrize("seed", [0, 5, 12345])
def test_jp_random_graphs_certificate_and_numpy(oracle_mod, seed):
    for n, m, s in ((40, 120, 1), (200, 1500, 2), (500, 500, 3)):
        g = gg.erdos_renyi(n, m, s)
        res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=seed)
        _structure(g, res)
        assert _check_certificate(oracle_mod, g, seed, res.colors)
        c2, nc2, r2, ws2 = oracle_mod.jp_numpy(g.n, g.rowptr, g.colidx, seed=seed)
        assert (c2 == res.colors).all() and nc2 == res.ncolors and ws2 == res.wsize.tolist()


def test_jp_larger_cross_check_and_quality_gap(oracle_mod):
    g = gg.erdos_renyi(20000, 160000, 4)
    res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=1)
    c2, nc2, _, _ = oracle_mod.jp_numpy(g.n, g.rowptr, g.colidx, seed=1)
    assert (c2 == res.colors).all() and nc2 == res.ncolors
    assert res.arcs.tolist()[0] == int(g.rowptr[-1])
    # the independent-set method needs more colours than speculative greedy (Sec. 2.2)
    sgr = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    assert res.ncolors > sgr.ncolors


def test_jp_self_loops_and_row_order_do_not_matter(oracle_mod):
    g = gg.erdos_renyi(300, 2000, 9)
    base = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=4).colors
    arcs = [(v, int(w)) for v in range(g.n) for w in g.colidx[g.rowptr[v]:g.rowptr[v + 1]]]
    arcs += [(v, v) for v in range(0, g.n, 3)]
    rng = np.random.default_rng(0)
    rng.shuffle(arcs)
    rp = np.zeros(g.n + 1, np.int64)
    for v, _ in arcs:
        rp[v + 1] += 1
    rp = np.cumsum(rp)
    ci = np.zeros(len(arcs), np.int32)
    pos = rp[:-1].copy()
    for v, w in arcs:
        ci[pos[v]] = w
        pos[v] += 1
    got = oracle_mod.jp(g.n, rp.astype(np.int32), ci, seed=4).colors
    assert (got == base).all()


# -- planted mistakes: plausible wrong versions of Algorithm 3 that the pins reject --

def _jp_mutant(oracle_mod, g, seed, kind):
    n = g.n
    col = np.zeros(n, np.int64)
    c = 0
    while (col == 0).any():
        c += 1
        W = [v for v in range(n) if col[v] == 0]
        pr = {v: oracle_mod.jp_priority(seed, 1 if kind == "fixed" else c, v) for v in range(n)}
        S = []
        for v in W:
            nb = [int(w) for w in g.colidx[g.rowptr[v]:g.rowptr[v + 1]] if w != v]
            if kind != "all_neighbours":
                nb = [w for w in nb if col[w] == 0]
            if all(pr[v] > pr[w] for w in nb):
                S.append(v)
        if kind == "smallest_free":
            for v in S:
                used = {col[int(w)] for w in g.colidx[g.rowptr[v]:g.rowptr[v + 1]]}
                col[v] = min(k for k in range(1, n + 2) if k not in used)
        else:
            for v in S:
                col[v] = c
        if c > 4 * n + 4:
            return None
    return col - 1


@pytest.mark.parametrize("kind", ["fixed", "all_neighbours", "smallest_free"])
def test_jp_pins_reject_planted_mistakes(oracle_mod, kind):
    caught = False
    for s in range(6):
        g = gg.erdos_renyi(30, 90, s)
        col = _jp_mutant(oracle_mod, g, 11, kind)
        if col is None:
            caught = True
            break
        res = oracle_mod.jp(g.n, g.rowptr, g.colidx, seed=11)
        ok = _check_certificate(oracle_mod, g, 11, col)
        ncol = int(col.max()) + 1
        if not ok or ncol != res.rounds:
            caught = True
            break
    assert caught


# -- topology-driven SGR --------------------------------------------------------

@pytest.mark.parametrize("rule", [0, 1])
def test_topo_equals_data_driven_all_5_vertex_graphs(oracle_mod, rule):
    for g in _all_graphs(5):
        a = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=rule)
        b = oracle_mod.sgr_topo(g.n, g.rowptr, g.colidx, rule=rule)
        assert (a.colors == b.colors).all() and a.rounds == b.rounds
        assert a.wsize.tolist() == b.wsize.tolist()
        assert b.visits.tolist() == [g.n] * b.rounds


@pytest.mark.parametrize("fname", ["sgr_c5.txt", "sgr_c7.txt"])
def test_topo_hand_traces(oracle_mod, fname):
    from tests.test_oracle_pins import _parse_trace
    rec = _parse_trace(fname)
    g = gg.from_edges(rec["n"], rec["edges"])
    res = oracle_mod.sgr_topo(g.n, g.rowptr, g.colidx)
    assert (res.colors + 1).tolist() == rec["final"]
    assert res.wsize.tolist() == [len(r[0]) for r in rec["rounds"]]


@pytest.mark.parametrize("rule", [0, 1])
def test_topo_equals_data_driven_random(oracle_mod, rule):
    for g in (gg.erdos_renyi(5000, 40000, 1), gg.rmat(12, 8, 2), gg.stencil27(9, 7, 5)):
        a = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=rule)
        b = oracle_mod.sgr_topo(g.n, g.rowptr, g.colidx, rule=rule)
        assert (a.colors == b.colors).all() and a.rounds == b.rounds and a.ncolors == b.ncolors
        assert a.wsize.tolist() == b.wsize.tolist()

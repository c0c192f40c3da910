"""Pins of the CPU oracle against facts fixed by the paper's definitions and by
mathematics -- not against the oracle itself.

  * hand-worked round traces (tests/golden), derived from Sec. 3.1 Algorithm Data-GC
    with the FirstFit / ConflictResolve routines of Sec. 3;
  * closed forms: K_n gets colours 1..n in n rounds; naturally numbered cycles use
    2 (even) / 3 (odd) colours; edgeless graphs use one colour in one round;
  * invariants of first-fit colourings: proper, Grundy (every colour is the mex of
    the neighbours' colours), colour(v) <= deg(v)+1, ncolors <= rounds;
  * brute force: chromatic number <= ncolors <= Grundy number on tiny graphs;
  * an independent vectorised implementation (oracle/sgr_numpy.py);
  * invariance under row order, self-loops, duplicate arcs and disjoint union.
"""
import os

import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_trace(fname):
    rec = {"rounds": []}
    with open(os.path.join(GOLDEN, fname)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "n":
                rec["n"] = int(tok[1])
            elif tok[0] == "edges":
                rec["edges"] = [tuple(int(x) for x in t.split("-")) for t in tok[1:]]
            elif tok[0] == "round":
                iW, iC, iL = tok.index("W"), tok.index("C"), tok.index("losers")
                rec["rounds"].append(([int(x) for x in tok[iW + 1:iC]],
                                      [int(x) for x in tok[iC + 1:iL]],
                                      [int(x) for x in tok[iL + 1:]]))
            elif tok[0] == "final":
                rec["final"] = [int(x) for x in tok[1:]]
            elif tok[0] == "serial_ff":
                rec["serial_ff"] = [int(x) for x in tok[1:]]
    return rec


@pytest.mark.parametrize("fname", ["sgr_c5.txt", "sgr_c7.txt"])
def test_golden_round_trace(oracle_mod, fname):
    rec = _parse_trace(fname)
    g = gg.from_edges(rec["n"], rec["edges"])
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    assert (res.colors + 1).tolist() == rec["final"]
    assert res.rounds == len(rec["rounds"])
    assert res.wsize.tolist() == [len(r[0]) for r in rec["rounds"]]
    assert res.ncolors == max(rec["final"])
    ff, nff = oracle_mod.serial_ff(g.n, g.rowptr, g.colidx)
    assert (ff + 1).tolist() == rec["serial_ff"]
    # the vectorised oracle reproduces every round of the hand trace
    trace = []
    c2, nc2, r2, _ = oracle_mod.sgr_numpy(g.n, g.rowptr, g.colidx, trace=trace)
    assert trace == [tuple(r) for r in rec["rounds"]]
    assert (c2 + 1).tolist() == rec["final"]


def test_golden_small_cases(oracle_mod):
    with open(os.path.join(GOLDEN, "sgr_p4_stars.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) >= 8
    for line in rows:
        name, n, edges, final, rounds = [x.strip() for x in line.split("|")]
        n = int(n)
        e = [tuple(int(x) for x in t.split("-")) for t in edges.split()]
        g = gg.from_edges(n, e)
        res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        assert (res.colors + 1).tolist() == [int(x) for x in final.split()], name
        assert res.rounds == int(rounds), name


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 65, 130])
def test_complete_graph_closed_form(oracle_mod, n):
    g = gg.complete(n)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    # round r settles exactly vertex r-1 with colour r
    assert res.colors.tolist() == list(range(n))
    assert res.ncolors == n and res.rounds == n
    assert res.wsize.tolist() == list(range(n, 0, -1))


@pytest.mark.parametrize("n", [4, 6, 8, 10, 100, 1000])
def test_even_cycle_two_colours(oracle_mod, n):
    g = gg.cycle(n)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    assert res.ncolors == 2
    assert res.colors.tolist() == [v % 2 for v in range(n)]


@pytest.mark.parametrize("n", [3, 5, 7, 9, 101, 1001])
def test_odd_cycle_three_colours(oracle_mod, n):
    g = gg.cycle(n)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    assert res.ncolors == 3
    assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, res.colors) == 0


@pytest.mark.parametrize("n", [0, 1, 7, 1000])
def test_edgeless(oracle_mod, n):
    g = gg.edgeless(n)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    assert res.colors.tolist() == [0] * n
    assert res.ncolors == (1 if n else 0) and res.rounds == (1 if n else 0)


def _invariants(oracle_mod, g, res):
    deg = g.degrees()
    assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, res.colors) == 0
    assert oracle_mod.non_grundy(g.n, g.rowptr, g.colidx, res.colors) == 0
    assert (res.colors + 1 <= deg + 1).all()
    if g.n:
        assert res.ncolors == int(res.colors.max()) + 1
        assert len(np.unique(res.colors)) == res.ncolors        # all colours used
        assert res.ncolors <= res.rounds <= g.n
        assert res.ncolors <= g.max_degree() + 1
        assert res.wsize[0] == g.n and (np.diff(res.wsize) < 0).all()


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n,p", [(12, 0.3), (40, 0.1), (150, 0.05), (300, 0.2)])
def test_invariants_random(oracle_mod, n, p, seed):
    g = gg.random_small(n, p, seed)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    _invariants(oracle_mod, g, res)


def test_invariants_workload_shapes(oracle_mod):
    for g in [gg.erdos_renyi(4000, 40000, 3), gg.stencil27(9, 7, 5), gg.rmat(10, 8, 2)]:
        res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        _invariants(oracle_mod, g, res)


# Hand-counted verdicts of the two checkers on known colourings (0-based colours).
# conflicts = directed arcs (v, w), v != w, with equal colours: each monochromatic edge
# counts twice.  non_grundy = vertices whose colour is not the smallest colour missing
# among their neighbours.
CHECKER_CASES = [
    # name, n, edges, colours, conflicts, non_grundy
    ("K3 proper", 3, [(0, 1), (1, 2), (2, 0)], [0, 1, 2], 0, 0),
    ("K3 one clash", 3, [(0, 1), (1, 2), (2, 0)], [0, 0, 1], 2, 2),      # v0, v1: mex {0,1} = 2
    ("K3 monochrome", 3, [(0, 1), (1, 2), (2, 0)], [0, 0, 0], 6, 3),     # every mex {0} = 1
    ("C5 SGR result", 5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)], [0, 1, 0, 2, 1], 0, 0),
    ("C5 closing clash", 5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)], [0, 1, 0, 1, 0], 2, 2),
    # v0 neighbours {1, 0}: mex 2; v4 neighbours {1, 0}: mex 2
    ("C5 swapped 3,4", 5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)], [0, 1, 0, 1, 2], 0, 0),
    # proper; v3 neighbours {0, 2}: mex 1 ok; v4 neighbours {1, 0}: mex 2 ok
    ("P4 Grundy", 4, [(0, 1), (1, 2), (2, 3)], [0, 1, 0, 1], 0, 0),
    ("P4 end one above mex", 4, [(0, 1), (1, 2), (2, 3)], [0, 1, 0, 2], 0, 1),   # v3: mex {0} = 1
    ("P4 inner one above mex", 4, [(0, 1), (1, 2), (2, 3)], [0, 2, 0, 1], 0, 1),  # v1: mex {0} = 1
    ("P4 colour below mex", 4, [(0, 1), (1, 2), (2, 3)], [0, 1, 1, 0], 2, 2),
    # v1 {0, 1}: mex 2; v2 {1, 0}: mex 2; v3 {1}: mex 0 ok
    ("star centre 2", 6, [(0, k) for k in range(1, 6)], [2, 0, 0, 0, 0, 0], 0, 1),  # centre: mex {0} = 1
    ("star leaves 1", 6, [(0, k) for k in range(1, 6)], [0, 1, 1, 1, 1, 1], 0, 0),
    ("edge both 1", 2, [(0, 1)], [1, 1], 2, 2),
    ("edgeless all 1", 3, [], [1, 1, 1], 0, 3),                           # mex of nothing = 0
]


@pytest.mark.parametrize("case", CHECKER_CASES, ids=[c[0] for c in CHECKER_CASES])
def test_checkers_on_known_colourings(oracle_mod, case):
    """The proper and Grundy checkers that the invariant pins rely on give the exact
    hand-counted numbers on good and bad colourings (a checker that always returned 0,
    or took the mex one off, fails here)."""
    _, n, edges, colours, n_conf, n_ng = case
    g = gg.from_edges(n, edges)
    c = np.array(colours, dtype=np.int32)
    assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, c) == n_conf
    assert oracle_mod.non_grundy(g.n, g.rowptr, g.colidx, c) == n_ng


def test_checkers_ignore_self_loops_and_count_duplicates_per_arc(oracle_mod):
    # a self-loop is not a conflict and is not a neighbour for the mex
    g = gg.raw_csr(2, [[0, 1], [1, 0]])
    c = np.array([0, 1], dtype=np.int32)
    assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, c) == 0
    assert oracle_mod.non_grundy(g.n, g.rowptr, g.colidx, c) == 0
    # a duplicated arc is counted once per stored arc
    g = gg.raw_csr(2, [[1, 1], [0]])
    c = np.array([0, 0], dtype=np.int32)
    assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, c) == 3
    assert oracle_mod.non_grundy(g.n, g.rowptr, g.colidx, c) == 2


@pytest.mark.parametrize("seed", range(4))
def test_checkers_see_one_changed_vertex(oracle_mod, seed):
    """Recolouring one vertex of an SGR result to a neighbour's colour creates exactly
    two conflicting arcs per neighbour holding that colour and breaks the Grundy
    property at that vertex at least."""
    g = gg.erdos_renyi(400, 2400, seed + 11)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    rng = np.random.default_rng(seed)
    for v in rng.choice(np.flatnonzero(g.degrees() > 0), 20, replace=False):
        nb = g.colidx[g.rowptr[v]:g.rowptr[v + 1]]
        c = res.colors.copy()
        c[v] = c[nb[0]]
        same = int(np.sum(c[nb] == c[v]))
        assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, c) == 2 * same
        assert oracle_mod.non_grundy(g.n, g.rowptr, g.colidx, c) >= 1


def test_brute_force_all_graphs_n5(oracle_mod):
    """chi(G) <= ncolors <= Grundy(G) on every labelled graph with 5 vertices."""
    import itertools
    from oracle import brute
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        e = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        g = gg.from_edges(5, e)
        res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        chi = brute.chromatic(g.n, g.rowptr, g.colidx)
        gam = brute.grundy(g.n, g.rowptr, g.colidx)
        assert chi <= res.ncolors <= gam, (e, chi, res.ncolors, gam)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random_n7_n8(oracle_mod, seed):
    from oracle import brute
    n = 7 if seed % 2 else 8
    g = gg.random_small(n, 0.45, 100 + seed)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    chi = brute.chromatic(g.n, g.rowptr, g.colidx)
    gam = brute.grundy(g.n, g.rowptr, g.colidx)
    assert chi <= res.ncolors <= gam


def test_brute_force_catches_non_grundy():
    """The Grundy bound is tight enough to matter: on the path 0-2-3-1 (natural order
    is not a path order) greedy orders can reach 3 colours but chi is 2."""
    from oracle import brute
    g = gg.from_edges(4, [(0, 2), (2, 3), (3, 1)])
    assert brute.chromatic(g.n, g.rowptr, g.colidx) == 2
    assert brute.grundy(g.n, g.rowptr, g.colidx) == 3


@pytest.mark.parametrize("seed", range(40))
def test_cross_check_vectorised(oracle_mod, seed):
    n = [5, 20, 60, 200, 700][seed % 5]
    p = [0.5, 0.2, 0.08, 0.03, 0.01][seed % 5]
    g = gg.random_small(n, p, seed)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    c, nc, r, ws = oracle_mod.sgr_numpy(g.n, g.rowptr, g.colidx)
    assert (c == res.colors).all() and nc == res.ncolors and r == res.rounds
    assert list(ws) == res.wsize.tolist()


def test_cross_check_workloads(oracle_mod):
    for g in [gg.config_er16k(1), gg.stencil27(12, 10, 9), gg.rmat(12, 16, 3)]:
        res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        c, nc, r, ws = oracle_mod.sgr_numpy(g.n, g.rowptr, g.colidx)
        assert (c == res.colors).all() and r == res.rounds, g.name


def test_row_order_self_loops_duplicates_do_not_matter(oracle_mod):
    g = gg.erdos_renyi(500, 3000, 9)
    ref = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    sh = gg.shuffle_rows(g, 4)
    res = oracle_mod.sgr(sh.n, sh.rowptr, sh.colidx)
    assert (res.colors == ref.colors).all() and res.rounds == ref.rounds
    # add a self-loop and a duplicate of the first arc to every non-empty row
    rows = []
    for v in range(g.n):
        r = g.colidx[g.rowptr[v]:g.rowptr[v + 1]].tolist()
        rows.append(([v] + r + r[:1]) if r else [v])
    raw = gg.raw_csr(g.n, rows)
    res2 = oracle_mod.sgr(raw.n, raw.rowptr, raw.colidx)
    assert (res2.colors == ref.colors).all() and res2.rounds == ref.rounds


def test_disjoint_union_is_componentwise(oracle_mod):
    parts = [gg.erdos_renyi(300, 1500, 1, 1), gg.stencil27(6, 5, 4), gg.complete(9), gg.cycle(11)]
    b = gg.concat_graphs(parts)
    whole = oracle_mod.sgr(b.n, b.rowptr, b.colidx)
    rounds = 0
    for i, p in enumerate(parts):
        r = oracle_mod.sgr(p.n, p.rowptr, p.colidx)
        assert (whole.colors[b.voff[i]:b.voff[i + 1]] == r.colors).all()
        rounds = max(rounds, r.rounds)
    assert whole.rounds == rounds


def test_serial_ff_is_sequential_greedy(oracle_mod):
    """Natural-order greedy alternates two colours along a naturally numbered path and
    always yields a proper Grundy colouring."""
    for n in [2, 3, 10, 33]:
        g = gg.path(n)
        ff, nff = oracle_mod.serial_ff(g.n, g.rowptr, g.colidx)
        assert ff.tolist() == [v % 2 for v in range(n)]
    g = gg.erdos_renyi(2000, 16000, 5)
    ff, nff = oracle_mod.serial_ff(g.n, g.rowptr, g.colidx)
    assert oracle_mod.conflicts(g.n, g.rowptr, g.colidx, ff) == 0
    assert oracle_mod.non_grundy(g.n, g.rowptr, g.colidx, ff) == 0


def test_greedy_in_colour_order_reproduces_result(oracle_mod):
    """A Grundy colouring is reproduced by sequential greedy applied in (colour, id)
    order; checked with an explicit Python greedy."""
    g = gg.erdos_renyi(800, 6000, 11)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    order = np.lexsort((np.arange(g.n), res.colors))
    col = np.full(g.n, -1)
    for v in order:
        nb = {int(col[w]) for w in g.colidx[g.rowptr[v]:g.rowptr[v + 1]] if col[w] >= 0}
        c = 0
        while c in nb:
            c += 1
        col[v] = c
    assert (col == res.colors).all()


def test_stats_shapes(oracle_mod):
    g = gg.config_er16k(1)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
    deg = g.degrees()
    assert res.arcs_ff[0] == g.nnz                     # round 1 scans every row
    assert len(res.wsize) == res.rounds
    assert (res.arcs_cr <= res.arcs_ff).all()
    assert oracle_mod.bytes_model(res, g.n) > 0
    assert int(deg.sum()) == g.nnz


def test_malformed_input_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.sgr(3, np.array([0, 1, 2, 2]), np.array([1, 5]))


def test_degree_rule_golden(oracle_mod):
    with open(os.path.join(GOLDEN, "sgr_degree_rule.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) >= 4
    for line in rows:
        name, n, edges, final, rounds = [x.strip() for x in line.split("|")]
        e = [tuple(int(x) for x in t.split("-")) for t in edges.split()]
        g = gg.from_edges(int(n), e)
        res = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=oracle_mod.RULE_DEGREE)
        assert (res.colors + 1).tolist() == [int(x) for x in final.split()], name
        assert res.rounds == int(rounds), name
        c2, _, r2, _ = oracle_mod.sgr_numpy(g.n, g.rowptr, g.colidx, rule=1)
        assert (c2 + 1).tolist() == [int(x) for x in final.split()] and r2 == int(rounds), name


@pytest.mark.parametrize("seed", range(20))
def test_degree_rule_cross_check_and_invariants(oracle_mod, seed):
    n = [9, 40, 150, 600][seed % 4]
    p = [0.4, 0.15, 0.05, 0.01][seed % 4]
    g = gg.random_small(n, p, 300 + seed)
    res = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=oracle_mod.RULE_DEGREE)
    c, nc, r, ws = oracle_mod.sgr_numpy(g.n, g.rowptr, g.colidx, rule=1)
    assert (c == res.colors).all() and r == res.rounds and list(ws) == res.wsize.tolist()
    _invariants(oracle_mod, g, res)


def test_degree_rule_regular_graph_equals_id_rule(oracle_mod):
    """On a regular graph every degree ties, so the rule falls back to the id rule."""
    for g in [gg.cycle(31), gg.complete(12), gg.stencil27(3, 3, 3)]:
        if len(set(g.degrees().tolist())) == 1:
            a = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=0)
            b = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=1)
            assert (a.colors == b.colors).all() and a.rounds == b.rounds


def test_degree_rule_workloads(oracle_mod):
    for g in [gg.rmat(12, 16, 2), gg.erdos_renyi(3000, 20000, 2)]:
        a = oracle_mod.sgr(g.n, g.rowptr, g.colidx, rule=1)
        c, nc, r, ws = oracle_mod.sgr_numpy(g.n, g.rowptr, g.colidx, rule=1)
        assert (c == a.colors).all() and r == a.rounds
        _invariants(oracle_mod, g, a)

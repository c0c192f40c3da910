"""GPU parity of the two other colouring methods behind the same C-ABI.

  * CSRCOLOR_ALGO_JP (Sec. 2.2, Algorithm 3) against oracle/jp_oracle.c: colours,
    colour count, rounds and per-round worklist sizes, bit for bit, for several seeds
    (the priorities are SplitMix64 outputs computed independently on each side);
  * CSRCOLOR_ALGO_SGR_TOPO (Sec. 3.1, Algorithm Topo-GC) against the data-driven
    oracle: the same colouring in the same rounds, both conflict rules.
Integer work, so the bar is exact equality.
"""
import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg
from tests.test_parity_gpu import _degree_ladder

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALGO_TOPO, ALGO_JP = 1, 2


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06025_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


def _run(g, dev, **kw):
    from paper_1606_06025_amd import api
    rp = torch.from_numpy(np.ascontiguousarray(g.rowptr, dtype=np.int32)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(g.colidx, dtype=np.int32)).to(dev)
    colors, nc, st = api.color(rp, ci, opts=api.make_opts(**kw), stats=True, stats_cap=1 << 16)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), nc, st


def _check(g, got, nc, st, ref_colors, ref_ncolors, ref_rounds, ref_wsize):
    bad = np.flatnonzero(got != ref_colors)
    assert bad.size == 0, f"{g.name}: {bad.size} differ, first {bad[:8]} got {got[bad[:8]]} want {ref_colors[bad[:8]]}"
    assert nc == ref_ncolors and st.rounds == ref_rounds, (nc, ref_ncolors, st.rounds, ref_rounds)
    k = min(len(st.wsize), ref_rounds)
    assert st.wsize[:k] == list(ref_wsize[:k])
    if g.n:
        assert st.arcs[0] == int(g.rowptr[-1])


def _jp_parity(g, dev, seed, **kw):
    import oracle
    ref = oracle.jp(g.n, g.rowptr, g.colidx, seed=seed)
    got, nc, st = _run(g, dev, algorithm=ALGO_JP, seed=seed, **kw)
    _check(g, got, nc, st, ref.colors, ref.ncolors, ref.rounds, ref.wsize.tolist())
    return got, ref


def _topo_parity(g, dev, rule=0, **kw):
    import oracle
    ref = oracle.sgr(g.n, g.rowptr, g.colidx, rule=rule)
    got, nc, st = _run(g, dev, algorithm=ALGO_TOPO, rule=rule, **kw)
    _check(g, got, nc, st, ref.colors, ref.ncolors, ref.rounds, ref.wsize.tolist())
    return got, ref


def _small_graphs():
    return [gg.from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]), gg.cycle(7), gg.path(4),
            gg.star(0, list(range(1, 6))), gg.star(5, list(range(5))), gg.complete(3), gg.edgeless(1),
            gg.from_edges(2, [(0, 1)]), gg.from_edges(3, [(1, 2)]), gg.edgeless(70000)]


@pytest.mark.parametrize("seed", [0, 1, 2**40 + 3, 2**64 - 1])
def test_jp_small_and_edge_cases(dev, seed):
    for g in _small_graphs():
        _jp_parity(g, dev, seed)


@pytest.mark.parametrize("seed", range(12))
def test_jp_fuzz(dev, seed):
    sizes = [(2, 1.0), (33, 0.3), (65, 0.9), (300, 0.02), (1000, 0.2), (4000, 0.03)]
    n, p = sizes[seed % len(sizes)]
    _jp_parity(gg.random_small(n, p, seed), dev, seed * 1000003)


@pytest.mark.parametrize("n", [64, 65, 300, 1100])
def test_jp_cliques(dev, n):
    got, ref = _jp_parity(gg.complete(n), dev, 7)
    assert sorted(got.tolist()) == list(range(n))


def test_jp_every_bucket_and_split_rows(dev):
    degs = [1, 5, 6, 13, 14, 29, 30, 61, 62, 64, 65, 300, 1023, 1024, 1025, 2000, 2049, 5000]
    for s in range(2):
        g = _degree_ladder(degs, s)
        _jp_parity(g, dev, 11 + s)
        _jp_parity(g, dev, 11 + s, t_wave=128, t_split=1024)
    for leaves, center in [(5000, 0), (40000, 20000)]:
        _jp_parity(gg.star(center, [i for i in range(leaves + 1) if i != center]), dev, 3)


def test_jp_workload_families(dev):
    for g in (gg.erdos_renyi(16384, 131072, 1), gg.rmat(15, 16, 3), gg.stencil27(16, 16, 16)):
        _jp_parity(g, dev, 1)
        _jp_parity(g, dev, 1, lane_detect=-1, blocks_per_cu=2, sync_every=3)


def test_jp_unsorted_rows_and_self_loops(dev):
    g = gg.erdos_renyi(3000, 30000, 5)
    rows = []
    for v in range(g.n):
        r = g.colidx[g.rowptr[v]:g.rowptr[v + 1]].tolist()
        rows.append(r[::-1] + [v] + r[:2])
    got, ref = _jp_parity(gg.raw_csr(g.n, rows), dev, 9)
    import oracle
    assert (got == oracle.jp(g.n, g.rowptr, g.colidx, seed=9).colors).all()


def test_jp_uses_more_colours_than_sgr(dev):
    g = gg.erdos_renyi(16384, 131072, 2)
    jp, ncj, _ = _run(g, dev, algorithm=ALGO_JP, seed=5)
    sgr, ncs, _ = _run(g, dev)
    assert ncj > ncs


@pytest.mark.parametrize("rule", [0, 1])
def test_topo_small_and_fuzz(dev, rule):
    for g in _small_graphs():
        _topo_parity(g, dev, rule)
    for seed in range(8):
        sizes = [(2, 1.0), (33, 0.3), (65, 0.9), (300, 0.02), (1000, 0.2), (4000, 0.03)]
        n, p = sizes[seed % len(sizes)]
        _topo_parity(gg.random_small(n, p, seed), dev, rule)


@pytest.mark.parametrize("rule", [0, 1])
def test_topo_hubs_cliques_and_families(dev, rule):
    degs = [1, 5, 6, 13, 14, 29, 30, 61, 62, 64, 65, 66, 300, 1025, 2049, 5000]
    _topo_parity(_degree_ladder(degs, 4), dev, rule)
    _topo_parity(gg.complete(1100), dev, rule)     # colours beyond one 64-bit mask
    _topo_parity(gg.star(20000, [i for i in range(40001) if i != 20000]), dev, rule)
    for g in (gg.erdos_renyi(16384, 131072, 1), gg.rmat(15, 16, 3), gg.stencil27(16, 16, 16)):
        _topo_parity(g, dev, rule)


def test_topo_unsorted_rows(dev):
    g = gg.shuffle_rows(gg.erdos_renyi(3000, 30000, 6), 2)
    _topo_parity(g, dev)

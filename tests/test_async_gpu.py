"""GPU: the asynchronous, device-planned boundary.

csrcolor_color_ex with a device colour count and no statistics enqueues the whole
colouring (Sec. 3.1, Algorithm Data-GC) without host read-backs, so it can be captured
into a graph and replayed; the batched entry point does the same in PERSISTENT mode.
Every result is compared with the CPU oracle bit for bit.  Also the regression cases
of releasing the workspace between colourings and of a malformed batched rowptr.
"""
import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06025_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


def _dev_graph(g, dev):
    return (torch.from_numpy(np.ascontiguousarray(g.rowptr, dtype=np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(g.colidx, dtype=np.int32)).to(dev))


def _ladder(degs, seed):
    edges = []
    nxt = len(degs)
    for h, d in enumerate(degs):
        for _ in range(d):
            edges.append((h, nxt))
            nxt += 1
    g0 = gg.random_small(nxt - len(degs), 2.0 / max(nxt - len(degs), 1), seed)
    src = np.concatenate([np.array([e[0] for e in edges], np.int64),
                          np.repeat(np.arange(g0.n), np.diff(g0.rowptr)) + len(degs)])
    dst = np.concatenate([np.array([e[1] for e in edges], np.int64), g0.colidx.astype(np.int64) + len(degs)])
    return gg.csr_from_arcs(nxt, src, dst, symmetrize=True, name="ladder")


GRAPHS = [
    lambda: gg.stencil27(24, 20, 16),
    lambda: gg.rmat(14, 16, 3),
    lambda: _ladder([5, 13, 29, 61, 300, 1500, 2500, 9000], 4),   # every bucket, split rows
    lambda: gg.erdos_renyi(20000, 160000, 5),
    lambda: gg.complete(90),
    lambda: gg.edgeless(33),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_async_matches_oracle(dev, gi):
    """No statistics and a device count: the call returns before the stream is done;
    after a synchronisation the colours and the count are the oracle's."""
    import oracle
    from paper_1606_06025_amd import api
    g = GRAPHS[gi]()
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    rp, ci = _dev_graph(g, dev)
    s = torch.cuda.Stream()
    for _ in range(2):      # the second call runs on the sized workspace without any wait
        out, nc = api.color_async(rp, ci, stream=s)
        s.synchronize()
        assert int(nc.item()) == ref.ncolors
        assert np.array_equal(out.cpu().numpy(), ref.colors)


@pytest.mark.parametrize("gi", [0, 1, 2, 3])
def test_async_graph_capture_replays(dev, gi):
    """Captured into a graph on its stream (after a first call there sized the
    workspace) and replayed three times, with the program's own eager work and
    synchronisations between the replays: every replay gives the oracle's colouring."""
    import oracle
    from paper_1606_06025_amd import api
    g = GRAPHS[gi]()
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    rp, ci = _dev_graph(g, dev)
    s = torch.cuda.Stream()
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    nc = torch.empty(1, dtype=torch.int32, device=dev)
    api.color_async(rp, ci, out=out, ncolors=nc, stream=s)
    s.synchronize()
    assert int(nc.item()) == ref.ncolors
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        api.color_async(rp, ci, out=out, ncolors=nc, stream=s)
    for _ in range(3):
        out.fill_(-1)
        nc.fill_(-99)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(nc.item()) == ref.ncolors
        assert np.array_equal(out.cpu().numpy(), ref.colors)
    del graph


def test_async_device_status(dev):
    """Errors found on the device come back in the count slot: a malformed CSR gives
    EBADCSR, a graph with more arcs than the workspace was sized for gives ENOMEM
    (nothing is read out of bounds), and a synchronous call sizes it again."""
    import oracle
    from paper_1606_06025_amd import _lib as L, api
    api.release_workspace()
    s = torch.cuda.Stream()
    small = gg.cycle(5000)
    rp, ci = _dev_graph(small, dev)
    out, nc = api.color_async(rp, ci, stream=s)
    s.synchronize()
    assert int(nc.item()) == 2
    # decreasing rowptr
    bad_rp = torch.tensor([0, 2, 1, 3], dtype=torch.int32, device=dev)
    bad_ci = torch.tensor([1, 2, 0], dtype=torch.int32, device=dev)
    _, nc = api.color_async(bad_rp, bad_ci, stream=s)
    s.synchronize()
    assert int(nc.item()) == L.EBADCSR
    # colidx out of range
    bad_ci = torch.tensor([1, 7, 0], dtype=torch.int32, device=dev)
    _, nc = api.color_async(torch.tensor([0, 1, 2, 3], dtype=torch.int32, device=dev), bad_ci, stream=s)
    s.synchronize()
    assert int(nc.item()) == L.EBADCSR
    # as many vertices as the first graph, far more arcs: the flag array cannot hold them
    big = gg.erdos_renyi(5000, 100000, 3)
    brp, bci = _dev_graph(big, dev)
    _, nc = api.color_async(brp, bci, stream=s)
    s.synchronize()
    assert int(nc.item()) == L.ENOMEM
    # a synchronous device-planned call sizes the workspace; then the asynchronous one works
    ref = oracle.sgr(big.n, big.rowptr, big.colidx)
    colors, ncs, _ = api.color(brp, bci, opts=api.make_opts(mode=L.MODE_PERSISTENT), stream=s)
    assert ncs == ref.ncolors and np.array_equal(colors.cpu().numpy(), ref.colors)
    out, nc = api.color_async(brp, bci, stream=s)
    s.synchronize()
    assert int(nc.item()) == ref.ncolors and np.array_equal(out.cpu().numpy(), ref.colors)


def test_async_options(dev):
    """Device-planned runs honour the options that only move work (FirstFit variants,
    thresholds, hints, live lists, ordered compaction) and the degree rule."""
    import oracle
    from paper_1606_06025_amd import api
    g = _ladder([5, 13, 29, 61, 300, 1500, 2500, 9000], 6)
    ref0 = oracle.sgr(g.n, g.rowptr, g.colidx)
    ref1 = oracle.sgr(g.n, g.rowptr, g.colidx, rule=1)
    rp, ci = _dev_graph(g, dev)
    s = torch.cuda.Stream()
    for kw in [dict(firstfit=1), dict(firstfit=2), dict(t_wave=61, t_split=1024), dict(hints=-1),
               dict(live_lists=-1), dict(ordered=1), dict(blocks_per_cu=1), dict(rule=1),
               dict(rule=1, firstfit=1)]:
        ref = ref1 if kw.get("rule") == 1 else ref0
        out, nc = api.color_async(rp, ci, opts=api.make_opts(**kw), stream=s)
        s.synchronize()
        assert int(nc.item()) == ref.ncolors, kw
        assert np.array_equal(out.cpu().numpy(), ref.colors), kw


def test_batched_persistent_async(dev):
    """The batched entry point in PERSISTENT mode colours the whole union in one
    device-planned launch and returns without waiting; every graph gets the oracle's
    colouring and count."""
    import oracle
    from paper_1606_06025_amd import api
    parts = [gg.erdos_renyi(1500, 12000, 1, 1), gg.stencil27(9, 8, 7), gg.complete(70),
             gg.star(3, [0, 1, 2, 4, 5, 6, 7]), gg.edgeless(50), gg.cycle(21),
             gg.rmat(11, 16, 4), _ladder([300, 2500, 5000], 2)]
    b = gg.concat_graphs(parts)
    voff = torch.from_numpy(b.voff).to(dev)
    rp = torch.from_numpy(b.rowptr).to(dev)
    ci = torch.from_numpy(b.colidx).to(dev)
    colors, ncol = api.color_batched(voff, rp, ci, opts=api.make_opts(mode=2))
    colors = colors.cpu().numpy()
    ncol = ncol.cpu().numpy()
    for i, p in enumerate(parts):
        ref = oracle.sgr(p.n, p.rowptr, p.colidx)
        assert np.array_equal(colors[b.voff[i]:b.voff[i + 1]], ref.colors), i
        assert ncol[i] == ref.ncolors


def test_batched_malformed_boundary_rowptr(dev):
    """A rowptr that is malformed at a graph boundary is reported as EBADCSR by the
    batched entry point (host-driven and device-planned) before any arc is read by the
    per-graph check."""
    from paper_1606_06025_amd import _lib as L, api
    g = gg.concat_graphs([gg.cycle(6), gg.cycle(5)])
    voff = torch.from_numpy(g.voff).to(dev)
    for bad in (-5, 1 << 30):
        rp = g.rowptr.copy()
        rp[6] = bad                     # the first vertex of the second graph
        trp = torch.from_numpy(rp).to(dev)
        tci = torch.from_numpy(g.colidx).to(dev)
        with pytest.raises(L.CsrColorError) as e:
            api.color_batched(voff, trp, tci)
        assert e.value.status == L.EBADCSR
        _, ncol = api.color_batched(voff, trp, tci, opts=api.make_opts(mode=2))
        assert (ncol.cpu().numpy() == L.EBADCSR).all()


def test_release_then_colour_again(dev):
    """Releasing the workspace and colouring again (wake flags on the stencil and ER,
    the device-planned path, the graph mode) gives the oracle's colourings."""
    import oracle
    from paper_1606_06025_amd import api
    gs = [gg.stencil27(20, 18, 16), gg.config_er16k(2)]
    refs = [oracle.sgr(g.n, g.rowptr, g.colidx) for g in gs]
    dg = [_dev_graph(g, dev) for g in gs]
    for it in range(2):
        for (rp, ci), ref in zip(dg, refs):
            for kw in (dict(), dict(wake=1), dict(mode=2), dict(mode=3)):
                colors, nc, st = api.color(rp, ci, opts=api.make_opts(**kw), stats=True)
                assert nc == ref.ncolors and st.rounds == ref.rounds, kw
                assert np.array_equal(colors.cpu().numpy(), ref.colors), kw
            out, ncd = api.color_async(rp, ci)
            torch.cuda.synchronize()
            assert int(ncd.item()) == ref.ncolors and np.array_equal(out.cpu().numpy(), ref.colors)
        api.release_workspace()

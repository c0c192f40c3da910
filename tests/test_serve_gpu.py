"""Serving on the GPU: continuous batching over several stream slots gives every
request exactly the colouring it gets alone (tolerance 0), and csrcolor_color_multi
matches per-graph calls."""
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


def _mix(k, seed):
    out = []
    for i in range(k):
        if i % 2:
            out.append(gg.rmat(10 + i % 5, 8 + 4 * (i % 4), seed, sub=i))
        else:
            out.append(gg.erdos_renyi(1000 + 997 * i, (1000 + 997 * i) * (4 + i % 12), seed, i))
    return out


def test_color_multi_equals_single(dev):
    import oracle
    from paper_1606_06025_amd import api
    gs = _mix(12, 1) + [gg.edgeless(5), gg.complete(40), gg.star(2, [0, 1, 3, 4])]
    dgs = [(torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.colidx).to(dev)) for g in gs]
    outs, ncol = api.color_multi(dgs)
    ncol = ncol.cpu().numpy()
    for i, g in enumerate(gs):
        ref = oracle.sgr(g.n, g.rowptr, g.colidx)
        assert (outs[i].cpu().numpy() == ref.colors).all()
        assert ncol[i] == ref.ncolors


def test_color_multi_rejects_bad_graph(dev):
    from paper_1606_06025_amd import _lib as L, api
    good = gg.cycle(9)
    rp = torch.tensor([0, 1, 2], dtype=torch.int32, device=dev)
    ci = torch.tensor([5, 0], dtype=torch.int32, device=dev)     # id 5 outside its 2-vertex graph
    with pytest.raises(L.CsrColorError) as e:
        api.color_multi([(torch.from_numpy(good.rowptr).to(dev), torch.from_numpy(good.colidx).to(dev)), (rp, ci)])
    assert e.value.status == L.EBADCSR


@pytest.mark.parametrize("small_grid", [0, 200_000])
def test_server_alone_vs_mix(dev, small_grid):
    """Every served result is the CPU oracle's colouring, and the one the graph gets
    alone (tolerance 0), also with small batches on one workgroup per CU.  Also the
    regression case of the first multi-graph call on fresh streams (each slot's
    workspace starts empty and grows while the union is being built)."""
    import oracle
    from paper_1606_06025_amd import api, serve
    gs = _mix(24, 7)
    refs = [oracle.sgr(g.n, g.rowptr, g.colidx) for g in gs]
    # alone: one library call per graph
    alone = []
    for g in gs:
        c, nc, _ = api.color(torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.colidx).to(dev))
        alone.append((c.cpu().numpy(), nc))
    limits = dict(max_batch=8, max_batch_vertices=8 * max(g.n for g in gs), max_batch_arcs=8 * max(g.nnz for g in gs))
    be = serve.HipBackend(nslots=3, small_grid_arcs=small_grid)
    reserved = 3 * be.workspace_bytes(limits["max_batch"], limits["max_batch_vertices"], limits["max_batch_arcs"])
    budget = reserved + 6 * max(serve.footprint_bytes(g.n, g.nnz) for g in gs)
    # every request is queued before the scheduler starts, so the first dispatch finds
    # several admitted requests whatever the speed of the GPU
    srv = serve.ColoringServer(be, budget, **limits)
    reqs = [srv.submit(g.rowptr, g.colidx) for g in gs]
    with srv:
        for r in reqs:
            assert r.wait(timeout=60)
        assert srv.peak_bytes <= budget
    assert max(r.batch_size for r in reqs) > 1
    for (c, nc), r, ref in zip(alone, reqs, refs):
        assert r.error is None
        assert np.array_equal(r.colors, ref.colors) and r.ncolors == ref.ncolors
        assert np.array_equal(r.colors, c) and r.ncolors == nc


def test_server_memory_within_budget(dev):
    """During a replay the library's workspaces plus the server's tensors never exceed
    the HBM budget the server admits against, and the workspaces stay within their
    reservation; every result is the oracle's."""
    import threading
    import time
    import oracle
    from paper_1606_06025_amd import api, serve
    api.release_workspace()
    torch.cuda.synchronize()
    gs = _mix(24, 11)
    refs = [oracle.sgr(g.n, g.rowptr, g.colidx) for g in gs]
    limits = dict(max_batch=6, max_batch_vertices=max(g.n for g in gs) * 3,
                  max_batch_arcs=max(g.nnz for g in gs) * 3)
    be = serve.HipBackend(nslots=2)
    reserved = 2 * be.workspace_bytes(limits["max_batch"], limits["max_batch_vertices"], limits["max_batch_arcs"])
    budget = reserved + 4 * max(serve.footprint_bytes(g.n, g.nnz) for g in gs)
    base = torch.cuda.memory_allocated()
    peak = {"total": 0, "lib": 0}
    stop = threading.Event()

    def sample():
        while not stop.is_set():
            lib = api.device_bytes_in_use()
            tot = lib + torch.cuda.memory_allocated() - base
            peak["lib"] = max(peak["lib"], lib)
            peak["total"] = max(peak["total"], tot)
            time.sleep(0.0002)

    th = threading.Thread(target=sample)
    th.start()
    try:
        with serve.ColoringServer(be, budget, **limits) as srv:
            reqs, _ = serve.replay(srv, [(g.rowptr, g.colidx) for g in gs], [0.001 * i for i in range(len(gs))])
            assert srv.peak_bytes <= budget
    finally:
        stop.set()
        th.join()
    # small per-batch tensors of the binding (the colour counts) are the only slack
    assert peak["lib"] <= reserved, (peak, reserved)
    assert peak["total"] <= budget + (1 << 20), (peak, budget)
    for r, ref in zip(reqs, refs):
        assert r.error is None and np.array_equal(r.colors, ref.colors) and r.ncolors == ref.ncolors


def test_malformed_request_fails_alone_in_a_batch(dev):
    """A request whose ids leave its graph is rejected by the library; the batch it was
    in runs again one request at a time, so only it fails."""
    import oracle
    from paper_1606_06025_amd import serve
    gs = _mix(8, 3)
    bad_rp = np.array([0, 1, 2], dtype=np.int32)
    bad_ci = np.array([7, 0], dtype=np.int32)            # id 7 outside the 2-vertex graph
    srv = serve.ColoringServer(serve.HipBackend(nslots=1), 8 << 30, max_batch=16)
    rs = [srv.submit(g.rowptr, g.colidx) for g in gs[:4]]
    rb = srv.submit(bad_rp, bad_ci)
    rs += [srv.submit(g.rowptr, g.colidx) for g in gs[4:]]
    with srv:
        for r in rs + [rb]:
            assert r.wait(timeout=60)
    assert rb.error
    for g, r in zip(gs, rs):
        ref = oracle.sgr(g.n, g.rowptr, g.colidx)
        assert r.error is None and np.array_equal(r.colors, ref.colors)

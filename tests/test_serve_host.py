"""Serving scheduler on the host: the CPU oracle stands in for the device.

Checks that admission never lets the admitted HBM footprint exceed the budget, that
every request gets the colouring it gets alone, that requests arriving while others
run are still batched and served, that an oversize request is rejected without
affecting the others, and that a failing request fails alone."""
import threading
import time

import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg
from paper_1606_06025_amd import serve


class OracleBackend(serve.Backend):
    def __init__(self, nslots=2, delay=0.002, fail_on=None):
        import oracle
        self.oracle = oracle
        self.nslots = nslots
        self.delay = delay
        self.fail_on = fail_on or set()
        self.live = 0
        self.lock = threading.Lock()
        self.batches = []

    def upload(self, rowptr, colidx, uploader=0):
        if len(rowptr) - 1 in self.fail_on:
            raise ValueError("bad graph")
        with self.lock:
            self.live += 1
        return (np.asarray(rowptr), np.asarray(colidx))

    def release(self, handle):
        if handle is not None:
            with self.lock:
                self.live -= 1

    def run_batch(self, slot, handles):
        self.batches.append(len(handles))
        time.sleep(self.delay)
        out = []
        for rp, ci in handles:
            r = self.oracle.sgr(len(rp) - 1, rp, ci)
            out.append((r.colors, r.ncolors))
        return out


def _graphs(k, seed=0):
    res = []
    for i in range(k):
        if i % 3 == 0:
            g = gg.rmat(8 + i % 4, 8, seed + i)
        elif i % 3 == 1:
            g = gg.erdos_renyi(500 + 37 * i, 2500 + 100 * i, seed, i)
        else:
            g = gg.stencil27(5 + i % 4, 6, 4)
        res.append(g)
    return res


def test_results_equal_alone_and_budget_respected(oracle_mod):
    gs = _graphs(30)
    fps = [serve.footprint_bytes(g.n, g.nnz) for g in gs]
    budget = 3 * max(fps)           # forces queueing: at most a few graphs admitted at once
    be = OracleBackend(nslots=2, delay=0.003)
    with serve.ColoringServer(be, budget, max_batch=4) as srv:
        reqs, wall = serve.replay(srv, [(g.rowptr, g.colidx) for g in gs], [0.0005 * i for i in range(len(gs))])
        assert srv.peak_bytes <= budget
    assert be.live == 0
    for g, r in zip(gs, reqs):
        assert r.error is None
        ref = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        assert (r.colors == ref.colors).all() and r.ncolors == ref.ncolors
        assert r.latency >= 0 and r.done_time >= r.started >= r.admitted >= r.arrival - 1e-9
    assert max(be.batches) > 1       # continuous batching actually grouped requests
    s = serve.latency_summary(reqs)
    assert s["count"] == len(gs) and s["p99_ms"] >= s["p50_ms"] > 0


class RecordingBackend(OracleBackend):
    def run_batch(self, slot, handles):
        self.groups = getattr(self, "groups", [])
        self.groups.append([int(np.diff(rp).max()).bit_length() for rp, _ in handles])
        return super().run_batch(slot, handles)


def test_batches_group_graphs_of_like_degree(oracle_mod):
    """Interleaved hub graphs (R-MAT) and flat graphs (cycles, small ER): every batch
    holds the oldest waiting request and only graphs whose largest degree has a bit
    length within one of its own; all results are still the stand-alone colourings."""
    gs = []
    for i in range(24):
        gs.append(gg.rmat(10, 16, i) if i % 2 == 0 else gg.cycle(50 + i))
    be = RecordingBackend(nslots=1, delay=0.01)
    with serve.ColoringServer(be, 1 << 40, max_batch=8) as srv:
        reqs = [srv.submit(g.rowptr, g.colidx) for g in gs]
        for r in reqs:
            assert r.wait(60)
    for b in be.groups:
        assert max(b) - min(b) <= 2 and all(abs(x - b[0]) <= 1 for x in b), be.groups
    assert max(len(b) for b in be.groups) > 1
    assert sorted(sum(be.groups, [])) == sorted(int(np.diff(g.rowptr).max()).bit_length() for g in gs)
    for g, r in zip(gs, reqs):
        ref = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        assert r.error is None and (r.colors == ref.colors).all()


def test_oversize_request_rejected_others_served():
    gs = _graphs(6, seed=3)
    big = gg.erdos_renyi(20000, 200000, 5)
    budget = serve.footprint_bytes(big.n, big.nnz) - 1
    be = OracleBackend(nslots=1)
    with serve.ColoringServer(be, budget) as srv:
        rb = srv.submit(big.rowptr, big.colidx)
        rs = [srv.submit(g.rowptr, g.colidx) for g in gs]
        for r in rs + [rb]:
            assert r.wait(30)
    assert rb.error and all(r.error is None for r in rs)


def test_failing_request_fails_alone():
    gs = _graphs(5, seed=7)
    bad = gg.cycle(13)
    be = OracleBackend(nslots=2, fail_on={13})
    with serve.ColoringServer(be, 1 << 40) as srv:
        rs = [srv.submit(g.rowptr, g.colidx) for g in gs[:2]]
        rb = srv.submit(bad.rowptr, bad.colidx)
        rs += [srv.submit(g.rowptr, g.colidx) for g in gs[2:]]
        for r in rs + [rb]:
            assert r.wait(30)
    assert rb.error and "bad graph" in rb.error
    assert all(r.error is None for r in rs)
    assert be.live == 0


def test_footprint_model_monotone():
    assert serve.footprint_bytes(10, 20) < serve.footprint_bytes(11, 20) < serve.footprint_bytes(11, 21)


class BatchFailBackend(OracleBackend):
    """The device rejects any batch holding the graph of `bad_n` vertices (as the library
    rejects a union with one malformed graph)."""

    def __init__(self, bad_n, **kw):
        super().__init__(**kw)
        self.bad_n = bad_n

    def run_batch(self, slot, handles):
        if any(len(rp) - 1 == self.bad_n for rp, _ in handles):
            raise RuntimeError("csrcolor status -2: malformed CSR")
        return super().run_batch(slot, handles)


def test_failed_batch_reruns_each_request_alone(oracle_mod):
    gs = [gg.cycle(20 + i) for i in range(8)]
    bad = gg.cycle(17)
    be = BatchFailBackend(17, nslots=1, delay=0.01)
    with serve.ColoringServer(be, 1 << 40, max_batch=16) as srv:
        # queued before the scheduler starts: the first batch holds the bad graph too
        rs = [srv.submit(g.rowptr, g.colidx) for g in gs[:4]]
        rb = srv.submit(bad.rowptr, bad.colidx)
        rs += [srv.submit(g.rowptr, g.colidx) for g in gs[4:]]
        for r in rs + [rb]:
            assert r.wait(30)
    assert rb.error and "malformed" in rb.error
    for g, r in zip(gs, rs):
        ref = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        assert r.error is None and (r.colors == ref.colors).all()
    assert be.live == 0


class SizedBackend(OracleBackend):
    def workspace_bytes(self, graphs, n, nnz):
        return 1000 + 7 * n + 3 * nnz + 11 * graphs


def test_ledger_reserves_slots_and_charges_requests(oracle_mod):
    """The slots' workspaces are reserved up front at the size for the batch limits;
    requests are charged their CSR and output; the total never exceeds the budget and
    a request above the batch limits is rejected."""
    gs = _graphs(20, seed=11)
    be = SizedBackend(nslots=2, delay=0.002)
    limits = dict(max_batch=4, max_batch_vertices=4000, max_batch_arcs=40000)
    reserved = 2 * be.workspace_bytes(4, 4000, 40000)
    budget = reserved + 3 * max(serve.footprint_bytes(g.n, g.nnz) for g in gs)
    big = gg.erdos_renyi(5000, 10000, 1)        # more vertices than a batch may hold
    with serve.ColoringServer(be, budget, **limits) as srv:
        assert srv.reserved_bytes == reserved
        rb = srv.submit(big.rowptr, big.colidx)
        reqs, _ = serve.replay(srv, [(g.rowptr, g.colidx) for g in gs], [0.0003 * i for i in range(len(gs))])
        assert reserved < srv.peak_bytes <= budget
    assert rb.error and "workspace" in rb.error
    for g, r in zip(gs, reqs):
        assert r.error is None
        assert r.batch_size <= 4
    with pytest.raises(ValueError):
        serve.ColoringServer(be, reserved - 1, **limits)


def test_small_request_slot(oracle_mod):
    """With small_arcs set, slot 0 only runs batches led by small requests; every result
    is still the stand-alone colouring."""
    class SlotBackend(OracleBackend):
        def run_batch(self, slot, handles):
            self.seen = getattr(self, "seen", [])
            self.seen.append((slot, int(handles[0][1].size)))       # the batch's lead request
            return super().run_batch(slot, handles)
    gs = [gg.erdos_renyi(3000, 30000, 1, i) if i % 3 == 0 else gg.cycle(30 + i) for i in range(18)]
    be = SlotBackend(nslots=2, delay=0.005)
    with serve.ColoringServer(be, 1 << 40, max_batch=2, small_arcs=1000) as srv:
        reqs, _ = serve.replay(srv, [(g.rowptr, g.colidx) for g in gs], [0.001 * i for i in range(len(gs))])
    assert all(lead <= 1000 for slot, lead in be.seen if slot == 0)
    assert any(slot == 0 for slot, _ in be.seen) and any(lead > 1000 for _, lead in be.seen)
    for g, r in zip(gs, reqs):
        ref = oracle_mod.sgr(g.n, g.rowptr, g.colidx)
        assert r.error is None and (r.colors == ref.colors).all()

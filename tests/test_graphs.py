"""Seeded generators: exact sizes, symmetry, determinism, degree structure."""
import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg


def _check_csr(g):
    rp, ci = g.rowptr.astype(np.int64), g.colidx.astype(np.int64)
    assert rp[0] == 0 and (np.diff(rp) >= 0).all() and rp[-1] == len(ci)
    assert ci.min(initial=0) >= 0 and ci.max(initial=-1) < g.n
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert not (src == ci).any()                                  # no self-loops
    key = src * g.n + ci
    assert (np.diff(key) > 0).all()                               # sorted, no duplicates
    rev = np.sort(ci * g.n + src)
    assert (rev == key).all()                                     # symmetric


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 4, 5), (8, 8, 8), (9, 7, 5), (1, 1, 6)])
def test_stencil_closed_form(dims):
    g = gg.stencil27(*dims)
    _check_csr(g)
    assert g.nnz == gg.stencil27_arcs(*dims)
    if min(dims) >= 3:
        assert g.max_degree() == 26


def test_stencil128_arc_count_formula():
    assert gg.stencil27_arcs(128, 128, 128) == 53645816


def test_er_deterministic_and_valid():
    a = gg.erdos_renyi(3000, 20000, 7)
    b = gg.erdos_renyi(3000, 20000, 7)
    c = gg.erdos_renyi(3000, 20000, 8)
    _check_csr(a)
    assert (a.colidx == b.colidx).all() and (a.rowptr == b.rowptr).all()
    assert a.nnz != c.nnz or (a.colidx != c.colidx).any()
    assert 0.97 * 40000 < a.nnz <= 40000


def test_er16k_shape():
    g = gg.config_er16k(1)
    _check_csr(g)
    assert g.n == 16384 and 0.99 * 262144 < g.nnz <= 262144


def test_rmat_shape():
    g = gg.rmat(12, 16, 1)
    _check_csr(g)
    deg = g.degrees()
    assert g.n == 4096
    assert 0.5 * 2 * 16 * 4096 < g.nnz <= 2 * 16 * 4096
    assert (deg == 0).mean() > 0.05                  # skewed: many isolated vertices
    assert deg.max() > 20 * deg.mean()               # and hubs
    g2 = gg.rmat(12, 16, 1)
    assert (g2.colidx == g.colidx).all()


def test_rmat_chunking_invariant():
    a = gg.rmat(10, 8, 3, chunk=1 << 20)
    b = gg.rmat(10, 8, 3, chunk=777)
    assert (a.colidx == b.colidx).all() and (a.rowptr == b.rowptr).all()


def test_rmat_uniform_params_has_no_hubs():
    g = gg.rmat(12, 8, 1, abcd=(0.25, 0.25, 0.25, 0.25))
    deg = g.degrees()
    assert deg.max() < 6 * deg.mean()


def test_batch_specs_and_concat():
    specs = gg.batch_specs(64, seed=2, nmax=2e4)
    assert len(specs) == 64
    assert sum(s.kind == "er" for s in specs) == 32
    for s in specs:
        assert s.est_vertices() >= 1000 or s.kind == "er"
        if s.kind == "stencil":
            assert all(8 <= d <= 48 for d in s.params)
    parts = [s.build() for s in specs[:6]]
    b = gg.concat_graphs(parts, keep_parts=True)
    assert b.G == 6 and b.voff[-1] == sum(p.n for p in parts)
    for i, p in enumerate(parts):
        v0, v1 = b.voff[i], b.voff[i + 1]
        sub = b.colidx[b.rowptr[v0]:b.rowptr[v1]]
        assert ((sub >= v0) & (sub < v1)).all()
        assert (sub - v0 == p.colidx).all()


def test_serve_stream_poisson():
    reqs = gg.serve_stream(400, qps=50.0, seed=3)
    t = np.array([r.arrival_s for r in reqs])
    assert (np.diff(t) > 0).all()
    gaps = np.diff(np.r_[0.0, t])
    assert 0.8 / 50 < gaps.mean() < 1.25 / 50
    kinds = [r.spec.kind for r in reqs]
    assert 120 < kinds.count("rmat") < 280
    for r in reqs:
        if r.spec.kind == "rmat":
            assert 10 <= r.spec.params[0] <= 20 and 8 <= r.spec.params[1] <= 32
        else:
            assert 1000 <= r.spec.params[0] <= 1e6


@pytest.mark.parametrize("n,d,abcd", [(1000, 10, gg.RMAT_ER), (3000, 4, gg.RMAT_G), (5000, 20, gg.RMAT_ER),
                                      (2, 3, gg.RMAT_G)])
def test_rmat_n_sweep_graphs(n, d, abcd):
    g = gg.rmat_n(n, d, 5, abcd=abcd)
    assert g.n == n and g.rowptr[0] == 0 and np.all(np.diff(g.rowptr) >= 0)
    assert g.colidx.min(initial=0) >= 0 and (g.nnz == 0 or g.colidx.max() < n)
    src = np.repeat(np.arange(n), np.diff(g.rowptr))
    assert not np.any(src == g.colidx)
    fwd = set(zip(src.tolist(), g.colidx.tolist()))
    assert all((w, v) in fwd for v, w in fwd)
    if n >= 1000:
        # duplicates and the id restriction cost a little; skewed parameters cost more
        assert 0.6 * d <= g.nnz / n <= 1.05 * d
    h = gg.rmat_n(n, d, 5, abcd=abcd)
    assert np.array_equal(g.colidx, h.colidx)


def test_rmat_n_skew():
    er = gg.rmat_n(1 << 15, 10, 1, abcd=gg.RMAT_ER)
    rg = gg.rmat_n(1 << 15, 10, 1, abcd=gg.RMAT_G)
    assert rg.max_degree() > 3 * er.max_degree()

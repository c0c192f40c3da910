"""GPU parity: the HIP colouring equals the CPU oracle bit for bit.

Every case runs through the C-ABI (csrcolor_color_ex / csrcolor_color_batched) and
compares colours, colour count, round count and per-round worklist sizes and arc
counts with the serial oracle on the same seeded input.  Integer work, so the bar is
exact equality.
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


def _run(g, dev, **kw):
    from paper_1606_06025_amd import api
    rp = torch.from_numpy(np.ascontiguousarray(g.rowptr, dtype=np.int32)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(g.colidx, dtype=np.int32)).to(dev)
    opts = api.make_opts(**kw) if kw else None
    colors, nc, st = api.color(rp, ci, opts=opts, stats=True, stats_cap=1 << 16)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), nc, st


def _assert_parity(g, dev, ref=None, **kw):
    import oracle
    if ref is None:
        ref = oracle.sgr(g.n, g.rowptr, g.colidx, rule=kw.get("rule", 0))
    got, nc, st = _run(g, dev, **kw)
    assert got.shape == ref.colors.shape
    bad = np.flatnonzero(got != ref.colors)
    assert bad.size == 0, f"{g.name}: {bad.size} vertices differ, first {bad[:8]} got {got[bad[:8]]} want {ref.colors[bad[:8]]}"
    assert nc == ref.ncolors, (nc, ref.ncolors)
    assert st.rounds == ref.rounds, (st.rounds, ref.rounds)
    k = min(len(st.wsize), ref.rounds)
    assert st.wsize[:k] == ref.wsize[:k].tolist()
    assert st.arcs[:k] == ref.arcs_ff[:k].tolist()
    return got, ref


def test_golden_small(dev):
    for n, edges in [(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]),
                     (7, [(i, (i + 1) % 7) for i in range(7)]),
                     (4, [(0, 1), (1, 2), (2, 3)]),
                     (6, [(0, k) for k in range(1, 6)]),
                     (6, [(5, k) for k in range(5)]),
                     (3, [(0, 1), (1, 2), (2, 0)]),
                     (1, []), (2, [(0, 1)]), (3, [(1, 2)])]:
        _assert_parity(gg.from_edges(n, edges), dev)


def test_hand_trace_values(dev):
    got, _, st = _run(gg.cycle(5), dev)
    assert (got + 1).tolist() == [1, 2, 1, 3, 2] and st.rounds == 3
    got, _, st = _run(gg.cycle(7), dev)
    assert (got + 1).tolist() == [1, 2, 1, 2, 1, 3, 2] and st.rounds == 4


@pytest.mark.parametrize("seed", range(24))
def test_fuzz_random(dev, seed):
    sizes = [(2, 1.0), (9, 0.5), (33, 0.3), (64, 0.2), (65, 0.9), (130, 0.05), (300, 0.02),
             (700, 0.01), (1000, 0.2), (2500, 0.004), (4000, 0.03), (5000, 0.001)]
    n, p = sizes[seed % len(sizes)]
    g = gg.random_small(n, p, seed)
    _assert_parity(g, dev)


@pytest.mark.parametrize("n", [33, 64, 65, 129, 300, 1025, 1100])
def test_complete_graphs_many_colours(dev, n):
    got, ref = _assert_parity(gg.complete(n), dev)
    assert got.tolist() == list(range(n))


def test_edgeless_and_single(dev):
    for n in [1, 2, 1000, 70000]:
        got, ref = _assert_parity(gg.edgeless(n), dev)
        assert (got == 0).all()


@pytest.mark.parametrize("leaves,center", [(200, 0), (5000, 0), (5000, 5000), (40000, 20000)])
def test_stars_hubs(dev, leaves, center):
    lv = [i for i in range(leaves + 1) if i != center]
    _assert_parity(gg.star(center, lv), dev)


def test_unsorted_rows_selfloops_duplicates(dev):
    import oracle
    g = gg.erdos_renyi(3000, 30000, 5)
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    got, _ = _assert_parity(gg.shuffle_rows(g, 1), dev)
    assert (got == ref.colors).all()
    rows = []
    for v in range(g.n):
        r = g.colidx[g.rowptr[v]:g.rowptr[v + 1]].tolist()
        rows.append(r[::-1] + [v] + r[:2])
    raw = gg.raw_csr(g.n, rows)
    got, _ = _assert_parity(raw, dev)          # stats from the oracle on the same raw input
    assert (got == ref.colors).all()           # self-loops / duplicates do not change colours


def test_mixed_degree_rmat(dev):
    for sc, ef, seed in [(12, 16, 1), (14, 8, 2), (15, 16, 3)]:
        _assert_parity(gg.rmat(sc, ef, seed), dev)


def test_mixed_stencils(dev):
    for dims in [(2, 2, 2), (3, 5, 7), (16, 16, 16), (40, 9, 11)]:
        _assert_parity(gg.stencil27(*dims), dev)


@pytest.mark.parametrize("kw", [dict(t_wave=61), dict(t_wave=64), dict(t_wave=200),
                                dict(blocks_per_cu=1), dict(blocks_per_cu=3), dict(sync_every=1),
                                dict(sync_every=5), dict(t_wave=70, blocks_per_cu=2, sync_every=3),
                                dict(hints=-1), dict(hints=1, lane_detect=-1), dict(hints=-1, lane_detect=-1),
                                dict(wake=-1), dict(wake=1, lane_detect=-1), dict(wake=1, firstfit=2),
                                dict(tile_limits=3 | (9 << 8) | (21 << 16)),
                                dict(tile_limits=1 | (1 << 8) | (1 << 16), wake=-1),
                                dict(tile_limits=2 | (5 << 8) | (13 << 16), firstfit=1, lane_detect=-1),
                                dict(tile_limits=2 | (5 << 8) | (13 << 16), mode=2)])
def test_launch_options_do_not_change_result(dev, kw):
    import oracle
    g = gg.rmat(13, 16, 9)
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    _assert_parity(g, dev, ref, **kw)


def test_repeated_runs_identical(dev):
    g = gg.erdos_renyi(20000, 200000, 4)
    a, _, _ = _run(g, dev)
    for _ in range(3):
        b, _, _ = _run(g, dev)
        assert (a == b).all()


def test_config_er16k_full(dev):
    for seed in (1, 2, 3):
        _assert_parity(gg.config_er16k(seed), dev)


def test_config_stencil128_full(dev):
    import oracle
    g = gg.config_stencil128()
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    assert ref.rounds == 197 and ref.ncolors == 8
    _assert_parity(g, dev, ref)


def test_malformed_inputs_are_rejected(dev):
    from paper_1606_06025_amd import _lib as L, api
    cases = [
        (np.array([0, 2, 1, 3], np.int32), np.array([1, 2, 0], np.int32)),      # rowptr decreasing
        (np.array([1, 2, 3, 4], np.int32), np.array([1, 2, 0, 1], np.int32)),   # rowptr[0] != 0
        (np.array([0, 1, 2, 3], np.int32), np.array([1, 7, 0], np.int32)),      # colidx >= n
        (np.array([0, 1, 2, 3], np.int32), np.array([1, -1, 0], np.int32)),     # colidx < 0
    ]
    for rp, ci in cases:
        t_rp = torch.from_numpy(rp).to(dev)
        t_ci = torch.from_numpy(ci).to(dev)
        with pytest.raises(L.CsrColorError) as e:
            api.color(t_rp, t_ci)
        assert e.value.status == L.EBADCSR
    # asymmetric graph under symmetry validation
    rp = torch.tensor([0, 1, 1, 1], dtype=torch.int32, device=dev)
    ci = torch.tensor([1], dtype=torch.int32, device=dev)
    with pytest.raises(L.CsrColorError) as e:
        api.color(rp, ci, opts=api.make_opts(validate=1))
    assert e.value.status == L.ENOTSYM
    # the library still works afterwards
    _assert_parity(gg.cycle(9), dev)


def test_symmetry_validation_accepts_valid(dev):
    _assert_parity(gg.erdos_renyi(2000, 9000, 3), dev, validate=1)


def test_raw_entry_point(dev):
    from paper_1606_06025_amd import api
    import oracle
    g = gg.erdos_renyi(1000, 5000, 2)
    rp = torch.from_numpy(g.rowptr).to(dev)
    ci = torch.from_numpy(g.colidx).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    nc = api.color_raw(g.n, rp.data_ptr(), ci.data_ptr(), out.data_ptr())
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    assert nc == ref.ncolors
    assert (out.cpu().numpy() == ref.colors).all()


def test_batched_equals_per_graph(dev):
    import oracle
    from paper_1606_06025_amd import api
    parts = [gg.erdos_renyi(1500, 12000, 1, 1), gg.stencil27(9, 8, 7), gg.complete(70),
             gg.star(3, [0, 1, 2, 4, 5, 6, 7]), gg.edgeless(50), gg.cycle(21),
             gg.rmat(11, 16, 4), gg.erdos_renyi(5000, 20000, 1, 2)]
    b = gg.concat_graphs(parts)
    voff = torch.from_numpy(b.voff).to(dev)
    rp = torch.from_numpy(b.rowptr).to(dev)
    ci = torch.from_numpy(b.colidx).to(dev)
    colors, ncol = api.color_batched(voff, rp, ci)
    colors = colors.cpu().numpy()
    ncol = ncol.cpu().numpy()
    for i, p in enumerate(parts):
        ref = oracle.sgr(p.n, p.rowptr, p.colidx)
        assert (colors[b.voff[i]:b.voff[i + 1]] == ref.colors).all(), i
        assert ncol[i] == ref.ncolors


def test_batched_rejects_cross_graph_arcs(dev):
    from paper_1606_06025_amd import _lib as L, api
    g = gg.cycle(6)
    voff = torch.tensor([0, 3, 6], dtype=torch.int64, device=dev)
    with pytest.raises(L.CsrColorError) as e:
        api.color_batched(voff, torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.colidx).to(dev))
    assert e.value.status == L.EBADCSR


def test_batched_validation_finds_every_cross_arc(dev):
    """The batch check spreads the arcs over the grid in fixed chunks and finds each
    chunk's graph by binary search: a union with empty graphs at the start, middle and
    end and a graph spanning many chunks passes (and colours as its parts do), and one
    arc moved into another graph is rejected wherever it sits (chunk edges, graph
    edges, first and last arc)."""
    import oracle
    from paper_1606_06025_amd import _lib as L, api
    parts = [gg.edgeless(3), gg.erdos_renyi(900, 5000, 7, 1), gg.edgeless(0), gg.rmat(12, 8, 3),
             gg.edgeless(5), gg.cycle(9), gg.edgeless(2)]
    b = gg.concat_graphs(parts)
    voff = torch.from_numpy(b.voff).to(dev)
    rp = torch.from_numpy(b.rowptr).to(dev)
    colors, ncol = api.color_batched(voff, rp, torch.from_numpy(b.colidx).to(dev))
    colors = colors.cpu().numpy()
    for i, p in enumerate(parts):
        if p.n:
            ref = oracle.sgr(p.n, p.rowptr, p.colidx)
            assert (colors[b.voff[i]:b.voff[i + 1]] == ref.colors).all(), i
    first = [int(b.rowptr[b.voff[i]]) for i in range(len(parts) + 1)]
    owner = np.searchsorted(np.array(first), np.arange(b.nnz), side="right") - 1
    spots = {0, 4095, 4096, 4097, 8191, 8192, b.nnz - 1}
    for i in range(len(parts)):
        if first[i + 1] > first[i]:
            spots |= {first[i], first[i + 1] - 1}
    for e in sorted(x for x in spots if 0 <= x < b.nnz):
        g = owner[e]
        ci = b.colidx.copy()
        # a vertex just outside graph g (below its range, or above it for the first graph)
        ci[e] = b.voff[g] - 1 if b.voff[g] > 0 else b.voff[g + 1]
        with pytest.raises(L.CsrColorError) as err:
            api.color_batched(voff, rp, torch.from_numpy(ci).to(dev))
        assert err.value.status == L.EBADCSR, e


@pytest.mark.parametrize("shift", [0, 1, 2, 3])
def test_validation_at_every_alignment(dev, shift):
    """The arc check streams colidx as aligned 16-byte quads: at every offset of the
    array it finds an out-of-range first or last entry, and a descent inside a row at
    quad, wavefront and loop-pass boundaries (unsorted rows, same colouring)."""
    import oracle
    from paper_1606_06025_amd import _lib as L, api
    g = gg.erdos_renyi(6000, 60000, shift + 1)
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    rp = torch.from_numpy(g.rowptr).to(dev)

    def view(ci):
        buf = torch.zeros(len(ci) + 8, dtype=torch.int32, device=dev)
        buf[shift:shift + len(ci)] = torch.from_numpy(ci).to(dev)
        v = buf[shift:shift + len(ci)]
        assert v.data_ptr() % 16 == 4 * shift
        return v

    colors, nc, st = api.color(rp, view(g.colidx), stats=True)
    assert st.rows_sorted and nc == ref.ncolors
    row = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    for t in [1, 3, 4, 5, 255, 256, 257, 1023, 1024, 4095, 65536, g.nnz - 1]:
        p = t - 1 if row[t - 1] == row[t] else t - 2     # swap positions p, p + 1 of one row
        assert row[p] == row[p + 1] and g.colidx[p] < g.colidx[p + 1]
        ci = g.colidx.copy()
        ci[p], ci[p + 1] = ci[p + 1], ci[p]
        colors, nc, st = api.color(rp, view(ci), stats=True)
        assert not st.rows_sorted, t
        assert (colors.cpu().numpy() == ref.colors).all() and nc == ref.ncolors
    for pos in [0, g.nnz - 1]:
        for bad in [-1, g.n]:
            ci = g.colidx.copy()
            ci[pos] = bad
            with pytest.raises(L.CsrColorError) as e:
                api.color(rp, view(ci))
            assert e.value.status == L.EBADCSR


@pytest.mark.parametrize("case", ["wake", "classic", "topo", "jp"])
def test_kernel_timing_stats(dev, case):
    """With time_kernels every per-round kernel is launched with start and stop events
    its dispatch stamps: the colouring is unchanged, every launch is counted, and the
    summed kernel times are positive and within the call's wall time."""
    import time
    import oracle
    from paper_1606_06025_amd import api
    g = gg.stencil27(24, 20, 16) if case in ("wake", "topo") else gg.rmat(13, 16, 2)
    kw = {"wake": dict(wake=1), "classic": dict(wake=-1), "topo": dict(algorithm=1),
          "jp": dict(algorithm=2, seed=5)}[case]
    ref = (oracle.jp(g.n, g.rowptr, g.colidx, seed=5) if case == "jp"
           else oracle.sgr(g.n, g.rowptr, g.colidx))
    rp = torch.from_numpy(g.rowptr).to(dev)
    ci = torch.from_numpy(g.colidx).to(dev)
    opts = api.make_opts(**kw)
    api.color(rp, ci, opts=opts)                       # workspace warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colors, nc, st = api.color(rp, ci, opts=opts, stats=True, time_kernels=True)
    wall_ms = (time.perf_counter() - t0) * 1e3
    assert (colors.cpu().numpy() == ref.colors).all() and nc == ref.ncolors
    assert st.n_assign > 0 and st.n_detect > 0
    assert st.n_detect >= ref.rounds - 1
    for ms in (st.ms_setup, st.ms_assign, st.ms_detect):
        assert np.isfinite(ms) and ms > 0
    assert st.ms_setup + st.ms_assign + st.ms_detect <= wall_ms


def _degree_ladder(degs, seed=0):
    """A graph with one hub per requested degree (hub joined to its own leaves) plus a
    random sprinkle of extra edges, so rows of every bucket boundary occur at
    assorted alignments."""
    edges = []
    nxt = len(degs)
    for h, d in enumerate(degs):
        for _ in range(d):
            edges.append((h, nxt))
            nxt += 1
    n = nxt
    h = len(degs)
    # random edges among the leaves only, so every hub keeps exactly its degree
    g0 = gg.random_small(n - h, 2.0 / max(n - h, 1), seed)
    src = np.concatenate([np.array([e[0] for e in edges], np.int64),
                          np.repeat(np.arange(n - h), np.diff(g0.rowptr)) + h])
    dst = np.concatenate([np.array([e[1] for e in edges], np.int64), g0.colidx.astype(np.int64) + h])
    return gg.csr_from_arcs(n, src, dst, symmetrize=True, name="ladder")


def test_bucket_boundary_degrees(dev):
    degs = [1, 2, 4, 5, 6, 7, 12, 13, 14, 15, 28, 29, 30, 31, 60, 61, 62, 63, 64, 65, 127, 128,
            1023, 1024, 1025, 2000]
    for seed in range(3):
        _assert_parity(_degree_ladder(degs, seed), dev)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_misaligned_colidx_view(dev, shift):
    import oracle
    from paper_1606_06025_amd import api
    for g in [gg.erdos_renyi(3000, 40000, shift), _degree_ladder([5, 13, 29, 61, 300, 1500], shift)]:
        ref = oracle.sgr(g.n, g.rowptr, g.colidx)
        buf = torch.zeros(g.nnz + 8, dtype=torch.int32, device=dev)
        buf[shift:shift + g.nnz] = torch.from_numpy(g.colidx).to(dev)
        ci = buf[shift:shift + g.nnz]
        assert ci.data_ptr() % 16 == 4 * shift
        rp = torch.from_numpy(g.rowptr).to(dev)
        colors, nc, st = api.color(rp, ci, stats=True)
        assert (colors.cpu().numpy() == ref.colors).all()
        assert nc == ref.ncolors and st.rounds == ref.rounds


@pytest.mark.parametrize("n", [1030, 1500])
def test_split_rows_beyond_hub_bitmap(dev, n):
    """With t_split at its minimum every vertex of K_n (degree n-1 > 1024) is a split
    row, and its colour exceeds the 1024 colours a hub bitmap covers."""
    got, ref = _assert_parity(gg.complete(n), dev, t_split=1024, t_wave=61)
    assert got.tolist() == list(range(n))


def test_split_rows_ladder(dev):
    degs = [2047, 2048, 2049, 3000, 4096, 4097, 9000, 20000]
    for seed in range(2):
        g = _degree_ladder(degs, seed)
        _assert_parity(g, dev)
        _assert_parity(g, dev, t_split=1024)


def test_split_rmat(dev):
    g = gg.rmat(16, 16, 5)
    import oracle
    ref = oracle.sgr(g.n, g.rowptr, g.colidx)
    for kw in [dict(), dict(t_split=1024), dict(t_split=1 << 20), dict(t_wave=61, t_split=1024)]:
        _assert_parity(g, dev, ref, **kw)


def _golden(name):
    import json
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", f"{name}_s1.json")
    if not os.path.exists(p):
        pytest.skip(f"{p} not generated")
    with open(p) as f:
        return json.load(f)


def _digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def test_config_rmat23_full_against_stored_oracle(dev):
    """R-MAT scale 23 at full size: the oracle takes minutes here, so its result was
    stored (tests/golden/make_golden.py) as digests plus per-round statistics."""
    gold = _golden("rmat23")
    g = gg.config_rmat23(1)
    assert _digest(g.rowptr) == gold["rowptr_sha256"] and _digest(g.colidx) == gold["colidx_sha256"]
    got, nc, st = _run(g, dev)
    assert nc == gold["ncolors"] and st.rounds == gold["rounds"]
    assert st.wsize == gold["wsize"] and st.arcs == gold["arcs_ff"]
    assert _digest(got) == gold["colors_sha256"]


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_drive_modes_match_oracle(dev, mode):
    """Host loop (1), one persistent cooperative launch (2) and replayed hipGraph
    rounds (3) give the oracle's colouring, round count and per-round statistics."""
    graphs = [gg.erdos_renyi(20000, 160000, 3), gg.rmat(13, 16, 2), gg.stencil27(20, 17, 9),
              gg.complete(70), gg.star(1500, [i for i in range(3001) if i != 1500]),
              _degree_ladder([5, 13, 29, 61, 300, 1500, 2500, 9000], 1), gg.cycle(101), gg.edgeless(9)]
    for g in graphs:
        _assert_parity(g, dev, mode=mode)


@pytest.mark.parametrize("mode", [2, 3])
def test_drive_modes_repeat_and_shrink(dev, mode):
    """Consecutive calls in one mode, the second on a smaller graph (graph mode must
    not replay a capture made for other arguments)."""
    for g in [gg.erdos_renyi(30000, 300000, 8), gg.erdos_renyi(30000, 300000, 8), gg.erdos_renyi(5000, 30000, 9),
              gg.rmat(12, 8, 3)]:
        _assert_parity(g, dev, mode=mode)


@pytest.mark.parametrize("firstfit", [1, 2, 3])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_firstfit_variants_match_oracle(dev, firstfit, mode):
    """FirstFit by rescanning neighbour colours every round (1) and by per-vertex
    forbidden bitmaps filled when neighbours settle (2) give the oracle's colouring
    in every drive mode, including hubs that win round 1 (star centred at 0)."""
    graphs = [gg.erdos_renyi(20000, 160000, 4), gg.rmat(14, 16, 6), gg.stencil27(21, 13, 11),
              gg.complete(90), gg.star(0, list(range(1, 40001))),
              _degree_ladder([5, 13, 29, 61, 300, 1500, 2500, 9000], 2), gg.cycle(77)]
    for g in graphs:
        _assert_parity(g, dev, mode=mode, firstfit=firstfit)


@pytest.mark.parametrize("firstfit", [1, 2, 3])
def test_firstfit_variants_split_heavy(dev, firstfit):
    g = gg.rmat(16, 16, 11)
    _assert_parity(g, dev, firstfit=firstfit, t_split=1024, t_wave=61)
    got, ref = _assert_parity(gg.complete(1300), dev, firstfit=firstfit, t_split=1024)
    assert got.tolist() == list(range(1300))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_degree_rule_matches_oracle(dev, mode):
    """Heuristic conflict resolve (Sec. 3.2): the smaller degree is requeued, the
    higher id on equal degree; bit-exact against the oracle's rule 1."""
    for g in [gg.from_edges(6, [(5, k) for k in range(5)]), gg.path(4),
              gg.from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)]),
              gg.erdos_renyi(20000, 160000, 5), gg.rmat(14, 16, 7), gg.stencil27(12, 9, 7),
              _degree_ladder([5, 13, 29, 61, 300, 1500, 2500, 9000], 3),
              gg.shuffle_rows(gg.rmat(12, 16, 8), 2)]:
        for ff in (1, 2):
            _assert_parity(g, dev, rule=1, mode=mode, firstfit=ff)


def _one_beater_graph(D, p, rule):
    """Hub H of degree D whose only beater sits at position p of H's row; the other
    neighbours are leaves.  Degree rule: sorted rows, the beater B has degree D + 1
    (ids: leaves 0..p-1, B = p, leaves p+1..D-1, H = D, B's own leaves after H).  Id
    rule: H = 1, the beater is vertex 0, every other neighbour has a higher id, and H's
    row lists them in descending order with 0 at position p (unsorted rows)."""
    if rule == 1:
        H, B = D, p
        edges = [(H, x) for x in range(D)] + [(B, D + 1 + k) for k in range(D)]
        g = gg.from_edges(2 * D + 1, edges, name=f"beater_r1_D{D}_p{p}")
        row = g.colidx[g.rowptr[H]:g.rowptr[H + 1]]
        assert row[p] == B and int(np.diff(g.rowptr)[B]) == D + 1
        return g
    n = D + 1
    others = list(range(n - 1, 1, -1))            # D - 1 higher neighbours, descending
    hub_row = others[:p] + [0] + others[p:]
    rows = {0: [1], 1: hub_row}
    for x in others:
        rows[x] = [1]
    rowptr = np.zeros(n + 1, np.int32)
    for v in range(n):
        rowptr[v + 1] = rowptr[v] + len(rows[v])
    colidx = np.concatenate([np.asarray(rows[v], np.int32) for v in range(n)])
    return gg.CSR(n, rowptr, colidx, f"beater_r0_unsorted_D{D}_p{p}")


@pytest.mark.parametrize("rule", [0, 1])
def test_round1_scan_finds_the_only_beater(dev, rule):
    """Without the id rule's first-arc test (degree rule, unsorted rows) round 1 scans a
    row up to its first beater: one lane up to 64 arcs, the wavefront up to 4096, the
    workgroup beyond, 256 or 1024 entries a step.  A hub whose only beater sits at a
    lane, step or workgroup boundary (or at the row's end) must lose in round 1, as in
    the oracle; a missed beater makes it a round-1 winner and changes the colouring."""
    for D in (40, 65, 300, 4096, 4097, 5000):
        for p in sorted({0, 3, 4, 63, 64, 255, 256, 1023, 1024, 4095, 4096, D - 1}):
            if p < D:
                _assert_parity(_one_beater_graph(D, p, rule), dev, rule=rule)


def test_degree_rule_split_and_unsorted(dev):
    g = gg.rmat(16, 16, 13)
    _assert_parity(g, dev, rule=1, t_split=1024, t_wave=61)
    _assert_parity(gg.shuffle_rows(g, 5), dev, rule=1)


@pytest.mark.parametrize("hints", [-1, 1])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_conflict_hints_on_and_off(dev, hints, mode):
    """The conflict test may first check the neighbour that requeued a vertex before;
    on or off, every bucket (tiles, lanes, wavefront, workgroup, split rows) and every
    drive mode gives the oracle's colouring, also with unsorted rows."""
    graphs = [gg.stencil27(24, 20, 16), gg.rmat(14, 16, 7),
              _degree_ladder([5, 13, 29, 61, 300, 1500, 2500, 9000], 5),
              gg.shuffle_rows(gg.erdos_renyi(20000, 200000, 6), 3), gg.complete(200)]
    for g in graphs:
        _assert_parity(g, dev, mode=mode, hints=hints)
        _assert_parity(g, dev, mode=mode, hints=hints, lane_detect=-1, t_wave=128, t_split=1024)


@pytest.mark.parametrize("live", [-1, 1])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_live_lists_on_and_off(dev, live, mode):
    """Vertices of degree > 61 may test lists of their still-uncoloured lower neighbours
    instead of their rows (wavefront, workgroup and split-row buckets); on or off, with
    hints on or off, sorted or unsorted rows, the colouring is the oracle's."""
    graphs = [gg.rmat(14, 16, 8), gg.complete(200), gg.complete(1100),
              _degree_ladder([61, 62, 300, 1024, 1025, 2048, 2049, 5000, 9000], 6),
              gg.star(3000, [i for i in range(6001) if i != 3000]),
              gg.shuffle_rows(gg.rmat(13, 16, 4), 5)]
    for g in graphs:
        _assert_parity(g, dev, mode=mode, live_lists=live)
        _assert_parity(g, dev, mode=mode, live_lists=live, hints=-1, t_wave=128, t_split=1024)


@pytest.mark.parametrize("mode", [1, 3])
@pytest.mark.parametrize("wake", [-1, 1])
@pytest.mark.parametrize("live", [-1, 1])
def test_wake_flags_on_and_off(dev, wake, live, mode):
    """A requeued vertex may be left untested until its colour or that of its conflict
    hint changes; on or off, with live lists on or off, bit or byte flags, every bucket
    (tiles, lanes, wavefront, workgroup, split rows), sorted or unsorted rows, in the
    host loop and in rounds replayed from a captured graph (whose kernels read the
    round number from the device), the colouring, the rounds and the per-round worklist
    sizes are the oracle's."""
    graphs = [gg.stencil27(24, 20, 16), gg.rmat(14, 16, 12), gg.complete(300),
              _degree_ladder([5, 13, 29, 61, 62, 300, 1024, 1025, 2500, 9000], 7),
              gg.star(3000, [i for i in range(6001) if i != 3000]),
              gg.shuffle_rows(gg.erdos_renyi(20000, 200000, 8), 4), gg.cycle(1001)]
    for g in graphs:
        _assert_parity(g, dev, wake=wake, live_lists=live, mode=mode)
        _assert_parity(g, dev, wake=wake, live_lists=live, mode=mode, firstfit=2, lane_detect=-1, t_wave=128,
                       t_split=1024)


def test_wake_flags_repeated_entries(dev):
    """Rows that repeat an entry (sorted or not, with self-loops) would let a recoloured
    vertex wake the same sleeper twice; the colouring and the statistics stay the
    oracle's."""
    base = gg.stencil27(12, 11, 10)
    for shuffle in (False, True):
        rows = []
        for v in range(base.n):
            r = base.colidx[base.rowptr[v]:base.rowptr[v + 1]].tolist()
            r = sorted(r + r[::3] + [v])
            rows.append(r[::-1] if shuffle else r)
        _assert_parity(gg.raw_csr(base.n, rows), dev)


def test_wake_flags_workspace_reuse(dev):
    """Consecutive runs of different sizes share the stamps and recolour lists of the
    workspace: stale entries of an earlier run must never be taken for this one's."""
    seq = [gg.stencil27(20, 20, 20), gg.rmat(13, 16, 3), gg.stencil27(9, 8, 7), gg.erdos_renyi(5000, 40000, 2),
           gg.stencil27(20, 20, 20)]
    for g in seq:
        _assert_parity(g, dev)


@pytest.mark.parametrize("n", [262144, 262145, 524289, 1048577])
def test_wake_flags_scan_widths(dev, n):
    """The flag scans take 64, 128, 256 or 512 vertices per wavefront by graph size;
    sizes at and just past each step give the oracle's colouring, including the padded
    tail of the last scan."""
    _assert_parity(gg.erdos_renyi(n, 4 * n, n % 97), dev, wake=1)


def test_wake_flags_byte_counting(dev):
    """The counting instantiations of the wake kernels colour exactly like the timed
    ones and report bytes; runs without wake flags report none."""
    import oracle
    from paper_1606_06025_amd import api
    for g, wake in [(gg.stencil27(30, 20, 10), 0), (gg.rmat(13, 16, 5), 1), (gg.rmat(13, 16, 5), -1)]:
        ref = oracle.sgr(g.n, g.rowptr, g.colidx)
        rp = torch.from_numpy(g.rowptr).to(dev)
        ci = torch.from_numpy(g.colidx).to(dev)
        colors, nc, st = api.color(rp, ci, opts=api.make_opts(wake=wake), stats=True, count_bytes=True)
        assert (colors.cpu().numpy() == ref.colors).all() and nc == ref.ncolors
        assert st.rounds == ref.rounds
        if wake >= 0:
            assert st.kernel_bytes[0] > 0 and st.kernel_bytes[1] > 0
        else:
            assert st.kernel_bytes == [0, 0]


def test_live_lists_workspace_reuse(dev):
    """Consecutive runs reuse the live-list buffers: stale lists of an earlier graph
    must never be read as built lists of the next one."""
    seq = [gg.rmat(14, 16, 9), gg.rmat(14, 16, 10), gg.rmat(12, 8, 11), gg.rmat(14, 16, 9)]
    for g in seq:
        _assert_parity(g, dev)


@pytest.mark.parametrize("ordered", [-1, 1])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_ordered_compaction_on_and_off(dev, ordered, mode):
    """Blocks may take tickets and place their losers after those of lower tickets
    (look-back prefix) so the worklist keeps id order; on or off, in every drive mode
    and with more blocks than fit on the device at once, the colouring is the oracle's."""
    graphs = [gg.stencil27(64, 64, 64), gg.rmat(16, 16, 12), gg.erdos_renyi(300000, 2400000, 13),
              _degree_ladder([5, 13, 29, 61, 300, 1500, 2500], 7), gg.edgeless(5000)]
    for g in graphs:
        _assert_parity(g, dev, mode=mode, ordered=ordered)
    if mode == 1:
        for kw in (dict(blocks_per_cu=1), dict(blocks_per_cu=32), dict(sync_every=1, blocks_per_cu=2)):
            _assert_parity(graphs[0], dev, ordered=ordered, **kw)
            _assert_parity(graphs[1], dev, ordered=ordered, **kw)

"""C-ABI library: loads, exports every declared symbol, and host-side argument checks
(no GPU work is issued by these calls)."""
import ctypes
import os
import re

import pytest

from paper_1606_06025_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csrcolor.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(csrcolor_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1606_06025_amd import build
        build.build()
    return L.load()


def test_header_declares_expected_entry_points():
    assert _declared() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(L.LIB_PATH)
    for name in _declared():
        assert hasattr(raw, name), name


def test_version_and_strerror(lib):
    assert lib.csrcolor_version() >= 100
    for code in [L.OK, L.EINVAL, L.EBADCSR, L.ENOMEM, L.EHIP, L.EOVERFLOW, L.ENOTSYM, L.ELIMIT, L.ETIMEOUT,
                 L.ETOOBIG]:
        assert lib.csrcolor_strerror(code)
    assert b"unknown" in lib.csrcolor_strerror(12345)


def test_argument_errors_without_device_work(lib):
    nc = ctypes.c_int32(-1)
    assert lib.csrcolor_color(-1, None, None, None, ctypes.byref(nc), None) == L.EINVAL
    assert lib.csrcolor_color(5, None, None, None, ctypes.byref(nc), None) == L.EINVAL
    assert lib.csrcolor_color(5, 1, 1, 1, None, None) == L.EINVAL
    assert lib.csrcolor_color(5, 1, 1, None, ctypes.byref(nc), None) == L.EINVAL
    assert lib.csrcolor_color_batched(-1, 0, None, None, None, None, None, None, None) == L.EINVAL
    assert lib.csrcolor_color_batched(0, 3, None, None, None, None, None, None, None) == L.EINVAL
    assert lib.csrcolor_color_batched(0, 0, None, None, None, None, None, None, None) == L.OK
    bad = L.Opts()
    bad.mode = 99
    assert lib.csrcolor_color_ex(3, 1, 1, 1, None, ctypes.byref(bad), None, None) == L.EINVAL


def test_empty_graph_is_host_only(lib):
    nc = ctypes.c_int32(-1)
    assert lib.csrcolor_color(0, None, None, None, ctypes.byref(nc), None) == L.OK
    assert nc.value == 0
    st = L.Stats()
    # the colour count of csrcolor_color_ex is a device pointer: none is passed here
    assert lib.csrcolor_color_ex(0, None, None, None, None, None, ctypes.byref(st), None) == L.OK
    assert st.rounds == 0 and st.ncolors == 0
    # the asynchronous (device-planned) form of an empty graph touches no memory either
    assert lib.csrcolor_color_ex(0, None, None, None, None, None, None, None) == L.OK


def test_algorithm_option_errors_without_device_work(lib):
    def opts(**kw):
        o = L.Opts()
        for k, v in kw.items():
            setattr(o, k, v)
        return ctypes.byref(o)
    ex = lambda o: lib.csrcolor_color_ex(3, 1, 1, 1, None, o, None, None)
    assert ex(opts(algorithm=3)) == L.EINVAL
    assert ex(opts(algorithm=-1)) == L.EINVAL
    assert ex(opts(rule=2)) == L.EINVAL
    assert ex(opts(firstfit=4)) == L.EINVAL
    assert ex(opts(hints=2)) == L.EINVAL
    assert ex(opts(hints=-2)) == L.EINVAL
    assert ex(opts(live_lists=2)) == L.EINVAL
    assert ex(opts(ordered=-3)) == L.EINVAL
    assert ex(opts(wake=2)) == L.EINVAL
    assert ex(opts(wake=-2)) == L.EINVAL
    assert ex(opts(tile_limits=6 | (13 << 8) | (29 << 16))) == L.EINVAL    # t0 above 5
    assert ex(opts(tile_limits=5 | (4 << 8) | (29 << 16))) == L.EINVAL     # not non-decreasing
    assert ex(opts(tile_limits=5 | (13 << 8) | (30 << 16))) == L.EINVAL    # t2 above 29
    assert ex(opts(tile_limits=1 << 24)) == L.EINVAL
    for algo in (L.ALGO_SGR_TOPO, L.ALGO_JP):
        for mode in (L.MODE_PERSISTENT, L.MODE_GRAPH):
            assert ex(opts(algorithm=algo, mode=mode)) == L.EINVAL
    # JP priorities depend on global ids, so the batched and multi entry points refuse it
    assert lib.csrcolor_color_batched(1, 3, 1, 1, 1, 1, 1, opts(algorithm=L.ALGO_JP), None) == L.EINVAL
    assert lib.csrcolor_color_batched(1, 3, 1, 1, 1, 1, 1, opts(rule=5), None) == L.EINVAL
    n = (ctypes.c_int32 * 1)(3)
    m = (ctypes.c_int64 * 1)(0)
    p = (ctypes.c_void_p * 1)(1)
    assert lib.csrcolor_color_multi(1, n, m, p, p, p, 1, opts(algorithm=L.ALGO_JP), None) == L.EINVAL


def _header_struct_fields(name):
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", txt).group(1)
    return re.findall(r"\b(\w+)\s*(?:\[\d+\])?;", body)


def test_struct_layouts_match_header():
    # csrcolor_opts: 18 x 32-bit fields (10 options, algorithm, two seed halves, hints, live lists, ordered,
    # wake lists, tile limits)
    # csrcolor_stats: 4 int32, int64, 2 int32, 2 pointers, 3 double, 2 int32, a pointer
    assert ctypes.sizeof(L.Opts) == 18 * 4
    assert ctypes.sizeof(L.Stats) == 4 * 4 + 8 + 2 * 4 + 2 * 8 + 3 * 8 + 2 * 4 + 8
    assert _header_struct_fields("csrcolor_opts") == [f[0] for f in L.Opts._fields_]
    assert _header_struct_fields("csrcolor_stats") == [f[0] for f in L.Stats._fields_]


def test_noalloc_limits_without_device_work(lib):
    """The allocation-free entry point refuses sizes above its fixed maxima, and bad
    arguments, before it touches the device; an empty graph with no count slot is a
    no-op."""
    assert lib.csrcolor_color_noalloc(L.NOALLOC_MAX_N + 1, 0, 1, 1, 1, None, None) == L.ETOOBIG
    assert lib.csrcolor_color_noalloc(3, L.NOALLOC_MAX_NNZ + 1, 1, 1, 1, None, None) == L.ETOOBIG
    assert lib.csrcolor_color_noalloc(-1, 0, None, None, None, None, None) == L.EINVAL
    assert lib.csrcolor_color_noalloc(3, -1, 1, 1, 1, None, None) == L.EINVAL
    assert lib.csrcolor_color_noalloc(3, 4, None, 1, 1, None, None) == L.EINVAL
    assert lib.csrcolor_color_noalloc(3, 4, 1, None, 1, None, None) == L.EINVAL
    assert lib.csrcolor_color_noalloc(3, 4, 1, 1, None, None, None) == L.EINVAL
    assert lib.csrcolor_color_noalloc(0, 0, None, None, None, None, None) == L.OK


def test_noalloc_limits_match_header():
    txt = open(HEADER).read()
    assert re.search(r"#define CSRCOLOR_NOALLOC_MAX_N\s+%d\b" % L.NOALLOC_MAX_N, txt)
    assert re.search(r"#define CSRCOLOR_NOALLOC_MAX_NNZ\s+%d\b" % L.NOALLOC_MAX_NNZ, txt)


def test_workspace_bytes_query(lib):
    """The workspace bound grows with the vertices, the arcs and the union copy, and is
    at least the per-vertex and per-arc arrays the library allocates."""
    wb = lib.csrcolor_workspace_bytes
    assert wb(0, -1, 0) == L.EINVAL and wb(-1, 10, 10) == L.EINVAL and wb(0, 10, -5) == L.EINVAL
    n, m = 1 << 20, 1 << 24
    base = wb(0, n, m)
    assert base > 0 and wb(0, n + 4096, m) > base and wb(0, n, m + 4096) > base
    assert wb(3, n, m) >= base + 4 * (2 * n + m)          # the union's CSR copy and colours
    assert base >= 55 * n + 5 * m                          # colour state, lists, flags, live lists
    assert lib.csrcolor_device_bytes_in_use() >= 0

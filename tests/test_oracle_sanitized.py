"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code,
gcc): a small driver runs every oracle entry point (both conflict rules, the
topology-driven rounds, JP, serial FirstFit, the two checkers) on assorted graphs,
including statistics arrays shorter than the run, self-loops, duplicate arcs, unsorted
rows and an out-of-range id.  The run must end cleanly, and its results must equal the
ordinary build's, so the oracle's results do not depend on reads outside its arrays."""
import os
import struct
import subprocess

import numpy as np
import pytest

import oracle
from paper_1606_06025_amd import graphs as gg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sgr_capped(int32_t, const int32_t *, const int32_t *, int32_t *, int32_t *, int32_t *,
                      int64_t *, int64_t *, int64_t *, int32_t, int32_t, int32_t);
int oracle_sgr_topo(int32_t, const int32_t *, const int32_t *, int32_t *, int32_t *, int32_t *,
                    int64_t *, int64_t *, int32_t, int32_t);
int oracle_jp(int32_t, const int32_t *, const int32_t *, uint64_t, int32_t *, int32_t *, int32_t *,
              int64_t *, int64_t *, int32_t);
int oracle_serial_ff(int32_t, const int32_t *, const int32_t *, int32_t *, int32_t *);
int64_t oracle_count_conflicts(int32_t, const int32_t *, const int32_t *, const int32_t *);
int64_t oracle_count_non_grundy(int32_t, const int32_t *, const int32_t *, const int32_t *);

static void put(FILE *f, int32_t rc, int32_t nc, int32_t rounds, const int32_t *c, int32_t n) {
    fwrite(&rc, 4, 1, f);
    fwrite(&nc, 4, 1, f);
    fwrite(&rounds, 4, 1, f);
    if (n > 0) fwrite(c, 4, (size_t)n, f);
}

int main(int argc, char **argv) {
    FILE *in = fopen(argv[1], "rb"), *out = fopen(argv[2], "wb");
    const int32_t cap = atoi(argv[3]);
    if (!in || !out) return 2;
    int32_t n;
    int64_t nnz;
    while (fread(&n, 4, 1, in) == 1) {
        if (fread(&nnz, 8, 1, in) != 1) return 3;
        /* exact-size allocations, so any read past an array end is reported */
        int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
        int32_t *ci = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        int32_t *c = calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
        int64_t *s1 = malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
        int64_t *s2 = malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
        int64_t *s3 = malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
        if (fread(rp, 4, (size_t)(n + 1), in) != (size_t)(n + 1)) return 4;
        if (nnz > 0 && fread(ci, 4, (size_t)nnz, in) != (size_t)nnz) return 5;
        int32_t nc = 0, r = 0;
        for (int rule = 0; rule <= 1; ++rule) {
            int rc = oracle_sgr_capped(n, rp, ci, c, &nc, &r, s1, s2, s3, cap, rule, 0);
            put(out, rc, nc, r, c, n);
            rc = oracle_sgr_topo(n, rp, ci, c, &nc, &r, s1, s2, cap, rule);
            put(out, rc, nc, r, c, n);
        }
        int rc = oracle_jp(n, rp, ci, 12345u, c, &nc, &r, s1, s2, cap);
        put(out, rc, nc, r, c, n);
        rc = oracle_serial_ff(n, rp, ci, c, &nc);
        put(out, rc, nc, 0, c, n);
        if (rc == 0) {
            int64_t k1 = oracle_count_conflicts(n, rp, ci, c), k2 = oracle_count_non_grundy(n, rp, ci, c);
            fwrite(&k1, 8, 1, out);
            fwrite(&k2, 8, 1, out);
        }
        free(rp); free(ci); free(c); free(s1); free(s2); free(s3);
    }
    fclose(in);
    fclose(out);
    return 0;
}
"""

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _graphs():
    g_dup = gg.from_edges(6, [(0, 1), (1, 2), (2, 0), (3, 4)])
    # a duplicate arc and a self-loop written into the CSR by hand
    rp = np.array([0, 3, 5, 7, 8, 9, 10], np.int32)
    ci = np.array([1, 1, 2, 0, 2, 0, 1, 4, 3, 5], np.int32)
    assert rp[-1] == len(ci)
    loops = gg.CSR(6, rp, ci, "dup_and_loop")
    bad = gg.CSR(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 7], np.int32), "id_out_of_range")
    return [gg.cycle(5), gg.cycle(8), gg.complete(12), gg.path(4), gg.edgeless(7), gg.edgeless(0),
            gg.star(3, [0, 1, 2, 4, 5]), g_dup, loops, gg.erdos_renyi(3000, 20000, 3),
            gg.rmat(11, 8, 2), gg.stencil27(7, 6, 5), gg.shuffle_rows(gg.rmat(10, 16, 4), 1), bad]


def _reference(g, cap):
    """The same calls through the ordinary build (ctypes)."""
    import ctypes
    lib = oracle._load()
    n = g.n
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rp = np.ascontiguousarray(g.rowptr, np.int32)
    ci = np.ascontiguousarray(g.colidx if len(g.colidx) else np.zeros(1, np.int32), np.int32)
    c = np.zeros(max(n, 1), np.int32)
    nc = np.zeros(1, np.int32)
    r = np.zeros(1, np.int32)
    s = [np.zeros(max(cap, 1), np.int64) for _ in range(3)]
    out = []
    for rule in (0, 1):
        rc = lib.oracle_sgr_capped(n, P(rp), P(ci), P(c), P(nc), P(r), P(s[0]), P(s[1]), P(s[2]), cap, rule, 0)
        out.append((rc, int(nc[0]), int(r[0]), c[:n].copy()))
        rc = lib.oracle_sgr_topo(n, P(rp), P(ci), P(c), P(nc), P(r), P(s[0]), P(s[1]), cap, rule)
        out.append((rc, int(nc[0]), int(r[0]), c[:n].copy()))
    rc = lib.oracle_jp(n, P(rp), P(ci), 12345, P(c), P(nc), P(r), P(s[0]), P(s[1]), cap)
    out.append((rc, int(nc[0]), int(r[0]), c[:n].copy()))
    rc = lib.oracle_serial_ff(n, P(rp), P(ci), P(c), P(nc))
    out.append((rc, int(nc[0]), 0, c[:n].copy()))
    checks = None
    if rc == 0:
        checks = (int(lib.oracle_count_conflicts(n, P(rp), P(ci), P(c))),
                  int(lib.oracle_count_non_grundy(n, P(rp), P(ci), P(c))))
    return out, checks


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_san")
    probe = d / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    try:
        subprocess.run(["gcc"] + SAN + ["-o", str(d / "probe"), str(probe)], check=True,
                       capture_output=True, timeout=120)
    except (subprocess.CalledProcessError, FileNotFoundError, subprocess.TimeoutExpired):
        pytest.skip("gcc with AddressSanitizer / UndefinedBehaviorSanitizer is not available")
    src = d / "driver.c"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["gcc", "-std=c11"] + SAN + ["-o", str(exe), str(src),
                    os.path.join(ROOT, "oracle", "sgr_oracle.c"), os.path.join(ROOT, "oracle", "jp_oracle.c")],
                   check=True, capture_output=True, timeout=300)
    return d, exe


@pytest.mark.parametrize("cap", [2, 1 << 12])
def test_sanitized_oracle_equals_ordinary_build(driver, cap):
    d, exe = driver
    gs = _graphs()
    inp = d / f"graphs_{cap}.bin"
    with open(inp, "wb") as f:
        for g in gs:
            f.write(struct.pack("<iq", g.n, int(g.rowptr[-1]) if g.n else 0))
            f.write(np.ascontiguousarray(g.rowptr, np.int32).tobytes())
            f.write(np.ascontiguousarray(g.colidx, np.int32).tobytes())
    outp = d / f"results_{cap}.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe), str(inp), str(outp), str(cap)], capture_output=True, text=True, env=env,
                         timeout=600)
    assert run.returncode == 0, run.stderr[-3000:]
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr, run.stderr[-3000:]
    buf = outp.read_bytes()
    pos = 0

    def take(fmt, k=1):
        nonlocal pos
        size = struct.calcsize(fmt) * k
        vals = struct.unpack_from("<" + fmt * k, buf, pos)
        pos += size
        return vals

    for g in gs:
        ref, checks = _reference(g, cap)
        for (rc, nc, rounds, colors) in ref:
            got_rc, got_nc, got_r = take("i", 3)
            got_c = np.array(take("i", g.n), np.int32) if g.n else np.zeros(0, np.int32)
            assert (got_rc, got_nc, got_r) == (rc, nc, rounds), g.name
            if rc == 0:
                assert np.array_equal(got_c, colors), g.name
        if checks is not None:
            assert take("q", 2) == checks, g.name
    assert pos == len(buf)

"""Seeded synthetic graph generators (input data only).

This module produces the undirected int32 CSR inputs that both the GPU path and
the CPU oracle consume.  It holds none of the coloring arithmetic: it only draws
random numbers, builds edge lists and packs them into symmetric, self-loop-free,
duplicate-free CSR with sorted rows.

Randomness is counter-based (SplitMix64, Steele/Lea/Flood 2014, as finalised by
Vigna): the i-th draw of stream `key` is ``mix64(key + (i + 1) * GOLDEN)``, so
every value is a pure function of (seed, stream, index) and chunked generation is
bit-identical to whole-array generation.

Workload families (the paper evaluates on R-MAT graphs and sparse matrices, Sec. 4,
Table 1; the sparse-matrix collection is not available here, so these synthetic
families stand in for it):
  * Erdos-Renyi G(n, m) by uniform endpoint pairs (the paper's rmat-er is R-MAT
    with a=b=c=d=0.25, which is the same uniform-endpoint model);
  * 3D 27-point stencil graphs (regular meshes such as thermal2 / atmosmodd);
  * R-MAT (Sec. 4, recursive quadrant sampling with parameters (a, b, c, d));
  * a batched set of many small ER and stencil graphs in one block-diagonal CSR;
  * a Poisson request stream of R-MAT / ER graphs for the serving loop.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Sequence, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_U64 = np.uint64

# Stream identifiers keep the draws of different purposes independent.
STREAM_ER_PAIRS = 1
STREAM_RMAT_BITS = 2
STREAM_RMAT_PERM = 3
STREAM_BATCH_SPEC = 4
STREAM_SERVE_SPEC = 5
STREAM_FUZZ = 6


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _U64(30))) * _M1
        z = (z ^ (z >> _U64(27))) * _M2
    return z ^ (z >> _U64(31))


def stream_key(seed: int, stream: int, sub: int = 0) -> np.uint64:
    """Derive the 64-bit key of one random stream from (seed, stream, sub)."""
    k = mix64(np.array([(seed * 0x100000001B3 + stream * 0x5851F42D4C957F2D + sub)
                        & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
    return k[0]


def draws(key: np.uint64, start: int, count: int) -> np.ndarray:
    """Counter-based uint64 draws number start .. start+count-1 of stream `key`."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(idx * _GOLDEN + key)


def _bounded(u32: np.ndarray, bound: int) -> np.ndarray:
    """Map uniform 32-bit values to [0, bound) by multiply-shift."""
    return ((u32.astype(np.uint64) * _U64(bound)) >> _U64(32)).astype(np.int64)


# ----------------------------------------------------------------------------
# CSR container and packing
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class CSR:
    """Undirected graph as symmetric CSR (int32 rowptr[n+1], int32 colidx[nnz])."""
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1]) if self.n > 0 else 0

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def max_degree(self) -> int:
        return int(self.degrees().max()) if self.n > 0 else 0


def csr_from_arcs(n: int, src: np.ndarray, dst: np.ndarray, symmetrize: bool = True,
                  drop_self: bool = True, name: str = "") -> CSR:
    """Pack an arc list into CSR with sorted, duplicate-free rows.

    With ``symmetrize`` every arc (u, v) also contributes (v, u), which makes the
    result the adjacency structure of an undirected graph."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if symmetrize:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    if drop_self:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    key = np.unique(src * np.int64(n) + dst)          # sorts rows and columns, dedups
    s = key // n
    d = (key - s * n).astype(np.int32)
    counts = np.bincount(s, minlength=n).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2 ** 31:
        raise OverflowError("graph has 2^31 or more arcs; int32 CSR cannot hold it")
    return CSR(n, rowptr.astype(np.int32), d, name)


# ----------------------------------------------------------------------------
# Families
# ----------------------------------------------------------------------------

def erdos_renyi(n: int, m: int, seed: int, sub: int = 0) -> CSR:
    """G(n, m) by m endpoint pairs drawn iid uniform on [0, n)^2.

    Self-loops and duplicate pairs are dropped (not resampled), then the pair list is
    symmetrised, so slightly fewer than m undirected edges remain."""
    key = stream_key(seed, STREAM_ER_PAIRS, sub)
    h = draws(key, 0, m)
    u = _bounded(h >> _U64(32), n)
    v = _bounded(h & _U64(0xFFFFFFFF), n)
    return csr_from_arcs(n, u, v, name=f"er_n{n}_m{m}_s{seed}")


def stencil27(X: int, Y: int, Z: int) -> CSR:
    """3D 27-point stencil on an X*Y*Z box, id = x + X*(y + Y*z).

    Every vertex is joined to all of its (up to 26) in-box neighbours at Chebyshev
    distance 1.  No randomness."""
    n = X * Y * Z
    ids = np.arange(n, dtype=np.int64)
    x = ids % X
    y = (ids // X) % Y
    z = ids // (X * Y)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dx, dy, dz) != (0, 0, 0)]
    # offsets in (dz, dy, dx) lexicographic order give increasing neighbour ids for
    # boxes of side >= 3; a final per-row sort makes it hold for any box.
    BIG = np.int64(1) << 40
    nb = np.empty((n, len(offs)), dtype=np.int64)
    for k, (dx, dy, dz) in enumerate(offs):
        ok = ((x + dx >= 0) & (x + dx < X) & (y + dy >= 0) & (y + dy < Y)
              & (z + dz >= 0) & (z + dz < Z))
        nb[:, k] = np.where(ok, ids + dx + X * (dy + Y * dz), BIG)
    if min(X, Y, Z) < 3:
        nb.sort(axis=1)
    valid = nb != BIG
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colidx = nb[valid].astype(np.int32)
    return CSR(n, rowptr.astype(np.int32), colidx, name=f"stencil27_{X}x{Y}x{Z}")


def stencil27_arcs(X: int, Y: int, Z: int) -> int:
    """Closed-form arc count of the 27-point stencil box: sum over axes pairs."""
    # number of ordered pairs at Chebyshev distance <= 1 minus self pairs
    return (3 * X - 2) * (3 * Y - 2) * (3 * Z - 2) - X * Y * Z


RMAT_DEFAULT = (0.57, 0.19, 0.19, 0.05)


def _rmat_chunk(key: np.uint64, start: int, cnt: int, scale: int, nh: int,
                t1: np.uint32, t2: np.uint32, t3: np.uint32) -> Tuple[np.ndarray, np.ndarray]:
    """Endpoints of R-MAT samples start .. start+cnt-1 (uint32 ids).

    Sample s uses draws s*nh + 1 .. s*nh + nh of the stream; each 64-bit draw gives two
    32-bit level values (high half first).  Per level: value < t1 -> quadrant (0,0),
    < t2 -> (0,1), < t3 -> (1,0), else (1,1); the quadrant appends one bit to the row
    id and one to the column id."""
    idx = np.arange(start, start + cnt, dtype=np.uint64) * _U64(nh)
    u = np.zeros(cnt, dtype=np.uint32)
    v = np.zeros(cnt, dtype=np.uint32)
    level = 0
    with np.errstate(over="ignore"):
        for j in range(nh):
            h = mix64((idx + _U64(j + 1)) * _GOLDEN + key)
            for half in ((h >> _U64(32)).astype(np.uint32), h.astype(np.uint32)):
                if level >= scale:
                    break
                a2 = half >= t2
                bv = ((half >= t1) & ~a2) | (half >= t3)
                u <<= np.uint32(1)
                u |= a2
                v <<= np.uint32(1)
                v |= bv
                level += 1
    return u, v


def _rmat_samples(scale: int, m: int, key: np.uint64, abcd: Sequence[float], chunk: int,
                  threads: Optional[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Endpoints of R-MAT samples 0 .. m-1 of stream `key` at `scale` levels."""
    import concurrent.futures
    import os
    a, b, c, _d = abcd
    t1 = np.uint32(min(int(a * 2 ** 32), 2 ** 32 - 1))
    t2 = np.uint32(min(int((a + b) * 2 ** 32), 2 ** 32 - 1))
    t3 = np.uint32(min(int((a + b + c) * 2 ** 32), 2 ** 32 - 1))
    nh = (scale + 1) // 2                      # two 32-bit level draws per uint64
    starts = list(range(0, m, chunk))
    nthr = threads or min(16, os.cpu_count() or 1)
    u = np.empty(m, dtype=np.int64)
    v = np.empty(m, dtype=np.int64)

    def work(st: int) -> None:
        cnt = min(chunk, m - st)
        cu, cv = _rmat_chunk(key, st, cnt, scale, nh, t1, t2, t3)
        u[st:st + cnt] = cu
        v[st:st + cnt] = cv

    if nthr > 1 and len(starts) > 1:
        with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, starts))
    else:
        for st in starts:
            work(st)
    return u, v


def _permutation(seed: int, n: int, sub: int) -> np.ndarray:
    """newid[old] of a seeded random relabelling of n ids."""
    pk = draws(stream_key(seed, STREAM_RMAT_PERM, sub), 0, n)
    order = np.argsort(pk, kind="stable")
    newid = np.empty(n, dtype=np.int64)
    newid[order] = np.arange(n, dtype=np.int64)
    return newid


RMAT_ER = (0.25, 0.25, 0.25, 0.25)     # Sec. 4: Rmat-er
RMAT_G = (0.45, 0.15, 0.15, 0.25)      # Sec. 4: Rmat-g


def rmat_n(n: int, avg_degree: float, seed: int, abcd: Sequence[float] = RMAT_ER, sub: int = 0,
           chunk: int = 1 << 22, threads: Optional[int] = None) -> CSR:
    """R-MAT graph with any vertex count n and a target average degree (the size and
    density sweeps of Sec. 4): samples are drawn on 2^s >= n ids, the ids relabelled by
    a seeded random permutation, and only samples with both endpoints below n kept.
    round(n * avg_degree / 2 * (2^s / n)^2) samples are drawn, so about n * avg_degree / 2
    of them survive the restriction; after symmetrising and dropping self-loops and
    duplicates the average degree is slightly below the target."""
    if n < 2:
        raise ValueError("n must be >= 2")
    scale = max(1, int(np.ceil(np.log2(n))))
    if scale > 30:
        raise ValueError("n must be <= 2^30")
    N = 1 << scale
    m = int(round(n * avg_degree / 2.0 * (N / n) ** 2))
    key = stream_key(seed, STREAM_RMAT_BITS, 1000 + sub)
    u, v = _rmat_samples(scale, m, key, abcd, chunk, threads)
    newid = _permutation(seed, N, 1000 + sub)
    u = newid[u]
    v = newid[v]
    keep = (u < n) & (v < n)
    tag = "er" if tuple(abcd) == RMAT_ER else ("g" if tuple(abcd) == RMAT_G else "x")
    return csr_from_arcs(n, u[keep], v[keep], name=f"rmat{tag}_n{n}_d{avg_degree:g}_s{seed}")


def rmat(scale: int, edge_factor: int, seed: int, abcd: Sequence[float] = RMAT_DEFAULT,
         permute: bool = True, sub: int = 0, chunk: int = 1 << 22, threads: Optional[int] = None) -> CSR:
    """R-MAT graph (Sec. 4): 2^scale vertices, edge_factor * 2^scale edge samples.

    Each sample picks one of four quadrants per level with probabilities (a, b, c, d)
    (32-bit thresholds), which fixes one bit of the row and one of the column.  No
    noise is added.  With ``permute`` the vertex ids are relabelled by a seeded random
    permutation.  The samples are symmetrised; self-loops and duplicates dropped.
    Chunks of samples are drawn on a thread pool; the result does not depend on the
    chunk size or the thread count (counter-based draws)."""
    if scale > 30:
        raise ValueError("scale must be <= 30 for int32 ids")
    n = 1 << scale
    m = edge_factor * n
    u, v = _rmat_samples(scale, m, stream_key(seed, STREAM_RMAT_BITS, sub), abcd, chunk, threads)
    if permute:
        newid = _permutation(seed, n, sub)
        u = newid[u]
        v = newid[v]
    return csr_from_arcs(n, u, v, name=f"rmat_s{scale}_ef{edge_factor}_s{seed}")


# ----------------------------------------------------------------------------
# The five workload configurations
# ----------------------------------------------------------------------------

def config_er16k(seed: int = 1) -> CSR:
    """ER n=16,384, m=131,072 pairs (average degree 16)."""
    return erdos_renyi(16384, 131072, seed)


def config_stencil128() -> CSR:
    """27-point stencil on a 128^3 grid (2,097,152 vertices, 53,645,816 arcs)."""
    return stencil27(128, 128, 128)


def config_rmat23(seed: int = 1) -> CSR:
    """R-MAT scale 23, edge factor 16, (0.57, 0.19, 0.19, 0.05), permuted ids."""
    return rmat(23, 16, seed)


# ----------------------------------------------------------------------------
# Batched set: many independent graphs in one block-diagonal CSR
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class GraphSpec:
    kind: str               # "er" | "stencil" | "rmat"
    params: Tuple[int, ...]  # er: (n, m, seed, sub); stencil: (X, Y, Z); rmat: (scale, ef, seed, sub)

    def build(self) -> CSR:
        if self.kind == "er":
            n, m, s, sub = self.params
            return erdos_renyi(n, m, s, sub)
        if self.kind == "stencil":
            return stencil27(*self.params)
        if self.kind == "rmat":
            sc, ef, s, sub = self.params
            return rmat(sc, ef, s, sub=sub)
        raise ValueError(self.kind)

    def est_vertices(self) -> int:
        if self.kind == "er":
            return self.params[0]
        if self.kind == "stencil":
            X, Y, Z = self.params
            return X * Y * Z
        return 1 << self.params[0]

    def est_arcs(self) -> int:
        if self.kind == "er":
            return 2 * self.params[1]
        if self.kind == "stencil":
            return stencil27_arcs(*self.params)
        return 2 * self.params[1] * (1 << self.params[0])


def batch_specs(G: int = 2048, seed: int = 1, nmin: float = 1e3, nmax: float = 2e5,
                dmin: float = 4.0, dmax: float = 64.0, side_min: int = 8,
                side_max: int = 48) -> List[GraphSpec]:
    """Specs of the batched workload: G/2 ER graphs (n log-uniform in [nmin, nmax],
    average degree log-uniform in [dmin, dmax]) and G/2 27-point stencils (box sides
    uniform in [side_min, side_max]; boxes with fewer than nmin vertices are redrawn),
    in a seeded shuffled order."""
    key = stream_key(seed, STREAM_BATCH_SPEC)
    specs: List[GraphSpec] = []
    ctr = 0

    def u01() -> float:
        nonlocal ctr
        h = int(draws(key, ctr, 1)[0])
        ctr += 1
        return (h >> 11) / float(1 << 53)

    for g in range(G // 2):
        n = int(round(math.exp(math.log(nmin) + u01() * (math.log(nmax) - math.log(nmin)))))
        d = math.exp(math.log(dmin) + u01() * (math.log(dmax) - math.log(dmin)))
        m = max(1, int(round(n * d / 2)))
        specs.append(GraphSpec("er", (n, m, seed, 1000 + g)))
    span = side_max - side_min + 1
    for g in range(G - G // 2):
        while True:
            X = side_min + min(span - 1, int(u01() * span))
            Y = side_min + min(span - 1, int(u01() * span))
            Z = side_min + min(span - 1, int(u01() * span))
            if X * Y * Z >= nmin:
                break
        specs.append(GraphSpec("stencil", (X, Y, Z)))
    # seeded shuffle of the graph order
    keys = draws(key, ctr, len(specs))
    order = np.argsort(keys, kind="stable")
    return [specs[i] for i in order]


@dataclasses.dataclass
class BatchedCSR:
    """Block-diagonal union of G graphs with global vertex ids.

    voff[g]..voff[g+1] are graph g's vertices; rowptr/colidx are one CSR over all."""
    G: int
    voff: np.ndarray      # int64[G+1]
    rowptr: np.ndarray    # int32[N+1]
    colidx: np.ndarray    # int32[nnz], global ids
    parts: Optional[List[CSR]] = None

    @property
    def n(self) -> int:
        return int(self.voff[-1])

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def concat_graphs(graphs: Sequence[CSR], keep_parts: bool = False) -> BatchedCSR:
    G = len(graphs)
    voff = np.zeros(G + 1, dtype=np.int64)
    eoff = np.zeros(G + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        voff[i + 1] = voff[i] + g.n
        eoff[i + 1] = eoff[i] + g.nnz
    N, E = int(voff[-1]), int(eoff[-1])
    if N >= 2 ** 31 or E >= 2 ** 31:
        raise OverflowError("batched union exceeds int32 vertex or arc range")
    rowptr = np.empty(N + 1, dtype=np.int32)
    colidx = np.empty(E, dtype=np.int32)
    for i, g in enumerate(graphs):
        v0, e0 = int(voff[i]), int(eoff[i])
        rowptr[v0:v0 + g.n] = g.rowptr[:-1].astype(np.int64) + e0
        colidx[e0:e0 + g.nnz] = g.colidx.astype(np.int64) + v0
    rowptr[N] = E
    return BatchedCSR(G, voff, rowptr, colidx, list(graphs) if keep_parts else None)


def build_graphs(specs: Sequence[GraphSpec], threads: Optional[int] = None) -> List[CSR]:
    """Build every spec, on a thread pool (each graph is a pure function of its spec)."""
    import concurrent.futures
    import os
    nthr = threads or min(16, os.cpu_count() or 1)
    if nthr <= 1 or len(specs) <= 1:
        return [s.build() for s in specs]
    with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
        return list(ex.map(lambda sp: sp.build(), specs))


def batch_graphs(specs: Sequence[GraphSpec], keep_parts: bool = False,
                 threads: Optional[int] = None) -> BatchedCSR:
    return concat_graphs(build_graphs(specs, threads), keep_parts=keep_parts)


# ----------------------------------------------------------------------------
# Serving stream
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    spec: GraphSpec


def serve_stream(nreq: int, qps: float, seed: int = 1, rmat_scale: Tuple[int, int] = (10, 20),
                 rmat_ef: Tuple[int, int] = (8, 32), er_n: Tuple[float, float] = (1e3, 1e6),
                 er_deg: Tuple[float, float] = (8.0, 32.0)) -> List[Request]:
    """Poisson request stream: exponential inter-arrival times at rate `qps`; each
    request is, with probability 1/2 each, an R-MAT graph (scale and edge factor
    uniform integers in the given ranges) or an ER graph (n log-uniform, average
    degree uniform in the given ranges)."""
    key = stream_key(seed, STREAM_SERVE_SPEC)
    ctr = 0

    def u01() -> float:
        nonlocal ctr
        h = int(draws(key, ctr, 1)[0])
        ctr += 1
        return (h >> 11) / float(1 << 53)

    t = 0.0
    out = []
    for r in range(nreq):
        t += -math.log(1.0 - u01()) / qps
        if u01() < 0.5:
            sc = rmat_scale[0] + min(rmat_scale[1] - rmat_scale[0], int(u01() * (rmat_scale[1] - rmat_scale[0] + 1)))
            ef = rmat_ef[0] + min(rmat_ef[1] - rmat_ef[0], int(u01() * (rmat_ef[1] - rmat_ef[0] + 1)))
            spec = GraphSpec("rmat", (sc, ef, seed, 5000 + r))
        else:
            n = int(round(math.exp(math.log(er_n[0]) + u01() * (math.log(er_n[1]) - math.log(er_n[0])))))
            d = er_deg[0] + u01() * (er_deg[1] - er_deg[0])
            spec = GraphSpec("er", (n, max(1, int(round(n * d / 2))), seed, 5000 + r))
        out.append(Request(r, t, spec))
    return out


# ----------------------------------------------------------------------------
# Small graphs for tests
# ----------------------------------------------------------------------------

def from_edges(n: int, edges: Sequence[Tuple[int, int]], name: str = "") -> CSR:
    if len(edges) == 0:
        return CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), name)
    e = np.asarray(edges, dtype=np.int64)
    return csr_from_arcs(n, e[:, 0], e[:, 1], name=name)


def complete(n: int) -> CSR:
    u, v = np.triu_indices(n, 1)
    return csr_from_arcs(n, u, v, name=f"K{n}")


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return csr_from_arcs(n, i, (i + 1) % n, name=f"C{n}")


def path(n: int) -> CSR:
    i = np.arange(n - 1)
    return csr_from_arcs(n, i, i + 1, name=f"P{n}")


def star(center: int, leaves: Sequence[int]) -> CSR:
    n = max([center] + list(leaves)) + 1
    return csr_from_arcs(n, np.full(len(leaves), center), np.asarray(leaves), name="star")


def edgeless(n: int) -> CSR:
    return CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), f"E{n}")


def random_small(n: int, p: float, seed: int, sub: int = 0) -> CSR:
    """G(n, p) on all n(n-1)/2 pairs with a counter-based coin per pair."""
    if n < 2:
        return edgeless(n)
    u, v = np.triu_indices(n, 1)
    h = draws(stream_key(seed, STREAM_FUZZ, sub), 0, len(u))
    keep = (h >> _U64(11)).astype(np.float64) / float(1 << 53) < p
    if not keep.any():
        return edgeless(n)
    return csr_from_arcs(n, u[keep], v[keep], name=f"gnp_{n}_{p}_{seed}_{sub}")


def raw_csr(n: int, rows: Sequence[Sequence[int]]) -> CSR:
    """CSR taken verbatim from per-row lists (unsorted rows, self-loops and duplicates
    are kept), for degenerate-input tests."""
    rowptr = np.zeros(n + 1, dtype=np.int64)
    for i, r in enumerate(rows):
        rowptr[i + 1] = rowptr[i] + len(r)
    col = np.array([w for r in rows for w in r], dtype=np.int32)
    return CSR(n, rowptr.astype(np.int32), col, "raw")


def shuffle_rows(g: CSR, seed: int) -> CSR:
    """Same graph with every row's entries in a seeded random order."""
    col = g.colidx.copy()
    key = draws(stream_key(seed, STREAM_FUZZ, 77), 0, len(col))
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr.astype(np.int64)))
    order = np.lexsort((key, rows))
    return CSR(g.n, g.rowptr.copy(), col[order], g.name + "_shuffled")

"""CPU oracle for speculative-greedy graph coloring -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never calls it, and it shares no code with the GPU
path.  It offers:

  * ``sgr``        -- serial speculative-greedy rounds (Sec. 3.1, Algorithm Data-GC with
                      FirstFit and ConflictResolve of Sec. 3), plain C (sgr_oracle.c);
  * ``sgr_topo``   -- the topology-driven variant (Sec. 3.1, Algorithm Topo-GC), plain C;
  * ``jp``         -- Jones-Plassmann independent-set colouring (Sec. 2.2, Algorithm 3)
                      with counter-based SplitMix64 priorities, plain C (jp_oracle.c);
  * ``serial_ff``  -- natural-order sequential greedy (Sec. 2.1, Algorithm 1), plain C;
  * ``conflicts`` / ``non_grundy`` -- checkers for a proper / Grundy colouring;
  * ``sgr_numpy``  -- an independent, vectorised re-implementation of the same rounds
                      (sgr_numpy.py) used to cross-check the C oracle;
  * ``jp_numpy``   -- the same for JP (jp_numpy.py);
  * ``brute``      -- exhaustive chromatic and Grundy numbers of tiny graphs.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "sgr_oracle.c"), os.path.join(_HERE, "jp_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib: Optional[ctypes.CDLL] = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc -O2 into oracle/liboracle.so."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_sgr.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, P, ctypes.c_int32]
        lib.oracle_sgr.restype = ctypes.c_int
        lib.oracle_sgr_rule.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_sgr_rule.restype = ctypes.c_int
        lib.oracle_sgr_capped.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32]
        lib.oracle_sgr_capped.restype = ctypes.c_int
        lib.oracle_sgr_topo.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_sgr_topo.restype = ctypes.c_int
        lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_splitmix64.restype = ctypes.c_uint64
        lib.oracle_jp_priority.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_jp_priority.restype = ctypes.c_uint64
        lib.oracle_jp.argtypes = [ctypes.c_int32, P, P, ctypes.c_uint64, P, P, P, P, P, ctypes.c_int32]
        lib.oracle_jp.restype = ctypes.c_int
        lib.oracle_serial_ff.argtypes = [ctypes.c_int32, P, P, P, P]
        lib.oracle_serial_ff.restype = ctypes.c_int
        lib.oracle_count_conflicts.argtypes = [ctypes.c_int32, P, P, P]
        lib.oracle_count_conflicts.restype = ctypes.c_int64
        lib.oracle_count_non_grundy.argtypes = [ctypes.c_int32, P, P, P]
        lib.oracle_count_non_grundy.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _as_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


@dataclasses.dataclass
class SGRResult:
    colors: np.ndarray       # int32[n], 0-based
    ncolors: int
    rounds: int
    wsize: np.ndarray        # int64[rounds]: |W_r|
    arcs_ff: np.ndarray      # int64[rounds]: arcs scanned by FirstFit
    arcs_cr: np.ndarray      # int64[rounds]: lower arcs examined by the conflict test


RULE_ID = 0        # higher id of a same-colour adjacent pair is requeued
RULE_DEGREE = 1    # heuristic conflict resolve (Sec. 3.2): smaller degree requeued, ties by id


def sgr(n: int, rowptr, colidx, stats_cap: int = 1 << 16, rule: int = RULE_ID, max_rounds: int = 0) -> SGRResult:
    """Run the serial SGR oracle.  Raises on malformed input.  max_rounds > 0 stops after
    that many rounds (a bounded timing sample; vertices still uncoloured read -1)."""
    lib = _load()
    rp, ci = _as_i32(rowptr), _as_i32(colidx)
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1, dtype=np.int32)
    ws = np.zeros(stats_cap, dtype=np.int64)
    af = np.zeros(stats_cap, dtype=np.int64)
    ac = np.zeros(stats_cap, dtype=np.int64)
    rc = lib.oracle_sgr_capped(n, _ptr(rp), _ptr(ci), _ptr(out), _ptr(nc), _ptr(rr),
                               _ptr(ws), _ptr(af), _ptr(ac), stats_cap, rule, max_rounds)
    if rc != 0:
        raise ValueError(f"oracle_sgr failed with status {rc}")
    r = int(rr[0])
    k = min(r, stats_cap)
    return SGRResult(out[:n].copy(), int(nc[0]), r, ws[:k].copy(), af[:k].copy(), ac[:k].copy())


@dataclasses.dataclass
class TopoResult:
    colors: np.ndarray       # int32[n], 0-based
    ncolors: int
    rounds: int
    wsize: np.ndarray        # int64[rounds]: vertices that ran FirstFit
    visits: np.ndarray       # int64[rounds]: vertices visited (n every round)


def sgr_topo(n: int, rowptr, colidx, stats_cap: int = 1 << 16, rule: int = RULE_ID) -> TopoResult:
    """Topology-driven SGR (Algorithm Topo-GC).  Raises on malformed input."""
    lib = _load()
    rp, ci = _as_i32(rowptr), _as_i32(colidx)
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1, dtype=np.int32)
    ws = np.zeros(stats_cap, dtype=np.int64)
    vi = np.zeros(stats_cap, dtype=np.int64)
    rc = lib.oracle_sgr_topo(n, _ptr(rp), _ptr(ci), _ptr(out), _ptr(nc), _ptr(rr), _ptr(ws), _ptr(vi),
                             stats_cap, rule)
    if rc != 0:
        raise ValueError(f"oracle_sgr_topo failed with status {rc}")
    k = min(int(rr[0]), stats_cap)
    return TopoResult(out[:n].copy(), int(nc[0]), int(rr[0]), ws[:k].copy(), vi[:k].copy())


def splitmix64(seed: int, k: int) -> int:
    """Output number k (k >= 1) of SplitMix64 seeded with `seed`."""
    return int(_load().oracle_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))


def jp_priority(seed: int, rnd: int, v: int) -> int:
    """JP priority of vertex v in round rnd (1-based): SplitMix64 output rnd * 2^32 + v."""
    return int(_load().oracle_jp_priority(seed & (2**64 - 1), rnd, v))


@dataclasses.dataclass
class JPResult:
    colors: np.ndarray       # int32[n], 0-based
    ncolors: int
    rounds: int
    wsize: np.ndarray        # int64[rounds]: |W_r|
    arcs: np.ndarray         # int64[rounds]: sum of row lengths over W_r


def jp(n: int, rowptr, colidx, seed: int = 0, stats_cap: int = 1 << 16) -> JPResult:
    """Jones-Plassmann colouring (Algorithm 3).  Raises on malformed input."""
    lib = _load()
    rp, ci = _as_i32(rowptr), _as_i32(colidx)
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1, dtype=np.int32)
    ws = np.zeros(stats_cap, dtype=np.int64)
    ar = np.zeros(stats_cap, dtype=np.int64)
    rc = lib.oracle_jp(n, _ptr(rp), _ptr(ci), seed & (2**64 - 1), _ptr(out), _ptr(nc), _ptr(rr),
                       _ptr(ws), _ptr(ar), stats_cap)
    if rc != 0:
        raise ValueError(f"oracle_jp failed with status {rc}")
    k = min(int(rr[0]), stats_cap)
    return JPResult(out[:n].copy(), int(nc[0]), int(rr[0]), ws[:k].copy(), ar[:k].copy())


def serial_ff(n: int, rowptr, colidx):
    """Natural-order sequential greedy: returns (colors 0-based, ncolors)."""
    lib = _load()
    rp, ci = _as_i32(rowptr), _as_i32(colidx)
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    rc = lib.oracle_serial_ff(n, _ptr(rp), _ptr(ci), _ptr(out), _ptr(nc))
    if rc != 0:
        raise ValueError(f"oracle_serial_ff failed with status {rc}")
    return out[:n].copy(), int(nc[0])


def conflicts(n: int, rowptr, colidx, colors) -> int:
    """Number of arcs whose two (distinct) endpoints share a colour."""
    lib = _load()
    rp, ci, co = _as_i32(rowptr), _as_i32(colidx), _as_i32(colors)
    k = int(lib.oracle_count_conflicts(n, _ptr(rp), _ptr(ci), _ptr(co)))
    if k < 0:
        raise ValueError(f"oracle_count_conflicts failed with status {k}")
    return k


def non_grundy(n: int, rowptr, colidx, colors) -> int:
    """Number of vertices whose 0-based colour differs from the mex of its neighbours."""
    lib = _load()
    rp, ci, co = _as_i32(rowptr), _as_i32(colidx), _as_i32(colors)
    k = int(lib.oracle_count_non_grundy(n, _ptr(rp), _ptr(ci), _ptr(co)))
    if k < 0:
        raise ValueError(f"oracle_count_non_grundy failed with status {k}")
    return k


def bytes_model(res: SGRResult, n: int) -> int:
    """Algorithmic HBM bytes of one SGR run with 4-byte ids and colours.

    Round 1 (all snapshot colours are 0, so every tentative colour is 1 and a vertex
    is requeued iff it has a lower neighbour): rowptr pair (8 B) + first arc (4 B) +
    colour write (4 B) + output write (4 B) per vertex, plus 4 B per requeued vertex.
    Later rounds, FirstFit: 16 B per worklist vertex (id, rowptr pair, colour write)
    + 8 B per scanned arc (colidx + neighbour colour); conflict test: 20 B per
    worklist vertex (id, rowptr pair, own colour, colour/output write) + 8 B per
    examined lower arc + 4 B per requeued vertex."""
    if res.rounds == 0:
        return 0
    w = [int(x) for x in res.wsize] + [0]
    b = 20 * n + 4 * w[1]
    for r in range(1, res.rounds):
        b += 16 * w[r] + 8 * int(res.arcs_ff[r])
        b += 20 * w[r] + 8 * int(res.arcs_cr[r]) + 4 * w[r + 1]
    return b


from .sgr_numpy import sgr_numpy  # noqa: E402
from .jp_numpy import jp_numpy  # noqa: E402
from . import brute  # noqa: E402

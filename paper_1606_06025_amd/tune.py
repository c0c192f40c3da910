"""Autotuner for the colouring launch options.

None of the options changes the colouring; they only move work between kernels and
launch shapes: drive mode (host loop / replayed hipGraph / persistent), FirstFit variant
(rescan / push bitmaps), the degree thresholds of the tile, wavefront and split-row buckets, the
workgroups per CU, how the low-degree conflict test maps lanes, and how often the
host reads the queue sizes back.  The tuner times candidates on the actual graph by
coordinate descent from the library defaults (each knob in turn, keeping the best
value), and caches the winner per (device, graph signature) in a JSON file.

The signature is coarse on purpose, so similar graphs share an entry: log2 of the
vertex and arc counts and the share of arcs in each degree bucket in tenths.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "csrcolor", "tune.json")

# knob -> values tried (0 = library default)
KNOBS: List[Tuple[str, Sequence[int]]] = [
    ("wake", (0, 1, -1)),
    ("firstfit", (3, 2, 1)),
    ("mode", (1, 3, 2)),
    ("t_wave", (1024, 256, 128)),
    ("t_split", (2048, 8192, 1024)),
    # tile-bucket degree limits t0 | t1 << 8 | t2 << 16 (0 = 5, 13, 29)
    ("tile_limits", (0, 3 | (9 << 8) | (21 << 16), 2 | (5 << 8) | (13 << 16))),
    ("blocks_per_cu", (6, 4, 8)),
    ("lane_detect", (-1, 15)),
    ("sync_every", (8, 16, 32)),
]

_BUCKET_EDGES = (5, 13, 29, 61, 1024, 2048)


def signature(rowptr: np.ndarray) -> str:
    rp = np.asarray(rowptr, dtype=np.int64)
    n = len(rp) - 1
    deg = np.diff(rp)
    nnz = int(rp[-1]) if n > 0 else 0
    b = np.searchsorted(np.array(_BUCKET_EDGES), deg, side="left")
    shares = np.bincount(b, weights=deg, minlength=len(_BUCKET_EDGES) + 1) / max(nnz, 1)
    q = tuple(int(round(x * 10)) for x in shares)
    return f"n{int(np.log2(max(n, 1)))}_e{int(np.log2(max(nnz, 1)))}_" + "".join(f"{x:x}" for x in q)


def device_key() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0).replace(" ", "_")
    except Exception:
        return "unknown"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def coordinate_descent(measure: Callable[[Dict[str, int]], float],
                       knobs: Sequence[Tuple[str, Sequence[int]]] = KNOBS,
                       start: Optional[Dict[str, int]] = None, log: Optional[Callable[[str], None]] = None
                       ) -> Tuple[Dict[str, int], float, int]:
    """Minimise measure(config) one knob at a time.  Returns (best config, its time,
    number of measurements)."""
    best = dict(start or {})
    best_t = measure(best)
    evals = 1
    for name, values in knobs:
        for v in values:
            if best.get(name, values[0]) == v:
                continue
            cand = dict(best)
            cand[name] = v
            t = measure(cand)
            evals += 1
            if log:
                log(f"tune {name}={v}: {t * 1e3:.3f} ms (best {best_t * 1e3:.3f})")
            if t < best_t:
                best, best_t = cand, t
    return best, best_t, evals


def tune(rowptr, colidx, voff=None, reps: int = 3, cache: Optional[str] = DEFAULT_CACHE,
         knobs: Sequence[Tuple[str, Sequence[int]]] = KNOBS, log: Optional[Callable[[str], None]] = None,
         force: bool = False) -> Dict[str, int]:
    """Best option set for this graph (device tensors rowptr/colidx, and voff for a
    batched union).  Uses the cache unless `force`."""
    import torch
    from . import api
    key = f"{device_key()}/{'batched/' if voff is not None else ''}{signature(rowptr.cpu().numpy())}"
    data = _load(cache) if cache else {}
    if not force and key in data:
        return dict(data[key]["opts"])
    out = torch.empty(rowptr.numel() - 1, dtype=torch.int32, device=rowptr.device)

    def run(cfg):
        o = api.make_opts(**cfg) if cfg else None
        if voff is not None:
            api.color_batched(voff, rowptr, colidx, out=out, opts=o)
        else:
            api.color(rowptr, colidx, out=out, opts=o)

    def measure(cfg):
        run(cfg)                               # warm (captures graphs, grows scratch)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            run(cfg)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    best, best_t, evals = coordinate_descent(measure, knobs, log=log)
    if cache:
        data = _load(cache)
        data[key] = {"opts": best, "ms": best_t * 1e3, "evals": evals, "time": time.time()}
        _save(cache, data)
    return best

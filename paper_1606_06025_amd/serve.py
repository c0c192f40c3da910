"""Continuous-batching colouring server.

Requests (one CSR graph each) arrive at any time.  A scheduler admits them in
arrival order while the HBM footprint of everything admitted stays within a budget,
uploads each admitted graph once (it stays device-resident until its result is
back), and whenever one of the execution slots is free hands it every admitted
request that is still waiting (up to a batch limit).  Each slot is a HIP stream with
its own library workspace and a worker thread; a batch is one
``csrcolor_color_multi`` call, so batches on different slots overlap on the GPU and
requests that arrive while others run join the next free slot.  Because the graphs
of a batch are independent components of one block-diagonal graph, every request
gets exactly the colouring it would get alone.

Latency of a request = completion time - arrival time; the server records both and
reports p50 / p99 and the arc throughput.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


def footprint_bytes(n: int, nnz: int) -> int:
    """HBM bytes one request holds while admitted: its CSR and output (4n+4+4nnz+4n)
    plus its share of the library scratch of a batch (union copy 4n+4+4nnz, union
    colours 4n, colour state 4n, worklists 8n, forbidden bitmaps (n+nnz)/8), rounded
    up generously for small graphs."""
    return 28 * n + 8 * nnz + (n + nnz) // 8 + 4096


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    nnz: int
    arrival: float
    payload: object = None           # backend handle once admitted
    colors: Optional[np.ndarray] = None
    ncolors: int = -1
    error: Optional[str] = None
    admitted: float = -1.0
    started: float = -1.0
    done_time: float = -1.0
    batch_size: int = 0
    group: int = 0                   # batching class: bit length of the largest degree
    _event: threading.Event = dataclasses.field(default_factory=threading.Event)

    def wait(self, timeout: Optional[float] = None) -> bool:
        return self._event.wait(timeout)

    @property
    def done(self) -> bool:
        return self._event.is_set()

    @property
    def latency(self) -> float:
        return self.done_time - self.arrival


class Backend:
    """Device side of the server (overridden by tests with a CPU stand-in)."""

    nslots = 1

    def upload(self, rowptr: np.ndarray, colidx: np.ndarray):
        raise NotImplementedError

    def release(self, handle) -> None:
        pass

    def run_batch(self, slot: int, handles: Sequence) -> List[Tuple[np.ndarray, int]]:
        raise NotImplementedError


class HipBackend(Backend):
    """Graphs live in device tensors; a batch is one csrcolor_color_multi call on the
    slot's stream.  Uploads are copies from the caller's (pageable) arrays on a stream of
    their own, so they overlap the batches running on the slots, each followed by an
    event the batch's stream waits for; a batch's colours come back in one pinned
    buffer.  (Pinning every request's arrays first costs more than it saves: the pinned
    allocation and its page locking ran at a fraction of the copy engine's rate.)"""

    def __init__(self, nslots: int = 2, device: str = "cuda:0", opts=None):
        import torch
        from . import _lib
        _lib.load()
        self.torch = torch
        self.device = torch.device(device)
        self.nslots = nslots
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(nslots)]
        self.up_stream = torch.cuda.Stream(device=self.device)
        self.opts = opts

    def upload(self, rowptr, colidx):
        torch = self.torch
        n = max(len(rowptr) - 1, 0)
        hrp = torch.from_numpy(np.ascontiguousarray(rowptr, dtype=np.int32))
        hci = torch.from_numpy(np.ascontiguousarray(colidx, dtype=np.int32))
        with torch.cuda.stream(self.up_stream):
            # from pageable memory the copy has taken the data when the call returns
            rp = hrp.to(self.device)
            ci = hci.to(self.device)
            out = torch.empty(n, dtype=torch.int32, device=self.device)
            ev = torch.cuda.Event()
            ev.record(self.up_stream)
        return (rp, ci, out, int(len(colidx)), ev, (hrp, hci))

    def run_batch(self, slot, handles):
        from . import api
        torch = self.torch
        st = self.streams[slot]
        for h in handles:
            st.wait_event(h[4])
        sizes = [h[2].numel() for h in handles]
        host = torch.empty(sum(sizes), dtype=torch.int32, pin_memory=True)
        with torch.cuda.stream(st):
            outs, ncol = api.color_multi([(h[0], h[1]) for h in handles], outs=[h[2] for h in handles],
                                         nnz=[h[3] for h in handles], opts=self.opts, stream=st)
            off = 0
            for o, k in zip(outs, sizes):
                host[off:off + k].copy_(o[:k], non_blocking=True)
                off += k
            nc = ncol.cpu().numpy()
        st.synchronize()
        res, off = [], 0
        for k in sizes:
            res.append(host[off:off + k].numpy().copy())
            off += k
        return [(res[i], int(nc[i])) for i in range(len(handles))]


class ColoringServer:
    def __init__(self, backend: Backend, hbm_budget: int, max_batch: int = 64,
                 max_batch_arcs: int = 1 << 30, clock: Callable[[], float] = time.perf_counter):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.max_batch_arcs = max_batch_arcs
        self.clock = clock
        self._cv = threading.Condition()
        self._pending: collections.deque = collections.deque()   # (Request, rowptr, colidx)
        self._admitted: collections.deque = collections.deque()  # Request
        self._inflight_bytes = 0
        self._peak_bytes = 0
        self._free_slots = list(range(backend.nslots))
        self._stop = False
        self._threads: List[threading.Thread] = []
        self._slot_work: Dict[int, List[Request]] = {}
        self._slot_cv = [threading.Condition(self._cv) for _ in range(backend.nslots)]
        self._next_id = 0
        self.finished: List[Request] = []

    # -- client side ---------------------------------------------------------
    def submit(self, rowptr: np.ndarray, colidx: np.ndarray, arrival: Optional[float] = None) -> Request:
        n = len(rowptr) - 1
        nnz = int(rowptr[-1]) if n > 0 else 0
        maxdeg = int(np.max(np.diff(np.asarray(rowptr, dtype=np.int64)))) if n > 0 else 0
        with self._cv:
            req = Request(self._next_id, n, nnz, self.clock() if arrival is None else arrival,
                          group=max(maxdeg, 0).bit_length())
            self._next_id += 1
            if footprint_bytes(n, nnz) > self.budget:
                req.error = "request larger than the HBM budget"
                req.done_time = self.clock()
                req._event.set()
                self.finished.append(req)
                return req
            self._pending.append((req, rowptr, colidx))
            self._cv.notify_all()
        return req

    # -- lifecycle -----------------------------------------------------------
    def start(self) -> "ColoringServer":
        t = threading.Thread(target=self._schedule, name="csrcolor-scheduler", daemon=True)
        self._threads.append(t)
        t.start()
        for s in range(self.backend.nslots):
            w = threading.Thread(target=self._worker, args=(s,), name=f"csrcolor-slot{s}", daemon=True)
            self._threads.append(w)
            w.start()
        return self

    def stop(self) -> None:
        with self._cv:
            self._stop = True
            self._cv.notify_all()
            for c in self._slot_cv:
                c.notify_all()
        for t in self._threads:
            t.join()

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    @property
    def peak_bytes(self) -> int:
        return self._peak_bytes

    # -- scheduler -----------------------------------------------------------
    def _schedule(self) -> None:
        while True:
            with self._cv:
                while not self._stop and not self._can_admit() and not self._can_dispatch():
                    self._cv.wait()
                if self._stop:
                    return
                admit = []
                while self._can_admit():
                    req, rp, ci = self._pending.popleft()
                    self._inflight_bytes += footprint_bytes(req.n, req.nnz)
                    self._peak_bytes = max(self._peak_bytes, self._inflight_bytes)
                    admit.append((req, rp, ci))
            # uploads happen outside the lock
            for req, rp, ci in admit:
                try:
                    req.payload = self.backend.upload(rp, ci)
                except Exception as e:  # a bad request fails alone
                    req.error = f"upload failed: {e}"
                req.admitted = self.clock()
            with self._cv:
                for req, _, _ in admit:
                    if req.error:
                        self._finish(req)
                    else:
                        self._admitted.append(req)
                while self._can_dispatch():
                    slot = self._free_slots.pop(0)
                    batch = self._take_batch()
                    self._slot_work[slot] = batch
                    self._slot_cv[slot].notify_all()

    def _take_batch(self) -> List[Request]:
        """The oldest admitted request and, in arrival order, the others of its batching
        class or an adjacent one (caller holds the lock).  A batch runs as many rounds as
        its slowest graph, and the rounds grow with the largest degree (hubs), so graphs
        of like degree share a batch rather than small ones waiting on a hub graph."""
        first = self._admitted.popleft()
        batch, arcs, keep = [first], first.nnz, collections.deque()
        while self._admitted:
            nxt = self._admitted.popleft()
            if (len(batch) < self.max_batch and abs(nxt.group - first.group) <= 1
                    and arcs + nxt.nnz <= self.max_batch_arcs):
                batch.append(nxt)
                arcs += nxt.nnz
            else:
                keep.append(nxt)
        self._admitted = keep
        return batch

    def _can_admit(self) -> bool:
        if not self._pending:
            return False
        req = self._pending[0][0]
        return self._inflight_bytes + footprint_bytes(req.n, req.nnz) <= self.budget

    def _can_dispatch(self) -> bool:
        return bool(self._admitted) and bool(self._free_slots)

    def _finish(self, req: Request) -> None:
        # caller holds the lock
        req.done_time = self.clock()
        self._inflight_bytes -= footprint_bytes(req.n, req.nnz)
        try:
            self.backend.release(req.payload)
        finally:
            req.payload = None
        self.finished.append(req)
        req._event.set()

    def _worker(self, slot: int) -> None:
        while True:
            with self._cv:
                while not self._stop and slot not in self._slot_work:
                    self._slot_cv[slot].wait()
                if self._stop:
                    return
                batch = self._slot_work.pop(slot)
            t0 = self.clock()
            for r in batch:
                r.started = t0
                r.batch_size = len(batch)
            try:
                results = self.backend.run_batch(slot, [r.payload for r in batch])
                err = None
            except Exception as e:
                results, err = None, str(e)
            with self._cv:
                for i, r in enumerate(batch):
                    if err is None:
                        r.colors, r.ncolors = results[i]
                    else:
                        r.error = err
                    self._finish(r)
                self._free_slots.append(slot)
                self._cv.notify_all()


def latency_summary(reqs: Sequence[Request]) -> Dict[str, float]:
    lat = np.array([r.latency for r in reqs if r.error is None], dtype=np.float64)
    if lat.size == 0:
        return {"p50_ms": float("nan"), "p99_ms": float("nan"), "mean_ms": float("nan"), "count": 0}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "count": int(lat.size)}


def replay(server: ColoringServer, graphs: Sequence[Tuple[np.ndarray, np.ndarray]], arrivals: Sequence[float],
           sleep: Callable[[float], None] = time.sleep) -> Tuple[List[Request], float]:
    """Submit graph i at start + arrivals[i] (seconds) and wait for all results.
    Returns (requests, wall seconds from the first arrival to the last completion)."""
    t0 = server.clock()
    reqs = []
    for (rp, ci), at in zip(graphs, arrivals):
        now = server.clock() - t0
        if at > now:
            sleep(at - now)
        reqs.append(server.submit(rp, ci, arrival=t0 + at))
    for r in reqs:
        r.wait()
    end = max(r.done_time for r in reqs) if reqs else t0
    return reqs, end - t0

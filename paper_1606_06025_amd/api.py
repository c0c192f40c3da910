"""Python entry points over the C-ABI (torch tensors for device memory and streams)."""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib as L


@dataclasses.dataclass
class ColorStats:
    rounds: int
    ncolors: int
    rows_sorted: bool
    max_degree: int
    nnz: int
    wsize: List[int]
    arcs: List[int]
    ms_setup: float = 0.0
    ms_assign: float = 0.0
    ms_detect: float = 0.0
    n_assign: int = 0
    n_detect: int = 0
    kernel_bytes: Optional[List[int]] = None   # [recolouring FirstFit, flag-scanning test] bytes moved


def make_opts(mode: int = 0, validate: int = 0, t_wave: int = 0, t_split: int = 0,
              blocks_per_cu: int = 0, sync_every: int = 0, lane_assign: int = 0,
              lane_detect: int = 0, firstfit: int = 0, rule: int = 0, algorithm: int = 0,
              seed: int = 0, hints: int = 0, live_lists: int = 0, ordered: int = 0,
              wake: int = 0, tile_limits: int = 0) -> L.Opts:
    o = L.Opts()
    o.mode, o.validate, o.t_wave, o.t_split = mode, validate, t_wave, t_split
    o.blocks_per_cu, o.sync_every = blocks_per_cu, sync_every
    o.lane_assign, o.lane_detect, o.firstfit, o.rule = lane_assign, lane_detect, firstfit, rule
    o.algorithm = algorithm
    o.hints = hints
    o.live_lists = live_lists
    o.ordered = ordered
    o.wake = wake
    o.tile_limits = tile_limits
    seed &= (1 << 64) - 1
    o.seed_lo, o.seed_hi = seed & 0xFFFFFFFF, seed >> 32
    return o


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _check_csr(rowptr: torch.Tensor, colidx: torch.Tensor) -> int:
    if rowptr.dtype != torch.int32 or colidx.dtype != torch.int32:
        raise TypeError("rowptr and colidx must be int32")
    if not (rowptr.is_cuda and colidx.is_cuda):
        raise TypeError("rowptr and colidx must be device tensors")
    if not (rowptr.is_contiguous() and colidx.is_contiguous()):
        raise ValueError("rowptr and colidx must be contiguous")
    if rowptr.dim() != 1 or rowptr.numel() < 1:
        raise ValueError("rowptr must be 1-D with n+1 entries")
    return rowptr.numel() - 1


def color(rowptr: torch.Tensor, colidx: torch.Tensor, out: Optional[torch.Tensor] = None,
          opts: Optional[L.Opts] = None, stats: bool = False, stats_cap: int = 4096,
          time_kernels: bool = False, count_bytes: bool = False,
          stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, int, Optional[ColorStats]]:
    """Colour one graph and wait for it.  Returns (colors int32[n] on the device,
    ncolors, stats).  Passes a statistics block to csrcolor_color_ex (of capacity 0
    unless `stats`), which selects the synchronous path: the host-driven modes, or the
    device-planned one with mode PERSISTENT.
    count_bytes: also count the bytes moved by the wake-flag kernels (slower kernels;
    ColorStats.kernel_bytes)."""
    lib = L.load()
    n = _check_csr(rowptr, colidx)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=rowptr.device)
    elif out.dtype != torch.int32 or out.numel() < n or not out.is_cuda:
        raise ValueError("out must be an int32 device tensor with n entries")
    want = stats or time_kernels or count_bytes
    cap = stats_cap if want else 0
    st = L.Stats()
    st.time_kernels = 1 if time_kernels else 0
    wbuf = (ctypes.c_int64 * max(cap, 1))()
    abuf = (ctypes.c_int64 * max(cap, 1))()
    st.cap = cap
    st.wsize = ctypes.cast(wbuf, ctypes.POINTER(ctypes.c_int64))
    st.arcs = ctypes.cast(abuf, ctypes.POINTER(ctypes.c_int64))
    kbuf = None
    if count_bytes:
        kbuf = (ctypes.c_int64 * 2)()
        st.kernel_bytes = ctypes.cast(kbuf, ctypes.POINTER(ctypes.c_int64))
    rc = lib.csrcolor_color_ex(n, rowptr.data_ptr(), colidx.data_ptr(), out.data_ptr(), None,
                               ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
                               _stream_ptr(stream))
    L.check(rc)
    cs = None
    if want:
        k = min(st.rounds, stats_cap)
        cs = ColorStats(st.rounds, st.ncolors, bool(st.rows_sorted), st.max_degree, st.nnz,
                        list(wbuf[:k]), list(abuf[:k]), st.ms_setup, st.ms_assign, st.ms_detect,
                        st.n_assign, st.n_detect, list(kbuf) if kbuf is not None else None)
    return out[:n], int(st.ncolors), cs


def color_async(rowptr: torch.Tensor, colidx: torch.Tensor, out: Optional[torch.Tensor] = None,
                ncolors: Optional[torch.Tensor] = None, opts: Optional[L.Opts] = None,
                stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Colour one graph without waiting (csrcolor_color_ex with a device colour count and
    no statistics: device-planned, capturable into a CUDA/HIP graph after a first call has
    sized the workspace).  Returns (colors int32[n], ncolors int32[1]) on the device;
    ncolors[0] holds the colour count, or a negative status found on the device."""
    lib = L.load()
    n = _check_csr(rowptr, colidx)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=rowptr.device)
    elif out.dtype != torch.int32 or out.numel() < n or not out.is_cuda:
        raise ValueError("out must be an int32 device tensor with n entries")
    if ncolors is None:
        ncolors = torch.empty(1, dtype=torch.int32, device=rowptr.device)
    elif ncolors.dtype != torch.int32 or ncolors.numel() < 1 or not ncolors.is_cuda:
        raise ValueError("ncolors must be an int32 device tensor")
    rc = lib.csrcolor_color_ex(n, rowptr.data_ptr(), colidx.data_ptr(), out.data_ptr(), ncolors.data_ptr(),
                               ctypes.byref(opts) if opts is not None else None, None, _stream_ptr(stream))
    L.check(rc)
    return out[:n], ncolors


def color_noalloc(rowptr: torch.Tensor, colidx: torch.Tensor, out: torch.Tensor, ncolors: torch.Tensor,
                  nnz: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None) -> None:
    """Colour one graph without any allocation by the library (csrcolor_color_noalloc:
    the device-planned run over the library's fixed scratch array).  The caller passes
    the outputs: `out` int32[n] and `ncolors` int32[1] on the device; `nnz` defaults to
    colidx.numel().  Returns without waiting; ncolors[0] receives the colour count or a
    negative status found on the device."""
    lib = L.load()
    n = _check_csr(rowptr, colidx)
    if out.dtype != torch.int32 or out.numel() < n or not out.is_cuda:
        raise ValueError("out must be an int32 device tensor with n entries")
    if ncolors.dtype != torch.int32 or ncolors.numel() < 1 or not ncolors.is_cuda:
        raise ValueError("ncolors must be an int32 device tensor")
    m = colidx.numel() if nnz is None else int(nnz)
    rc = lib.csrcolor_color_noalloc(n, m, rowptr.data_ptr(), colidx.data_ptr() if colidx.numel() else None,
                                    out.data_ptr(), ncolors.data_ptr(), _stream_ptr(stream))
    L.check(rc)


def color_raw(n: int, rowptr_ptr: int, colidx_ptr: int, out_ptr: int,
              stream: Optional[torch.cuda.Stream] = None) -> int:
    """csrcolor_color on raw device pointers; returns the status code unchanged."""
    lib = L.load()
    nc = ctypes.c_int32(0)
    rc = lib.csrcolor_color(n, rowptr_ptr, colidx_ptr, out_ptr, ctypes.byref(nc), _stream_ptr(stream))
    return rc if rc != L.OK else int(nc.value)


def color_batched(voff: torch.Tensor, rowptr: torch.Tensor, colidx: torch.Tensor,
                  out: Optional[torch.Tensor] = None, opts: Optional[L.Opts] = None,
                  stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Colour G graphs stored block-diagonally.  Returns (colors, ncolors int32[G])."""
    lib = L.load()
    n = _check_csr(rowptr, colidx)
    if voff.dtype != torch.int64 or not voff.is_cuda or voff.dim() != 1 or voff.numel() < 1:
        raise TypeError("voff must be an int64 device tensor with G+1 entries")
    G = voff.numel() - 1
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=rowptr.device)
    ncol = torch.empty(max(G, 1), dtype=torch.int32, device=rowptr.device)
    rc = lib.csrcolor_color_batched(G, n, voff.data_ptr(), rowptr.data_ptr(), colidx.data_ptr(),
                                    out.data_ptr(), ncol.data_ptr(),
                                    ctypes.byref(opts) if opts is not None else None, _stream_ptr(stream))
    L.check(rc)
    return out[:n], ncol[:G]


def color_multi(graphs: Sequence[Tuple[torch.Tensor, torch.Tensor]], outs: Optional[Sequence[torch.Tensor]] = None,
                nnz: Optional[Sequence[int]] = None, opts: Optional[L.Opts] = None,
                stream: Optional[torch.cuda.Stream] = None) -> Tuple[List[torch.Tensor], torch.Tensor]:
    """Colour several separate graphs (device (rowptr, colidx) pairs) in one library
    call.  Returns (per-graph colour tensors, ncolors int32[G] on the device).  `nnz`
    gives each graph's arc count (default: colidx.numel())."""
    lib = L.load()
    G = len(graphs)
    ns = (ctypes.c_int32 * max(G, 1))()
    es = (ctypes.c_int64 * max(G, 1))()
    rps = (ctypes.c_void_p * max(G, 1))()
    cis = (ctypes.c_void_p * max(G, 1))()
    cos = (ctypes.c_void_p * max(G, 1))()
    if outs is None:
        outs = [torch.empty(max(rp.numel() - 1, 0), dtype=torch.int32, device=rp.device) for rp, _ in graphs]
    for g, (rp, ci) in enumerate(graphs):
        n = _check_csr(rp, ci) if ci.numel() else rp.numel() - 1
        ns[g] = n
        es[g] = int(nnz[g]) if nnz is not None else ci.numel()
        rps[g] = rp.data_ptr()
        cis[g] = ci.data_ptr() if ci.numel() else None
        cos[g] = outs[g].data_ptr() if n else None
    dev = graphs[0][0].device if G else torch.device("cuda")
    ncol = torch.empty(max(G, 1), dtype=torch.int32, device=dev)
    rc = lib.csrcolor_color_multi(G, ctypes.addressof(ns), ctypes.addressof(es), ctypes.addressof(rps),
                                  ctypes.addressof(cis), ctypes.addressof(cos), ncol.data_ptr(),
                                  ctypes.byref(opts) if opts is not None else None, _stream_ptr(stream))
    L.check(rc)
    return [o[:ns[g]] for g, o in enumerate(outs)], ncol[:G]


def release_workspace() -> None:
    L.load().csrcolor_release_workspace()


def workspace_bytes(n: int, nnz: int, graphs: int = 0) -> int:
    """Upper bound of the device bytes one stream's workspace needs for a graph (or, with
    graphs >= 1, a union given to color_multi) of n vertices and nnz arcs."""
    return int(L.load().csrcolor_workspace_bytes(graphs, n, nnz))


def device_bytes_in_use() -> int:
    """Device bytes the library's workspaces hold now."""
    return int(L.load().csrcolor_device_bytes_in_use())

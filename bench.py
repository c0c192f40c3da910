#!/usr/bin/env python3
"""Benchmark: arcs/s of one round-complete speculative-greedy colouring on MI355X.

A step is one complete colouring (every round until the worklist is empty) of a
synthetic graph whose CSR is already resident in HBM; the workload defaults to the
27-point stencil on a 128^3 grid (2,097,152 vertices, 53,645,816 arcs).

Printed (one JSON line on stdout): value = arcs / second over the K timed steps;
``roofline`` for the dominant kernel (FirstFit) from its algorithmic bytes and its
average launch time, measured with HIP events on the library's stream during a
second pass of K steps; ``cpu_baseline`` = the serial CPU oracle on the same graph.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak, GB/s


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_graph(workload: str, seed: int):
    from paper_1606_06025_amd import graphs as gg
    if workload == "stencil128":
        return gg.config_stencil128()
    if workload == "er16k":
        return gg.config_er16k(seed)
    if workload == "rmat23":
        return gg.config_rmat23(seed)
    if workload.startswith("rmat"):
        return gg.rmat(int(workload[4:]), 16, seed)
    if workload.startswith("stencil"):
        L = int(workload[7:])
        return gg.stencil27(L, L, L)
    raise SystemExit(f"unknown workload {workload}")


def assign_bytes(wsize, arcs) -> int:
    """Algorithmic bytes of every FirstFit launch (rounds 2..R): per worklist vertex
    16 B (its id, the rowptr pair, the colour write) + per scanned arc 8 B (colidx
    entry + the neighbour's colour)."""
    return sum(16 * int(w) + 8 * int(a) for w, a in zip(wsize[1:], arcs[1:]))


def cpu_baseline(g, budget_s: float = 20.0):
    import oracle
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.sgr(g.n, g.rowptr, g.colidx)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s * 0.5 or el / reps * (reps + 1) > budget_s:
            break
    per = el / reps
    return {"value": g.nnz / per, "unit": "arcs/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full serial colouring(s) of {g.name} ({g.nnz} arcs), "
                      f"{per:.2f} s each, single thread"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="stencil128")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--mode", type=int, default=0, help="csrcolor_mode (0 = library default)")
    ap.add_argument("--lane-assign", type=int, default=0, help="csrcolor_opts.lane_assign (0 = default)")
    ap.add_argument("--lane-detect", type=int, default=0, help="csrcolor_opts.lane_detect (0 = default)")
    ap.add_argument("--t-wave", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--sync-every", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build colours one graph on one GPU; runs on more than one GPU "
              "are not supported (use --gpus 1).", file=sys.stderr)
        return 2

    import torch
    import numpy as np
    from paper_1606_06025_amd import api, _lib

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    _lib.load()
    dev = torch.device("cuda:0")

    log(f"generating {args.workload} (seed {args.seed})")
    g = make_graph(args.workload, args.seed)
    log(f"n={g.n} nnz={g.nnz} maxdeg={g.max_degree()}")
    rp = torch.from_numpy(g.rowptr).to(dev)
    ci = torch.from_numpy(g.colidx).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    tuned = dict(mode=args.mode, lane_assign=args.lane_assign, lane_detect=args.lane_detect,
                 t_wave=args.t_wave, blocks_per_cu=args.blocks_per_cu, sync_every=args.sync_every)
    opts = api.make_opts(**tuned) if any(tuned.values()) else None

    # warmup (also allocates the library workspace)
    for _ in range(args.warmup):
        api.color(rp, ci, out=out, opts=opts)
    torch.cuda.synchronize()
    log("warmup done")

    # timed region: exactly K complete colourings
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    ncolors = 0
    for _ in range(args.steps):
        _, ncolors, _ = api.color(rp, ci, out=out, opts=opts)
    stop.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ev_ms = start.elapsed_time(stop)
    ms_per_step = max(wall_ms, ev_ms) / args.steps
    value = g.nnz / (ms_per_step * 1e-3)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value / 1e9:.3f} G arcs/s")

    # second pass: per-kernel HIP-event timing and round statistics
    _, _, st = api.color(rp, ci, out=out, opts=opts, stats=True, stats_cap=1 << 16)
    roofline = None
    kern = {}
    if not args.no_kernel_timing:
        tot_a = tot_d = tot_s = 0.0
        na = nd = 0
        for _ in range(args.steps):
            _, _, s2 = api.color(rp, ci, out=out, opts=opts, stats=True, stats_cap=1 << 16,
                                 time_kernels=True)
            tot_a += s2.ms_assign
            tot_d += s2.ms_detect
            tot_s += s2.ms_setup
            na += s2.n_assign
            nd += s2.n_detect
        ab = assign_bytes(st.wsize, st.arcs)
        launches_per_step = na / args.steps
        avg_launch_ms = tot_a / na if na else float("nan")
        bytes_per_launch = ab / launches_per_step if launches_per_step else 0.0
        achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if na else 0.0
        roofline = {"bound": "hbm", "kernel": "k_assign (FirstFit)", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None, "bytes_per_launch": round(bytes_per_launch),
                    "avg_launch_us": round(avg_launch_ms * 1e3, 2),
                    "launches_per_step": launches_per_step}
        kern = {"ms_assign_per_step": round(tot_a / args.steps, 3),
                "ms_detect_per_step": round(tot_d / args.steps, 3),
                "ms_setup_per_step": round(tot_s / args.steps, 3)}
        log(f"kernel time per step: assign {kern['ms_assign_per_step']} ms, detect "
            f"{kern['ms_detect_per_step']} ms, setup {kern['ms_setup_per_step']} ms")

    import oracle
    ff_colors = oracle.serial_ff(g.n, g.rowptr, g.colidx)[1]
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(g)

    rec = {
        "metric": "arcs/s per round-complete coloring",
        "value": value,
        "unit": "arcs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": g.name, "n": g.n, "nnz": g.nnz, "rounds": st.rounds,
                   "ncolors": ncolors, "serial_ff_colors": ff_colors,
                   "colors_vs_serial_ff": round(ncolors / ff_colors, 4) if ff_colors else None,
                   **{k: v for k, v in tuned.items() if v}, **kern},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

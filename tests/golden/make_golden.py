"""Write stored oracle results for the full-size workloads (run by hand; the GPU tests
read the JSON files this writes).

Calls only the seeded generators and the CPU oracle.  For each workload it stores
SHA-256 digests of the generated CSR arrays (so a test can confirm it regenerated the
same graph) and of the oracle's colouring, plus the colour count, the round count and
the per-round worklist sizes and scanned-arc counts.

    python tests/golden/make_golden.py [rmat23] [stencil128] [er16k] [batched]

`batched` is the batched workload (2048 graphs, half Erdos-Renyi, half 27-point
stencils, seed 1): per graph the oracle's colour count, round count and the first 16 hex
digits of the SHA-256 of its colouring, plus the SHA-256 of the union colouring (the
graphs' colourings concatenated in union order) and of the union CSR.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1606_06025_amd import graphs as gg  # noqa: E402

WORKLOADS = {
    "rmat23": lambda: gg.config_rmat23(1),
    "stencil128": gg.config_stencil128,
    "er16k": lambda: gg.config_er16k(1),
}


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def main(names):
    for name in names:
        t0 = time.time()
        g = WORKLOADS[name]()
        t1 = time.time()
        res = oracle.sgr(g.n, g.rowptr, g.colidx)
        t2 = time.time()
        ff = oracle.serial_ff(g.n, g.rowptr, g.colidx)[1]
        rec = {
            "workload": g.name, "n": g.n, "nnz": g.nnz, "max_degree": g.max_degree(),
            "rowptr_sha256": digest(g.rowptr), "colidx_sha256": digest(g.colidx),
            "colors_sha256": digest(res.colors), "ncolors": res.ncolors, "rounds": res.rounds,
            "serial_ff_colors": ff,
            "wsize": [int(x) for x in res.wsize], "arcs_ff": [int(x) for x in res.arcs_ff],
            "arcs_cr": [int(x) for x in res.arcs_cr],
            "note": "written by tests/golden/make_golden.py from the CPU oracle",
        }
        with open(os.path.join(HERE, f"{name}_s1.json"), "w") as f:
            json.dump(rec, f)
        print(f"{name}: gen {t1 - t0:.1f} s, oracle {t2 - t1:.1f} s, ncolors {res.ncolors}, rounds {res.rounds}",
              flush=True)


def batched(G: int = 2048, seed: int = 1, threads: int = 8):
    import concurrent.futures
    t0 = time.time()
    specs = gg.batch_specs(G, seed=seed)
    parts = gg.build_graphs(specs)
    b = gg.concat_graphs(parts)
    t1 = time.time()

    def run(p):
        # the C oracle runs outside the interpreter lock, so threads colour graphs in parallel
        return oracle.sgr(p.n, p.rowptr, p.colidx)

    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(run, parts))
    t2 = time.time()
    h = hashlib.sha256()
    for r in res:
        h.update(np.ascontiguousarray(r.colors, dtype=np.int32).tobytes())
    rec = {
        "workload": f"batched_{G}_graphs_s{seed}", "G": G, "n": b.n, "nnz": b.nnz,
        "voff_sha256": hashlib.sha256(np.ascontiguousarray(b.voff, dtype=np.int64).tobytes()).hexdigest(),
        "rowptr_sha256": digest(b.rowptr), "colidx_sha256": digest(b.colidx),
        "colors_sha256": h.hexdigest(),
        "ncolors": [int(r.ncolors) for r in res], "rounds": [int(r.rounds) for r in res],
        "colors_sha256_16": [digest(r.colors)[:16] for r in res],
        "note": "written by tests/golden/make_golden.py from the CPU oracle",
    }
    with open(os.path.join(HERE, "batched_s1.json"), "w") as f:
        json.dump(rec, f)
    print(f"batched: gen {t1 - t0:.1f} s, oracle {t2 - t1:.1f} s, G {G}, n {b.n}, nnz {b.nnz}, "
          f"max rounds {max(rec['rounds'])}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS) + ["batched"]
    if "batched" in names:
        batched()
    main([x for x in names if x != "batched"])

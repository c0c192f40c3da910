"""GPU: the full batched workload (2048 graphs, half Erdos-Renyi, half 27-point
stencils, seed 1; 62.2M vertices, 1.43G arcs) coloured as one block-diagonal union
in every drive mode and with the autotuner's options.  Every graph's colouring and
colour count are compared with the CPU oracle's, stored by tests/golden/make_golden.py
(which calls only the oracle): by independence of components (Sec. 3.1 rounds only
read neighbours, and the requeue rule is invariant under a constant id shift) each
graph must get exactly its stand-alone colouring."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1606_06025_amd import graphs as gg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "batched_s1.json")


def _sha(a, dtype=np.int32):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def union():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06025_amd import _lib
    _lib.load()
    gold = json.load(open(GOLD))
    print(f"generating the batched set ({gold['G']} graphs)", flush=True)
    parts = gg.build_graphs(gg.batch_specs(gold["G"], seed=1))
    b = gg.concat_graphs(parts)
    assert b.n == gold["n"] and b.nnz == gold["nnz"]
    assert _sha(b.voff, np.int64) == gold["voff_sha256"]
    assert _sha(b.rowptr) == gold["rowptr_sha256"] and _sha(b.colidx) == gold["colidx_sha256"]
    dev = torch.device("cuda:0")
    d = (torch.from_numpy(b.voff).to(dev), torch.from_numpy(b.rowptr).to(dev), torch.from_numpy(b.colidx).to(dev))
    del parts
    return b, d, gold


def _check(b, gold, colors, ncol):
    """Per-graph digests and counts against the oracle's; returns the graphs that differ."""
    colors = colors.cpu().numpy()
    ncol = ncol.cpu().numpy()
    bad = []
    for g in range(b.G):
        c = colors[b.voff[g]:b.voff[g + 1]]
        if _sha(c)[:16] != gold["colors_sha256_16"][g] or int(ncol[g]) != gold["ncolors"][g]:
            bad.append(g)
    return bad


@pytest.mark.parametrize("mode", [1, 2, 3], ids=["loop", "persistent", "graph"])
def test_batched_full_set_matches_oracle(union, mode):
    from paper_1606_06025_amd import api
    b, (voff, rp, ci), gold = union
    out = torch.empty(b.n, dtype=torch.int32, device=rp.device)
    for _ in range(2):     # the second call runs on the sized workspace
        out.fill_(-1)
        _, ncol = api.color_batched(voff, rp, ci, out=out, opts=api.make_opts(mode=mode))
        torch.cuda.synchronize()
        bad = _check(b, gold, out, ncol)
        assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:5]}"


def test_batched_full_set_tuned(union, tmp_path):
    """The autotuner's pick on the union (times candidates; none changes colourings)."""
    from paper_1606_06025_amd import api, tune
    b, (voff, rp, ci), gold = union
    opts = tune.tune(rp, ci, voff=voff, reps=1, cache=str(tmp_path / "tune.json"),
                     log=lambda m: print(m, flush=True))
    print("tuned:", opts, flush=True)
    out = torch.empty(b.n, dtype=torch.int32, device=rp.device)
    _, ncol = api.color_batched(voff, rp, ci, out=out, opts=api.make_opts(**opts) if opts else None)
    torch.cuda.synchronize()
    bad = _check(b, gold, out, ncol)
    assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:5]}"

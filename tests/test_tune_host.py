"""Autotuner logic on the host (no GPU): coordinate descent finds the optimum of a
separable synthetic cost, the signature is stable and coarse, the cache round-trips."""
import numpy as np

from paper_1606_06025_amd import graphs as gg
from paper_1606_06025_amd import tune


def test_coordinate_descent_separable():
    target = {"a": 3, "b": 7}
    knobs = [("a", (1, 2, 3, 4)), ("b", (5, 6, 7))]

    def cost(cfg):
        return abs(cfg.get("a", 1) - target["a"]) + abs(cfg.get("b", 5) - target["b"]) + 1.0

    best, t, evals = tune.coordinate_descent(cost, knobs)
    assert best == target and t == 1.0 and evals == 1 + 3 + 2


def test_signature_coarse_and_stable():
    a = gg.erdos_renyi(5000, 40000, 1)
    b = gg.erdos_renyi(5000, 40000, 2)
    c = gg.rmat(14, 16, 1)
    assert tune.signature(a.rowptr) == tune.signature(a.rowptr)
    assert tune.signature(a.rowptr) == tune.signature(b.rowptr)
    assert tune.signature(a.rowptr) != tune.signature(c.rowptr)


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "t.json")
    tune._save(p, {"k": {"opts": {"mode": 3}}})
    assert tune._load(p)["k"]["opts"] == {"mode": 3}
    assert tune._load(str(tmp_path / "missing.json")) == {}

"""Autotuner host logic (CPU) and its effect on a Simulator (GPU)."""
import numpy as np
import pytest

from paper_2605_29514_amd import tune
from paper_2605_29514_amd import workload as W


def test_pick_fastest_and_ties():
    t = {(1, 0, 0): 5.0, (2, 128, 0): 3.0, (2, 64, 0): 3.0, (2, 256, 64): 9.0}
    assert tune.pick(t) == (2, 64, 0)                   # tie -> earlier candidate
    assert tune.pick({(2, 256, 64): 1.0, (1, 0, 0): 2.0}) == (2, 256, 64)
    assert all(c[0] == 2 for c in tune.FUSED) and set(tune.FUSED) < set(tune.CANDIDATES)


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("STN_TUNE_CACHE", path)
    assert tune.load_cache() == {}
    k = tune.problem_key("gfx950", 49, 1024, 256, "fp32", "d5")
    tune.store_cache(k, {"choice": [2, 128], "ms": {"2/128": 1.0}})
    tune.store_cache("other", {"choice": [1, 0]})
    got = tune.load_cache()
    assert got[k]["choice"] == [2, 128] and got["other"]["choice"] == [1, 0]
    with open(path, "w") as f:
        f.write("not json")
    assert tune.load_cache() == {}


def test_layers_stop():
    ops = [("gates",), ("rotate",), ("noise",), ("rotate",), ("measure",)]
    assert tune.layers_stop(ops, 1) == 2
    assert tune.layers_stop(ops, 2) == 4
    assert tune.layers_stop(ops, 3) == 5
    assert tune.layers_stop(ops, 1, start=2) == 4       # counted from the window start


@pytest.mark.gpu
def test_autotune_leaves_initial_state(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29514_amd import stn
    monkeypatch.setenv("STN_TUNE_CACHE", str(tmp_path / "tune.json"))
    circ = W.memory_circuit(3, 2, 64, seed=71, theta_law="per_coupling", nnn=True, p=0.01)
    sim = stn.Simulator(circ.n, circ.n_shots, 8, "fp64")
    ops = stn.prepare(circ)
    r = tune.autotune(sim, ops, tune.layers_stop(ops, 2), key="k")
    assert r["choice"] in tune.CANDIDATES and not r["cached"]
    got = stn.run_circuit(circ, 8, "fp64", sim=sim)
    ref = stn.run_circuit(circ, 8, "fp64", layer_mode=r["choice"][0], layer_threads=r["choice"][1],
                          layer_lds=r["choice"][2])
    assert np.array_equal(got["records"], ref["records"])
    assert np.array_equal(got["prob"], ref["prob"])
    again = tune.autotune(sim, ops, tune.layers_stop(ops, 2), key="k")
    assert again["cached"] and again["choice"] == r["choice"]
    # a window inside the second round, reached once and restored per candidate
    start = next(i for i, op in enumerate(ops) if op[0] == "measure") + 1
    w = tune.autotune(sim, ops, tune.layers_stop(ops, 2, start), start=start, key="k2")
    assert w["choice"] in tune.CANDIDATES and not w["cached"]
    got = stn.run_circuit(circ, 8, "fp64", sim=sim)
    ref = stn.run_circuit(circ, 8, "fp64", layer_mode=w["choice"][0], layer_threads=w["choice"][1],
                          layer_lds=w["choice"][2])
    assert np.array_equal(got["records"], ref["records"])
    assert np.array_equal(got["prob"], ref["prob"])

"""Profiling hooks of the library on the GPU: the device work counters and
the timing-only mode (launch events without counters) leave every result
unchanged; timing-only records launches and times but counts no work; the
counted pass counts the same launches and positive work."""
import numpy as np
import pytest

from paper_2605_29514_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29514_amd import stn
    stn.load()
    return stn


@pytest.mark.parametrize("threads", [64, 128])
def test_timing_only_profile(B, threads):
    circ = W.memory_circuit(3, 2, 64, seed=13, theta_law="per_coupling", nnn=True, p=0.01)
    ref = B.run_circuit(circ, 8, "fp32", layer_mode=2, layer_threads=threads)
    outs = {}
    for counters in (False, True):
        sim = B.Simulator(circ.n, circ.n_shots, 8, "fp32", layer_mode=2, layer_threads=threads)
        sim.profile(None, counters=counters)
        got = B.run_circuit(circ, 8, "fp32", sim=sim)
        prof = sim.profile_read()
        sim.profile([])
        assert np.array_equal(got["records"], ref["records"])
        assert np.array_equal(got["prob"], ref["prob"])
        outs[counters] = prof
    t, c = outs[False], outs[True]
    assert t["layer"]["launches"] > 0 and t["layer"]["launches"] == c["layer"]["launches"]
    assert t["expect"]["launches"] == c["expect"]["launches"] > 0
    assert t["layer"]["ms"] > 0
    assert t["layer"]["flops"] == 0 and t["layer"]["bytes"] == 0 and t["eigen_sweeps"] == 0
    assert c["layer"]["flops"] > 0 and c["layer"]["bytes"] > 0 and c["eigen_sweeps"] > 0

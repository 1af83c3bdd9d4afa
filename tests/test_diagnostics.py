"""Truncation diagnostics: detection rates (CPU, hand-made records) and the
device Schmidt spectrum (GPU: stn_spectrum against the oracle MPS's
schmidt_values, which tests/test_oracle_pins.py pins to a dense SVD)."""
import numpy as np
import pytest

from paper_2605_29514_amd import diagnostics as D
from paper_2605_29514_amd import workload as W


def test_detection_rates():
    circ = W.memory_circuit(3, 3, 4, seed=1, theta_nn=0.0)
    rounds = D.measurement_rounds(circ)
    assert [len(q) for q in rounds] == [8, 8, 8]
    rec = np.zeros((4, circ.n_measurements), np.uint8)
    assert D.detection_rates(circ, rec) == [0.0, 0.0, 0.0]
    # shot 0: one ancilla flips in round 2 and stays flipped
    rec[0, 8 + 0] = 1
    rec[0, 16 + 0] = 1
    r = D.detection_rates(circ, rec)
    assert r[1] == pytest.approx(1 / 32) and r[2] == 0.0
    # round 1 counts only the Z checks
    zc = [i for i, qq in enumerate(rounds[0]) if int(qq) in set(circ.layout.z_anc)]
    rec2 = np.zeros_like(rec)
    rec2[:, zc[0]] = 1
    assert D.detection_rates(circ, rec2)[0] == pytest.approx(1 / len(zc))


@pytest.mark.gpu
def test_chi_sweep_spectra_match_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import stn as ostn
    from paper_2605_29514_amd import stn
    stn.load()
    circ = W.memory_circuit(3, 2, 4, seed=17, theta_nn=0.1, nnn=True)
    res = D.chi_sweep(circ, [2, 64], "fp64", shot=1)
    assert max(res[64]["trunc_err"]) < 1e-10 < max(res[2]["trunc_err"])
    stops = [i for i, op in enumerate(circ.ops) if op["op"] == "measure" and op["reset"]]
    for k, stop in enumerate(stops):
        o = ostn.run_shot(circ, 1, chi_max=64, eps_cut=1e-14, stop_after_ops=stop)
        sv = o.mps.schmidt_values(circ.n // 2 - 1) ** 2
        ref = sv / sv.sum()
        got = np.array(res[64]["spectra"][k])
        m = min(len(ref), len(got))
        assert np.allclose(got[:m], ref[:m], atol=1e-10), k
        assert np.allclose(ref[m:], 0, atol=1e-10) and np.allclose(got[m:], 0, atol=1e-10)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_device_spectrum_every_shot_every_cut(prec):
    """stn_spectrum for all shots at several cuts of a d=3 two-round run
    (bonds up to 16) equals the oracle's Schmidt values (FP64 1e-10, FP32
    1e-6 absolute on values normalised to sum 1); the bond dimension it
    reports equals the GPU state's."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import stn as ostn
    from paper_2605_29514_amd import stn
    stn.load()
    circ = W.memory_circuit(3, 2, 6, seed=19, theta_law="per_coupling", nnn=True, p=0.01)
    g = stn.run_circuit(circ, 64, prec, 1e-14 if prec == "fp64" else 1e-12)
    sim = g["sim"]
    ores = [ostn.run_shot(circ, s, chi_max=64, eps_cut=1e-14 if prec == "fp64" else 1e-12) for s in range(6)]
    tol = 1e-10 if prec == "fp64" else 1e-6
    for bond in (1, 5, circ.n // 2, circ.n - 2):
        vals, rank = sim.spectrum(bond)
        vals, rank = vals.cpu().numpy(), rank.cpu().numpy()
        assert np.array_equal(rank, sim.bonds()[:, bond])
        for s, o in enumerate(ores):
            if not np.array_equal(g["records"][s], np.array(o.record, np.uint8)):
                continue                    # a near-tie record: another trajectory
            sv = o.mps.copy().schmidt_values(bond - 1) ** 2
            ref = sv / sv.sum()
            m = min(len(ref), vals.shape[1])
            assert np.allclose(vals[s, :m], ref[:m], atol=tol), (bond, s)
            assert abs(vals[s].sum() - 1) < 1e-9

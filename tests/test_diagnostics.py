"""Truncation diagnostics: Schmidt spectra of a returned state and detection
rates (CPU: against a dense SVD and hand-made records; GPU: the chi sweep's
spectra against the oracle's MPS at the same points)."""
import numpy as np
import pytest

from paper_2605_29514_amd import diagnostics as D
from paper_2605_29514_amd import workload as W


def random_mps(n, rng, bond=3):
    dims = [1] + [min(bond, 2 ** min(j, n - j)) for j in range(1, n)] + [1]
    return [rng.normal(size=(dims[j], 2, dims[j + 1])) + 1j * rng.normal(size=(dims[j], 2, dims[j + 1]))
            for j in range(n)]


def dense(ts):
    v = ts[0]
    for t in ts[1:]:
        v = np.tensordot(v, t, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


@pytest.mark.parametrize("cut", [0, 2, 4])
def test_schmidt_values_match_dense_svd(cut):
    rng = np.random.default_rng(cut)
    ts = random_mps(6, rng)
    psi = dense(ts)
    s = np.linalg.svd(psi.reshape(2 ** (cut + 1), -1), compute_uv=False) ** 2
    s = s / s.sum()
    got = D.schmidt_values(ts, cut)
    assert np.allclose(got, s[:len(got)], atol=1e-12)
    assert abs(got.sum() - 1) < 1e-12


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
        ref = D.schmidt_values(o.mps.A, circ.n // 2 - 1)
        got = np.array(res[64]["spectra"][k])
        m = min(len(ref), len(got))
        assert np.allclose(got[:m], ref[:m], atol=1e-10), k

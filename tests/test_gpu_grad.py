"""GPU adjoint gradient of log P(record) against the dense gradient oracle.

The oracle (oracle/grad.py) runs each shot, records its steps and computes
dJ/dtheta by a dense adjoint pinned by finite differences and, without
truncation, by the physical statevector; the GPU runs the same circuits
with the oracle's records forced, checkpointed per stretch, and its adjoint
pass (stn_backward) must give the same gradient: FP64 to 1e-8 and FP32 to
1e-4 relative to the largest entry.  Shots whose truncation is
ill-conditioned at a binding cut are skipped, as in the parity tests, and so
are shots where the chi decision at some cut is within a factor MIN_MARGIN of
the relative cut eps: whether such a step counts as truncated (and gets a
frozen projector) is then set by rounding: the GPU's squared Schmidt values
near the cut carry errors of about a tenth of eps times their sum.
"""
import sys

import numpy as np
import pytest

from oracle import grad as G
from oracle import stn as ostn
from paper_2605_29514_amd import workload as W
from tests._circuits import entangling_circuit

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-8, "fp32": 1e-4}
EPS = {"fp64": 1e-14, "fp32": 1e-12}
# the FP32 limit is the parity tests' one: sensitivity x 2^-24 up to 1e-5
MAX_SENS = {"fp64": 1e6, "fp32": 1e-5 / 2.0 ** -24}
MIN_MARGIN = 10.0


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29514_amd import adjoint, stn
    stn.load()
    return adjoint


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_case(circ, chi, prec):
    tapes, recs, sens = [], [], []
    for s in range(circ.n_shots):
        t = G.record(circ, s, chi, EPS[prec])
        tapes.append(t)
        r = ostn.run_shot(circ, s, chi_max=chi, eps_cut=EPS[prec])
        recs.append(r.record)
        sens.append((r.cut_sensitivity, r.flag_margin))
    return tapes, np.array(recs, np.uint8), sens


def check(A, circ, chi, prec, segments=None):
    say(f"gradient n={circ.n} S={circ.n_shots} chi={chi} {prec}")
    tapes, recs, sens = oracle_case(circ, chi, prec)
    run = A.GradientRun(circ, chi, recs, prec, EPS[prec], segments=segments)
    lp = run.forward().cpu().numpy()
    g = run.backward().cpu().numpy()
    assert not run.adjoint_truncated.any(), "adjoint bond cap reached"
    used = 0
    for s, t in enumerate(tapes):
        if sens[s][0] > MAX_SENS[prec] or sens[s][1] < MIN_MARGIN:
            say(f"  shot {s}: skipped (cut sensitivity {sens[s][0]:.3g}, chi decision margin {sens[s][1]:.3g})")
            continue
        used += 1
        go = G.adjoint_gradient(t)
        scale = max(1.0, float(np.abs(go).max()))
        err = float(np.abs(g[s] - go).max()) / scale
        say(f"  shot {s}: logp {lp[s]:.12f} vs {t.logp:.12f}, max |g| {np.abs(go).max():.3e}, rel err {err:.2e}, "
            f"truncating steps {sum(x.truncated for x in t.steps)}")
        assert abs(lp[s] - t.logp) <= TOL[prec] * max(1.0, abs(t.logp))
        assert err <= TOL[prec], f"shot {s}: gradient error {err:.3e}"
    assert used >= max(1, circ.n_shots // 2)
    return g


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("chi", [64, 3, 2])
def test_gradient_matches_oracle(A, prec, chi):
    circ = entangling_circuit(9, 6, 4, 1)
    check(A, circ, chi, prec)


@pytest.mark.parametrize("chi", [64, 4])
def test_gradient_d3_memory(A, chi):
    """d=3 memory experiment, 2 rounds, one angle per rotation instance (the
    c4 parametrisation at d=3), Pauli noise; chi 64 is exact, chi 4 binds."""
    circ = W.memory_circuit(3, 2, 4, seed=5, theta_nn=0.1, p=0.02, per_layer_params=True)
    check(A, circ, chi, "fp64")


def test_gradient_matches_gpu_central_differences(A):
    """The adjoint gradient against central differences (h = 1e-4) of the
    GPU's own FP64 forward log P on a d=3 two-round memory experiment at chi
    64 (exact: no truncation), one angle per rotation instance: the forward
    runs the base angles and every +h / -h move of six round-2 angles as
    shots of one batch with the same forced record (the first round's
    gradient vanishes, every outcome there has probability 1/2 or 1)."""
    import torch
    P = 6
    S = 1 + 2 * P
    circ = W.memory_circuit(3, 2, S, seed=5, theta_nn=0.1, p=0.0, per_layer_params=True)
    rec = np.array(ostn.run_shot(circ, 0, chi_max=64, eps_cut=EPS["fp64"]).record, np.uint8)
    run = A.GradientRun(circ, 64, np.tile(rec, (S, 1)), "fp64", EPS["fp64"])
    th0 = np.concatenate([op["theta"] for op in circ.ops if op["op"] == "rotate"], axis=1)[0]
    picks = np.linspace(run.R // 2, run.R - 1, P).astype(int)
    h = 1e-4
    th = np.tile(th0, (S, 1))
    for i, q in enumerate(picks):
        th[1 + i, q] += h
        th[1 + P + i, q] -= h
    run.set_theta(torch.tensor(th, dtype=torch.float64, device="cuda:0"))
    lp = run.forward().cpu().numpy()
    g = run.backward().cpu().numpy()
    assert not run.adjoint_truncated.any()
    fd = (lp[1:1 + P] - lp[1 + P:]) / (2 * h)
    ad = g[0, picks]
    err = float(np.abs(fd - ad).max())
    say(f"  adjoint {np.array2string(ad, precision=8)}\n  central {np.array2string(fd, precision=8)}\n"
        f"  max abs diff {err:.2e}")
    assert float(np.abs(ad).max()) > 1e-4
    assert err <= 1e-6 * max(1.0, float(np.abs(ad).max()))


def test_checkpoint_stretches_agree(A):
    """One stretch over the whole circuit and one per measurement give the
    same gradient (the adjoint state carries over between stretches)."""
    circ = entangling_circuit(9, 6, 2, 3)
    tapes, recs, _ = oracle_case(circ, 3, "fp64")
    a = A.GradientRun(circ, 3, recs, "fp64", EPS["fp64"])
    a.forward()
    ga = a.backward().cpu().numpy()
    b = A.GradientRun(circ, 3, recs, "fp64", EPS["fp64"], segments=[(0, len(a.ops))])
    b.forward()
    gb = b.backward().cpu().numpy()
    assert len(a.segments) > 2
    assert np.max(np.abs(ga - gb)) <= 1e-9 * max(1.0, np.abs(gb).max())


def test_adjoint_cap_is_reported(A):
    """A cap equal to the forward's is too small for this adjoint: the flag says so."""
    circ = W.memory_circuit(3, 2, 2, seed=5, theta_nn=0.1, p=0.02, per_layer_params=True)
    _, recs, _ = oracle_case(circ, 4, "fp64")
    run = A.GradientRun(circ, 4, recs, "fp64", EPS["fp64"], chi_adj=4)
    run.forward()
    run.backward()
    assert run.adjoint_truncated.any()


def test_autograd_function(A):
    import torch
    circ = entangling_circuit(9, 6, 3, 2)
    _, recs, _ = oracle_case(circ, 64, "fp64")
    run = A.GradientRun(circ, 64, recs, "fp64", EPS["fp64"])
    th = np.concatenate([op["theta"] for op in circ.ops if op["op"] == "rotate"], axis=1)
    theta = torch.tensor(th, dtype=torch.float64, device="cuda:0", requires_grad=True)
    f = A.CircuitLogProb(run)
    lp = f(theta)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda:0")
    (lp * w).sum().backward()
    ref = np.stack([G.adjoint_gradient(G.record(circ, s, 64, EPS["fp64"])) for s in range(3)])
    got = theta.grad.cpu().numpy()
    assert np.allclose(got, ref * w.cpu().numpy()[:, None], atol=1e-8, rtol=1e-8)

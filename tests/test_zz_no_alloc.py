"""stn_tape_begin_static, the allocation-free variant of stn_tape_begin
(needs an MI355X): the gradient recorded into the library's static per-GPU
tape equals the one recorded into a caller buffer, bit for bit, on two
calls in a row, the second with a smaller input (fewer steps and shots)."""
import numpy as np
import pytest

from oracle import stn as ostn
from paper_2605_29514_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29514_amd import adjoint, stn
    stn.load()
    return adjoint


def grads(A, circ, chi, prec, static):
    recs = np.array([ostn.run_shot(circ, s, chi_max=chi, eps_cut=1e-14).record for s in range(circ.n_shots)],
                    np.uint8)
    run = A.GradientRun(circ, chi, recs, prec, 1e-14, static_tape=static)
    lp = run.forward().cpu().numpy()
    return lp, run.backward().cpu().numpy()


def test_static_tape_matches_caller_tape(A):
    big = W.memory_circuit(3, 2, 4, seed=77, theta_law="per_shot", theta_range=(0.02, 0.08), nnn=True, p=0.01)
    small = W.memory_circuit(3, 1, 2, seed=78, theta_nn=0.06, p=0.0)
    for circ in (big, small):            # the second call records fewer steps for fewer shots
        lp_a, g_a = grads(A, circ, 8, "fp64", static=False)
        lp_b, g_b = grads(A, circ, 8, "fp64", static=True)
        assert np.array_equal(lp_a, lp_b)
        assert np.array_equal(g_a, g_b)
        if circ is big:
            assert np.abs(g_a).max() > 0


def test_static_tape_rejects_oversized(A):
    from paper_2605_29514_amd import stn
    sim = stn.Simulator(49, 64, 64, "fp32", None, "cuda:0")
    steps = 10 ** 6
    with pytest.raises(stn.STNError) as e:
        sim.tape_begin_static(steps)
    assert e.value.status == -2 and "static tape" in str(e.value)

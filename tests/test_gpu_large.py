"""GPU parity at the bond dimensions the d=5 workload reaches from its second
syndrome round on (needs an MI355X).

Each test drives the fused per-shot kernel (or the per-step kernels) through
a named route and asserts, from the device branch counters
(stn_profile_paths), that the route was taken:
  * environment Grams for doubled bonds 65..128 with eigen-solves of order
    up to 128 in global scratch;
  * the Householder QR sweep (doubled bonds above 128, reflectors for more
    than 64 rows in global scratch) with eigen-solves of order above 128,
    and on the FP64 path the two-sided Jacobi above order 32;
  * chi_max binding on the FP32 path at orders above 64.
The comparison with the oracle uses the bars of test_gpu_parity.py.
"""
import numpy as np
import pytest

from _circuits import entangling_circuit
from oracle import stn as ostn
from test_gpu_parity import EPS, B, check_tableau, mps_fidelity, ptol_shot, say, _uniform_of, fp32_sens_limit  # noqa: F401

pytestmark = pytest.mark.gpu


def run_counted(B, circ, chi, prec, mode, forced=None, env=None, lds=0):
    lm, nt = mode
    sim = B.Simulator(circ.n, circ.n_shots, chi, prec, EPS[prec], "cuda:0", layer_mode=lm, layer_threads=nt,
                      layer_lds=lds)
    if env is not None:
        sim.set_layer_env(env)
    sim.profile(["layer", "expect"], counters=True)
    g = B.run_circuit(circ, chi, prec, EPS[prec], forced=forced, sim=sim)
    paths = sim.profile_paths()
    sim.profile([])
    return g, paths


def parity_large(B, circ, chi, prec, shots, mode, env=None, lds=0):
    say(f"large-bond parity n={circ.n} S={circ.n_shots} chi={chi} {prec} mode {mode}")
    eps = EPS[prec]
    ores = {s: ostn.run_shot(circ, s, chi_max=chi, eps_cut=eps) for s in shots}
    lim = 1e6 if prec == "fp64" else fp32_sens_limit()
    cmp = [s for s in shots if ores[s].cut_sensitivity <= lim]
    say(f"  oracle max bonds {[max(ores[s].bond_trace) for s in shots]}, sensitivities "
        f"{[round(ores[s].cut_sensitivity, 1) for s in shots]}, compared {len(cmp)} of {len(shots)}")
    assert cmp, "no well-conditioned shot"
    g, paths = run_counted(B, circ, chi, prec, mode, env=env, lds=lds)
    tie = 1e-9 if prec == "fp64" else 1e-4
    for s in cmp:
        rg, ro = g["records"][s], np.array(ores[s].record, np.uint8)
        if not np.array_equal(rg, ro):
            k = int(np.nonzero(rg != ro)[0][0])
            assert abs(_uniform_of(circ, s, k) - ores[s].p0[k]) <= tie, f"shot {s}: record differs at {k}"
    forced = np.array([ores[s].record if s in ores else g["records"][s] for s in range(circ.n_shots)], np.uint8)
    gf, _ = run_counted(B, circ, chi, prec, mode, forced=forced, env=env, lds=lds)
    errs = {}
    for s in cmp:
        po = np.array(ores[s].prob)
        errs[s] = float(np.max(np.abs(gf["prob"][s] - po) / po))
    say(f"  per-shot max rel p err / bar: " + ", ".join(f"{errs[s]:.2e}/{ptol_shot(prec, ores[s]):.2e}" for s in cmp))
    say(f"  paths {paths}")
    for s in cmp:
        assert errs[s] <= ptol_shot(prec, ores[s]), f"shot {s}: max relative probability error {errs[s]:.3e}"
    check_tableau(gf["sim"], ores, cmp)
    for s in cmp:
        f = mps_fidelity(gf["sim"], s, ores[s].mps)
        assert f <= ptol_shot(prec, ores[s]), f"shot {s} fidelity deficit {f:.3e}"
    return paths, ores


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_environment_path_doubled_bonds_to_256(B, prec):
    """Bonds reach 128: the environment Grams take doubled bonds up to 256
    (packed in the shot's store), and eigen-solves reach order 256."""
    circ = entangling_circuit(14, 20, 3, 7, meas_every=6)
    paths, ores = parity_large(B, circ, 128, prec, range(0, 3, 2), (2, 256))
    assert max(max(o.bond_trace) for o in ores.values()) == 128
    assert paths["env_steps"] > 0 and paths["qr_steps"] == 0 and paths["max_order"] == 256


@pytest.mark.parametrize("prec,lds", [("fp32", 32), ("fp32", 64), ("fp64", 0)])
def test_environment_path_orders_to_128(B, prec, lds):
    """Bonds reach 64 (chi_max 64 does not bind): truncations of order
    65..128 with rho in global scratch.  FP32: where the relative cut alone
    decides and its pivot count fits the LDS tile (42 with tile 32, 64 with
    tile 64), the kept space is the orthonormalised leading rows of the
    pivoted Cholesky factor; other cuts take the Gram of the factor in LDS or
    the one-sided Jacobi on the factor rows in global scratch."""
    circ = entangling_circuit(12, 20, 4, 7, meas_every=6)
    paths, ores = parity_large(B, circ, 64, prec, range(0, 4), (2, 256), lds=lds)
    assert max(max(o.bond_trace) for o in ores.values()) == 64
    assert paths["env_steps"] > 0 and paths["qr_steps"] == 0
    assert paths["eig_global"] > 0 and paths["max_order"] == 128
    if prec == "fp32":
        assert paths["cholqr"] > 0


@pytest.mark.parametrize("prec,mode", [("fp32", (2, 256)), ("fp64", (2, 256)), ("fp32", (2, 128)),
                                       ("fp32", (2, 512)), ("fp64", (1, 0))])
def test_qr_path_orders_to_256(B, prec, mode):
    """Bonds reach 128 and eigen-solves order 256.  The environment Grams are
    limited to doubled bonds of 64 here, so wider spans take the QR sweep
    (more than 64 rows: reflectors in global scratch); on the FP64 path the
    two-sided Jacobi runs above order 32 in global scratch.  The per-step
    kernels run the same sizes."""
    circ = entangling_circuit(14, 20, 3, 7, meas_every=6)
    paths, ores = parity_large(B, circ, 128, prec, range(0, 3, 2), mode, env=64)
    assert max(max(o.bond_trace) for o in ores.values()) == 128
    if mode[0] == 2:
        assert paths["qr_steps"] > 0 and paths["eig_global_gt128"] > 0 and paths["max_order"] == 256
        if prec == "fp64":
            assert paths["jacobi_global"] > 0


def test_fp32_chi_binding_at_orders_above_64(B):
    """chi_max = 48 binds at most cuts (half the weight is discarded over the
    run): the FP32 truncation of order up to 96 follows the oracle's SVD
    within the per-shot bar of the binding regime (test_gpu_parity.ptol_shot):
    here about 700 summed sensitivity, i.e. 3e-4 instead of 1e-5."""
    circ = entangling_circuit(14, 20, 4, 7, meas_every=6)
    paths, ores = parity_large(B, circ, 48, "fp32", range(0, 4), (2, 256))
    assert any(o.trunc_err > 0.1 for o in ores.values())
    assert paths["max_order"] == 96 and paths["eig_global"] > 0
    # binding cuts need the eigenvalues: not all global-scratch cuts can take
    # the Cholesky rows
    assert paths["cholqr"] < paths["eig_global"] + paths["eig_global_gt128"]

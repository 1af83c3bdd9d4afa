"""Pins of the gradient oracle (oracle/grad.py) -- CPU only.

* The frozen forward replays the recorded run: J at the recorded angles is
  the oracle's log P.
* The adjoint gradient equals central finite differences of the frozen
  forward (projectors held fixed), with and without chi_max truncation.
* Without truncation the gradient is that of the physical circuit: central
  finite differences of the brute-force statevector log-probability of the
  same record (no MPS, no frame).
* With real Clifford gates only (H, CNOT) J is even in the angles (the
  projectors are real too), so its gradient is odd.
A planted sign error in the adjoint fails the finite-difference pin.
"""
import copy

import numpy as np
import pytest

from oracle import grad as G
from oracle import statevector as SV
from tests._circuits import entangling_circuit


def _with_theta(circ, shot, index, value):
    c = copy.deepcopy(circ)
    k = 0
    for op in c.ops:
        if op["op"] == "rotate":
            R = len(op["paulis"])
            if index < k + R:
                op["theta"][shot, index - k] = value
                return c
            k += R
    raise IndexError(index)


def _theta_of(circ, shot, index):
    k = 0
    for op in circ.ops:
        if op["op"] == "rotate":
            R = len(op["paulis"])
            if index < k + R:
                return float(op["theta"][shot, index - k])
            k += R
    raise IndexError(index)


def _negated(circ):
    c = copy.deepcopy(circ)
    for op in c.ops:
        if op["op"] == "rotate":
            op["theta"] = -op["theta"]
    return c


@pytest.mark.parametrize("seed,chi", [(1, 64), (2, 64), (3, 2), (4, 3), (5, 2)])
def test_frozen_forward_replays_logp(seed, chi):
    circ = entangling_circuit(9, 6, 2, seed)
    for shot in range(2):
        tape = G.record(circ, shot, chi, 1e-16)
        assert abs(G.frozen_logp(tape) - tape.logp) <= 1e-10 * max(1.0, abs(tape.logp))


@pytest.mark.parametrize("seed,chi", [(1, 2), (2, 3), (3, 2), (5, 3)])
def test_adjoint_matches_frozen_fd_with_truncation(seed, chi):
    circ = entangling_circuit(9, 6, 1, seed)
    tape = G.record(circ, 0, chi, 1e-16)
    assert any(s.truncated for s in tape.steps), "case must truncate"
    assert any(s.kind == "meas" and s.pivot is not None for s in tape.steps)
    ga = G.adjoint_gradient(tape)
    gf = G.fd_gradient(tape, h=1e-5)
    assert np.max(np.abs(ga - gf)) <= 1e-7 * max(1.0, np.max(np.abs(gf)))


@pytest.mark.parametrize("seed", [1, 2, 7])
def test_untruncated_gradient_is_physical(seed):
    circ = entangling_circuit(8, 5, 1, seed)
    tape = G.record(circ, 0, 1 << 10, 1e-16)
    assert not any(s.truncated for s in tape.steps)
    ga = G.adjoint_gradient(tape)
    assert np.max(np.abs(ga)) > 1e-2
    rec = SV.run_shot(circ, 0)[0]
    h = 1e-5
    for i in range(tape.n_rot):
        t0 = _theta_of(circ, 0, i)
        lp = SV.run_shot(_with_theta(circ, 0, i, t0 + h), 0, forced=rec)[3]
        lm = SV.run_shot(_with_theta(circ, 0, i, t0 - h), 0, forced=rec)[3]
        fd = (lp - lm) / (2 * h)
        assert abs(ga[i] - fd) <= 1e-7 * max(1.0, abs(fd)), (i, ga[i], fd)


def test_d3_memory_gradient_is_physical():
    """d=3 memory experiment (17 qubits), 2 rounds, Pauli noise, one angle per
    rotation instance: sampled entries against statevector differences."""
    from paper_2605_29514_amd import workload as W
    circ = W.memory_circuit(3, 2, 1, seed=5, theta_nn=0.1, p=0.02, per_layer_params=True)
    tape = G.record(circ, 0, 1 << 10, 1e-16)
    ga = G.adjoint_gradient(tape)
    rec = SV.run_shot(circ, 0)[0]
    big = np.argsort(-np.abs(ga))[:4]
    pick = list(big) + [int(i) for i in np.random.default_rng(0).choice(tape.n_rot, 4, replace=False)]
    h = 1e-5
    for i in pick:
        t0 = _theta_of(circ, 0, i)
        lp = SV.run_shot(_with_theta(circ, 0, i, t0 + h), 0, forced=rec)[3]
        lm = SV.run_shot(_with_theta(circ, 0, i, t0 - h), 0, forced=rec)[3]
        fd = (lp - lm) / (2 * h)
        assert abs(ga[i] - fd) <= 1e-7 * max(1.0, abs(fd)), (i, ga[i], fd)
    assert np.abs(ga).max() > 0.1


def test_gradient_is_odd_in_theta():
    circ = entangling_circuit(8, 5, 1, 2, phase_gates=False)
    rec = SV.run_shot(circ, 0)[0]
    ta = G.record(circ, 0, 1 << 10, 1e-16, forced=rec)
    tb = G.record(_negated(circ), 0, 1 << 10, 1e-16, forced=rec)
    ga, gb = G.adjoint_gradient(ta), G.adjoint_gradient(tb)
    assert np.allclose(ga, -gb, atol=1e-9)
    assert np.max(np.abs(ga)) > 1e-3


def test_planted_sign_error_is_caught():
    circ = entangling_circuit(9, 6, 1, 2)
    tape = G.record(circ, 0, 2, 1e-16)
    real = G.apply_ops

    def bad_adjoint(t):                       # R instead of R^dag in the backward pass
        g = np.zeros(t.n_rot)
        mu = np.zeros((2,) * t.n, complex)
        for stp in reversed(t.steps):
            if stp.truncated:
                mu = G.project(mu, stp.l, stp.basis)
            if stp.kind == "rot":
                mu = (np.cos(stp.theta) * mu - 1j * stp.sigma * np.sin(stp.theta) * real(mu, stp.ops)) / stp.norm
                g[stp.index] = 2 * float(np.vdot(mu, -1j * stp.sigma * real(stp.phi, stp.ops)).real)
            else:
                mu = G._measure_map(stp, mu, adjoint=True) / stp.norm
                a = 0.5 * (stp.phi + stp.s * stp.sigma * real(stp.phi, stp.ops))
                mu = mu + a / stp.p - stp.phi
        return g

    gf = G.fd_gradient(tape)
    assert np.max(np.abs(bad_adjoint(tape) - gf)) > 1e-4

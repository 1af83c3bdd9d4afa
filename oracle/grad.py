"""Gradient of log P(record) with respect to the crosstalk angles.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Dense (2^n amplitudes),
for small n.  Parity pins: tests/test_oracle_grad.py (central finite
differences of the frozen forward below; without truncation, central finite
differences of the brute-force statevector log-probability; the theta ->
-theta oddness of the gradient).

Objective: J = sum_k log p_k over the measurements of one shot with a fixed
record (the quantity the sampler accumulates).  In the MPS frame the
non-Clifford steps of the STN run (Sec. IV.A-B) act on the frame vector phi
as linear maps F followed by renormalisation:
  rotation r:     F = T_r R_r,  R_r = cos(t) - i sigma sin(t) P'      (Eq. 4)
  measurement k:  F = T_k M_k,  M_k = (I + s sigma Z^z)/2 when P' has no X/Y
                                M_k = Pi0_k (I + s sigma P') with pivot k
                  and p_k = ||A_k phi_k||^2, A_k = (I + s sigma P'_k)/2.
Clifford gates, Pauli noise, frame changes and the record do not depend on
the angles.

Reading of "truncation projectors held fixed": T is the identity for a step
whose compression dropped nothing above the relative cut (it only removed
numerically null directions, so the step is exact, and without any chi_max
truncation J and its gradient are those of the physical circuit); otherwise
T is the orthogonal projector onto (sites <= l) x span{right Schmidt vectors
of the post-step state across the cut right of site l} -- the kept subspace
of the whole step -- held at its value in the recorded forward.

Adjoint (normalised frame; n = ||F phi|| of the recorded forward):
  mu = 0 after the last step; backwards through a step: mu <- F^dag mu / n;
  at measurement k then add A_k phi_k / p_k - phi_k;
  for rotation r, once mu is back before it:
      dJ/dtheta_r = 2 Re <mu | (-i sigma P'_r) | phi_{r-1}>,
  since dR/dtheta = (-i sigma P') R and R^dag commutes with P'.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from .mps import MPS
from .stn import PI0, Shot, site_ops, z_string


@dataclass
class Step:
    kind: str                       # "rot" or "meas"
    phi: np.ndarray                 # normalised pre-step frame vector, shape (2,)*n
    sigma: int                      # sign of P' = sigma * (phase-free Pauli string)
    ops: Dict[int, np.ndarray]      # site operators of the Pauli string
    l: int
    norm: float                     # ||F phi|| before renormalisation
    truncated: bool
    basis: Optional[np.ndarray] = None   # rows: right Schmidt basis across cut after l
    index: int = -1                 # rotation: position among the shot's rotations
    theta: float = 0.0
    s: int = 1                      # measurement: (-1)^m
    pivot: Optional[int] = None
    p: float = 1.0                  # measurement: probability of the recorded outcome


@dataclass
class Tape:
    n: int
    steps: List[Step] = field(default_factory=list)
    logp: float = 0.0
    n_rot: int = 0


def _dense(mps: MPS) -> np.ndarray:
    return mps.dense().reshape((2,) * mps.n)


def _right_basis(mps: MPS, l: int) -> np.ndarray:
    """Rows = right Schmidt basis vectors across the cut between l and l+1
    (sites l+1..n-1 of a state whose centre is at l, right-orthonormal)."""
    t = mps.A[l + 1]
    v = t.reshape(t.shape[0], -1)
    for j in range(l + 2, mps.n):
        u = mps.A[j]
        v = (v.reshape(-1, u.shape[0]) @ u.reshape(u.shape[0], -1)).reshape(t.shape[0], -1)
    return v


def apply_ops(vec: np.ndarray, ops: Dict[int, np.ndarray]) -> np.ndarray:
    """prod_j ops[j] acting on axis j of a (2,)*n array."""
    out = vec
    for j, o in ops.items():
        out = np.moveaxis(np.tensordot(o, out, axes=([1], [j])), 0, j)
    return out


def project(vec: np.ndarray, l: int, basis: np.ndarray) -> np.ndarray:
    """(I on sites <= l) x (projector onto the row space of basis)."""
    sh = vec.shape
    m = vec.reshape(2 ** (l + 1), -1)
    return ((m @ basis.conj().T) @ basis).reshape(sh)


def record(circ, shot: int, chi_max: int, eps_cut: float, forced=None) -> Tape:
    """Runs the oracle forward of one shot and records every non-Clifford
    step (pre-step state, operator, norm, frozen projector)."""
    st = Shot(circ.n, chi_max, eps_cut)
    tape = Tape(circ.n)
    mi = 0
    for op in circ.ops:
        kind = op["op"]
        if kind == "gates":
            for name, q0, q1 in op["gates"]:
                st.gate(name, [q0, q1])
        elif kind == "noise":
            st.pauli_noise(op["x"][shot], op["z"][shot])
        elif kind == "rotate":
            for ri, qs in enumerate(op["paulis"]):
                qs = [int(q) for q in qs]
                p = st.tab.image(z_string(circ.n, qs))
                phi = _dense(st.mps)
                phi = phi / np.linalg.norm(phi)
                th = float(op["theta"][shot, ri])
                st.rotate(qs, th)
                sup = p.support()
                l = int(sup[0])
                m = st.mps
                tape.steps.append(Step("rot", phi, p.sign(), site_ops(p), l, m.last_norm, m.last_truncated,
                                       _right_basis(m, l) if m.last_truncated else None,
                                       index=tape.n_rot, theta=th))
                tape.n_rot += 1
        elif kind == "measure":
            for mj, q in enumerate(op["qubits"]):
                p = st.tab.rz(int(q))
                phi = _dense(st.mps)
                phi = phi / np.linalg.norm(phi)
                xs = np.nonzero(p.x)[0]
                f = None if forced is None else forced[mi]
                mm = st.measure(int(q), float(op["u"][shot, mj]), f, bool(op["reset"]))
                l = int(p.support()[0])
                m = st.mps
                tape.steps.append(Step("meas", phi, p.sign(), site_ops(p), l, m.last_norm, m.last_truncated,
                                       _right_basis(m, l) if m.last_truncated else None,
                                       s=1 - 2 * mm, pivot=int(xs[0]) if len(xs) else None,
                                       p=st.res.prob[-1]))
                mi += 1
        else:
            raise ValueError(kind)
    tape.logp = st.res.logp
    return tape


def _measure_map(stp: Step, vec: np.ndarray, adjoint: bool) -> np.ndarray:
    c = stp.s * stp.sigma
    if stp.pivot is None:                     # (I + s sigma Z^z) / 2, Hermitian
        return 0.5 * (vec + c * apply_ops(vec, stp.ops))
    pk = {stp.pivot: PI0}
    if not adjoint:                           # Pi0_k (I + s sigma P')
        return apply_ops(vec + c * apply_ops(vec, stp.ops), pk)
    w = apply_ops(vec, pk)                    # (I + s sigma P') Pi0_k
    return w + c * apply_ops(w, stp.ops)


def frozen_logp(tape: Tape, thetas: Optional[Dict[int, float]] = None) -> float:
    """J of the frozen forward: the recorded steps with the given angles
    (rotation index -> angle; others as recorded) and projectors held fixed."""
    thetas = thetas or {}
    n = tape.n
    phi = np.zeros((2,) * n, complex)
    phi[(0,) * n] = 1.0
    J = 0.0
    for stp in tape.steps:
        if stp.kind == "rot":
            t = thetas.get(stp.index, stp.theta)
            phi = np.cos(t) * phi - 1j * stp.sigma * np.sin(t) * apply_ops(phi, stp.ops)
        else:
            a = 0.5 * (phi + stp.s * stp.sigma * apply_ops(phi, stp.ops))
            J += float(np.log(np.vdot(a, a).real / np.vdot(phi, phi).real))
            phi = _measure_map(stp, phi, adjoint=False)
        if stp.truncated:
            phi = project(phi, stp.l, stp.basis)
        phi = phi / np.linalg.norm(phi)
    return J


def adjoint_gradient(tape: Tape) -> np.ndarray:
    """dJ/dtheta for every rotation of the shot, in circuit order."""
    g = np.zeros(tape.n_rot)
    mu = np.zeros((2,) * tape.n, complex)
    for stp in reversed(tape.steps):
        if stp.truncated:
            mu = project(mu, stp.l, stp.basis)
        if stp.kind == "rot":
            t = stp.theta
            mu = (np.cos(t) * mu + 1j * stp.sigma * np.sin(t) * apply_ops(mu, stp.ops)) / stp.norm
            d = -1j * stp.sigma * apply_ops(stp.phi, stp.ops)
            g[stp.index] = 2.0 * float(np.vdot(mu, d).real)
        else:
            mu = _measure_map(stp, mu, adjoint=True) / stp.norm
            a = 0.5 * (stp.phi + stp.s * stp.sigma * apply_ops(stp.phi, stp.ops))
            mu = mu + a / stp.p - stp.phi
    return g


def fd_gradient(tape: Tape, h: float = 1e-5, indices=None) -> np.ndarray:
    """Central differences of frozen_logp (O(h^2))."""
    idx = range(tape.n_rot) if indices is None else indices
    g = np.zeros(tape.n_rot)
    theta0 = {s.index: s.theta for s in tape.steps if s.kind == "rot"}
    for i in idx:
        g[i] = (frozen_logp(tape, {i: theta0[i] + h}) - frozen_logp(tape, {i: theta0[i] - h})) / (2 * h)
    return g

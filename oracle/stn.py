"""One shot of the hybrid stabilizer-tensor-network simulation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Parity pins:
tests/test_oracle_stn.py (statevector agreement without truncation, the
closed form of Eq. 6, the Aaronson-Gottesman records at theta = 0, the
theta -> -theta symmetry, norms and probability sums).

State psi = C |MPS> (Sec. IV.A, Eq. 7), C stored as its inverse tableau.
  * Clifford gate or Pauli noise: C <- G C, the MPS is untouched (Sec. IV.A).
  * Crosstalk exp(-i theta Z_i Z_j [Z_k]) (Eq. 4, sign read as exp(-i theta P)):
    P' = C^dag P C = sigma * (Pauli string); the MPS becomes
    cos(theta) phi - i sin(theta) sigma P' phi (Sec. IV.A), then is
    compressed to chi_max (Sec. IV.B).
  * Z measurement of qubit a: P' = C^dag Z_a C = sigma * Q.  Outcome
    probabilities p(m) = <phi|(I + s P')/2|phi> / <phi|phi>, s = (-1)^m;
    m = 0 iff u < p(0).  The projection is applied to the MPS (Sec. IV.A):
      - Q diagonal (no X/Y site): phi <- (I + s sigma Z^z)/2 phi;
      - otherwise, with k the first X/Y site of Q: phi <- Pi0_k (I + s P') phi
        and C <- C V with V = D_k CQ0_k H_k, where Q0 is Q without site k,
        alpha = 1 (X at k) or i (Y at k), D_k = diag(1, s sigma alpha).
        V maps |0>_k (x) a to the normalised (I + sP') image, so psi is
        unchanged while the MPS stays |0...0> in a Clifford-only run (the
        reading of "applied to the tensor network" under which the MPS holds
        only the error part of the state, Sec. IV.A).
    Reset (ancillas): X_a when m = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .mps import MPS
from .tableau import InverseTableau, Pauli, site_op

PI0 = np.array([[1, 0], [0, 0]], dtype=complex)


@dataclass
class ShotResult:
    record: List[int] = field(default_factory=list)
    prob: List[float] = field(default_factory=list)        # p(recorded outcome)
    p0: List[float] = field(default_factory=list)          # p(0) of each measurement
    logp: float = 0.0
    trunc_err: float = 0.0
    max_bond: int = 1
    bond_trace: List[int] = field(default_factory=list)    # max bond after each rotation
    pivot_events: int = 0
    cut_sensitivity: float = 0.0                            # worst binding cut (see MPS)
    cut_sensitivity_sum: float = 0.0                        # summed over binding cuts (see MPS)
    flag_margin: float = float("inf")                       # closest chi decision to the eps cut (see MPS)
    tableau: Optional[InverseTableau] = None
    mps: Optional[MPS] = None


def z_string(n: int, qubits) -> Pauli:
    p = Pauli.identity(n)
    for q in qubits:
        if q >= 0:
            p.z[q] = True
    return p


def site_ops(p: Pauli) -> dict:
    """Per-site operators i^(xz) X^x Z^z of a Pauli string (phase excluded)."""
    return {int(j): site_op(int(p.x[j]), int(p.z[j])) for j in p.support()}


class Shot:
    """Mutable STN state of one shot."""

    def __init__(self, n: int, chi_max: int, eps_cut: float):
        self.n = n
        self.tab = InverseTableau(n)
        self.mps = MPS(n, chi_max, eps_cut)
        self.res = ShotResult()

    # ----------------------------------------------------------- Clifford
    def gate(self, name: str, qubits) -> None:
        self.tab.apply_gate(name, [q for q in qubits if q >= 0])

    def pauli_noise(self, x_row: np.ndarray, z_row: np.ndarray) -> None:
        for q in np.nonzero(x_row | z_row)[0]:
            name = {(1, 0): "X", (0, 1): "Z", (1, 1): "Y"}[(int(x_row[q]), int(z_row[q]))]
            self.tab.apply_gate(name, [int(q)])

    # ----------------------------------------------------------- rotation
    def rotate(self, qubits, theta: float) -> None:
        p = self.tab.image(z_string(self.n, qubits))
        sigma = p.sign()
        sup = p.support()
        ops = site_ops(p)
        l, r = int(sup[0]), int(sup[-1])
        self.mps.apply_two_term(l, r, np.cos(theta), {}, -1j * np.sin(theta) * sigma, ops)
        self.res.bond_trace.append(max(self.mps.bonds() or [1]))

    # -------------------------------------------------------- measurement
    def measure(self, q: int, u: Optional[float], forced: Optional[int],
                reset: bool) -> int:
        p = self.tab.rz(q)
        sigma = p.sign()
        ops = site_ops(p)
        ev = self.mps.expect(ops).real / self.mps.norm2()
        p0 = 0.5 * (1.0 + sigma * ev)
        p0 = min(1.0, max(0.0, p0))
        if forced is None:
            m = 0 if u < p0 else 1
        else:
            m = int(forced)
        pm = p0 if m == 0 else 1.0 - p0
        if pm <= 0.0:
            raise ZeroDivisionError(f"outcome {m} of qubit {q} has probability 0")
        s = 1 - 2 * m
        sup = p.support()
        l, r = int(sup[0]), int(sup[-1])
        xs = np.nonzero(p.x)[0]
        if len(xs) == 0:
            # diagonal: phi <- (I + s sigma Z^z)/2 phi
            self.mps.apply_two_term(l, r, 0.5, {}, 0.5 * s * sigma, ops)
        else:
            k = int(xs[0])
            alpha = 1j if p.z[k] else 1.0
            o1 = {k: PI0}
            o2 = dict(ops)
            o2[k] = PI0 @ ops[k]
            self.mps.apply_two_term(l, r, 1.0, o1, s * sigma, o2)
            # frame C <- C V, V = D_k CQ0 H_k: rows conjugated by D_k, then by
            # each controlled Pauli from k, then by H_k.
            dk = s * sigma * alpha
            dname = {1: "I", -1: "Z", 1j: "S", -1j: "SDG"}[complex(dk)]
            if dname != "I":
                self.tab.apply_right(dname, [k])
            for j in p.support():
                j = int(j)
                if j == k:
                    continue
                cname = {(1, 0): "CX", (0, 1): "CZ", (1, 1): "CY"}[(int(p.x[j]), int(p.z[j]))]
                self.tab.apply_right(cname, [k, j])
            self.tab.apply_right("H", [k])
            self.res.pivot_events += 1
        if reset and m == 1:
            self.tab.apply_gate("X", [q])
        self.res.record.append(m)
        self.res.prob.append(pm)
        self.res.p0.append(p0)
        self.res.logp += float(np.log(pm))
        return m


def run_shot(circ, shot: int, chi_max: int = 1 << 30, eps_cut: float = 0.0,
             forced=None, stop_after_ops: Optional[int] = None) -> ShotResult:
    """Simulate one shot of a workload Circuit.  forced: optional sequence of
    outcomes (replaces sampling from the measurement uniforms)."""
    st = Shot(circ.n, chi_max, eps_cut)
    mi = 0
    for oi, op in enumerate(circ.ops):
        if stop_after_ops is not None and oi >= stop_after_ops:
            break
        kind = op["op"]
        if kind == "gates":
            for name, q0, q1 in op["gates"]:
                st.gate(name, [q0, q1])
        elif kind == "noise":
            st.pauli_noise(op["x"][shot], op["z"][shot])
        elif kind == "rotate":
            th = op["theta"][shot]
            for ri, qs in enumerate(op["paulis"]):
                st.rotate([int(q) for q in qs], float(th[ri]))
        elif kind == "measure":
            for mj, q in enumerate(op["qubits"]):
                f = None if forced is None else forced[mi]
                st.measure(int(q), float(op["u"][shot, mj]), f, bool(op["reset"]))
                mi += 1
        else:
            raise ValueError(kind)
    st.res.trunc_err = 1.0 - st.mps.fidelity
    st.res.max_bond = max(st.mps.bonds() or [1])
    st.res.cut_sensitivity = st.mps.max_cut_sensitivity
    st.res.cut_sensitivity_sum = st.mps.sum_cut_sensitivity
    st.res.flag_margin = st.mps.min_flag_margin
    st.res.tableau = st.tab
    st.res.mps = st.mps
    return st.res

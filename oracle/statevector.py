"""Brute-force statevector simulation of the same circuits (n <= ~20).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  This is the physical
definition the STN method rewrites (Sec. IV.A): without truncation, the STN
oracle must reproduce its outcome probabilities, records and log-probability
to rounding.  Crosstalk exp(-i theta Z...Z) (Eq. 4, sign read as
exp(-i theta P)) is a diagonal phase; measurements project and renormalise;
outcome m = 0 iff u < p(0).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .tableau import GATES


class StateVector:
    def __init__(self, n: int):
        if n > 24:
            raise ValueError("statevector limited to 24 qubits")
        self.n = n
        self.psi = np.zeros((2,) * n, complex)
        self.psi[(0,) * n] = 1.0

    def gate(self, name: str, qubits) -> None:
        qubits = [q for q in qubits if q >= 0]
        u = GATES[name]
        k = len(qubits)
        u = u.reshape((2,) * (2 * k))
        psi = np.tensordot(u, self.psi, axes=(list(range(k, 2 * k)), qubits))
        self.psi = np.moveaxis(psi, list(range(k)), qubits)

    def rotate(self, qubits, theta: float) -> None:
        """exp(-i theta Z_q1 Z_q2 ...): eigenvalue (-1)^parity."""
        par = np.zeros((2,) * self.n, np.int64)
        for q in qubits:
            if q < 0:
                continue
            shape = [1] * self.n
            shape[q] = 2
            par = par + np.arange(2).reshape(shape)
        eig = 1 - 2 * (par % 2)
        self.psi = self.psi * np.exp(-1j * theta * eig)

    def prob0(self, q: int) -> float:
        w = np.abs(self.psi) ** 2
        tot = float(w.sum())
        return float(np.take(w, 0, axis=q).sum()) / tot

    def measure(self, q: int, u: Optional[float], forced: Optional[int], reset: bool):
        p0 = self.prob0(q)
        m = (0 if u < p0 else 1) if forced is None else int(forced)
        pm = p0 if m == 0 else 1.0 - p0
        if pm <= 0:
            raise ZeroDivisionError("zero-probability outcome")
        idx = [slice(None)] * self.n
        idx[q] = 1 - m
        self.psi[tuple(idx)] = 0.0
        self.psi /= np.linalg.norm(self.psi)
        if reset and m == 1:
            self.gate("X", [q])
        return m, pm, p0


def run_shot(circ, shot: int, forced=None):
    """Returns (record, p(recorded), p(0) list, log P, final state)."""
    sv = StateVector(circ.n)
    rec, probs, p0s = [], [], []
    mi = 0
    for op in circ.ops:
        kind = op["op"]
        if kind == "gates":
            for name, q0, q1 in op["gates"]:
                sv.gate(name, [q0, q1])
        elif kind == "noise":
            xr, zr = op["x"][shot], op["z"][shot]
            for q in np.nonzero(xr | zr)[0]:
                if xr[q]:
                    sv.gate("X", [int(q)])
                if zr[q]:
                    sv.gate("Z", [int(q)])
        elif kind == "rotate":
            for ri, qs in enumerate(op["paulis"]):
                sv.rotate([int(q) for q in qs], float(op["theta"][shot, ri]))
        elif kind == "measure":
            for mj, q in enumerate(op["qubits"]):
                f = None if forced is None else forced[mi]
                m, pm, p0 = sv.measure(int(q), float(op["u"][shot, mj]), f, bool(op["reset"]))
                rec.append(m)
                probs.append(pm)
                p0s.append(p0)
                mi += 1
    return rec, probs, p0s, float(np.sum(np.log(probs))), sv.psi.reshape(-1)

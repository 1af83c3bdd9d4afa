"""Aaronson-Gottesman stabilizer simulation (the paper's ref. for stabilizer
simulators, Sec. III), used to pin theta = 0 runs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written from the
published algorithm: a tableau of n destabilizers and n stabilizers with
x, z bits and a sign bit r per row, one scratch row, gate rules for H, CNOT
and Paulis, and the rowsum phase function g.  A measurement is random (p = 1/2)
when some stabilizer anticommutes with Z_a, else deterministic.  Outcome rule
as everywhere: m = 0 iff u < p(0).
"""
from __future__ import annotations

import numpy as np


def _g(x1, z1, x2, z2) -> int:
    """Exponent of i picked up when multiplying the single-site Paulis."""
    if x1 == 0 and z1 == 0:
        return 0
    if x1 == 1 and z1 == 1:
        return int(z2) - int(x2)
    if x1 == 1 and z1 == 0:
        return int(z2) * (2 * int(x2) - 1)
    return int(x2) * (1 - 2 * int(z2))


class CHP:
    def __init__(self, n: int):
        self.n = n
        self.x = np.zeros((2 * n + 1, n), np.uint8)
        self.z = np.zeros((2 * n + 1, n), np.uint8)
        self.r = np.zeros(2 * n + 1, np.uint8)
        for i in range(n):
            self.x[i, i] = 1          # destabilizer X_i
            self.z[n + i, i] = 1      # stabilizer Z_i

    def h(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.x[:, a], self.z[:, a] = self.z[:, a].copy(), self.x[:, a].copy()

    def cx(self, a, b):
        self.r ^= self.x[:, a] & self.z[:, b] & (self.x[:, b] ^ self.z[:, a] ^ 1)
        self.x[:, b] ^= self.x[:, a]
        self.z[:, a] ^= self.z[:, b]

    def pauli(self, a, px, pz):
        if px:
            self.r ^= self.z[:, a]
        if pz:
            self.r ^= self.x[:, a]

    def _rowsum(self, h, i):
        tot = 2 * int(self.r[h]) + 2 * int(self.r[i])
        for j in range(self.n):
            tot += _g(self.x[i, j], self.z[i, j], self.x[h, j], self.z[h, j])
        tot %= 4
        if tot not in (0, 2):
            raise AssertionError("rowsum produced an imaginary phase")
        self.r[h] = tot // 2
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def measure(self, a, u, forced=None):
        n = self.n
        ps = [p for p in range(n, 2 * n) if self.x[p, a]]
        if ps:
            p = ps[0]
            for i in range(2 * n):
                if i != p and self.x[i, a]:
                    self._rowsum(i, p)
            self.x[p - n], self.z[p - n], self.r[p - n] = self.x[p].copy(), self.z[p].copy(), self.r[p]
            self.x[p] = 0
            self.z[p] = 0
            self.z[p, a] = 1
            m = (0 if u < 0.5 else 1) if forced is None else int(forced)
            self.r[p] = m
            return m, 0.5
        s = 2 * n
        self.x[s] = 0
        self.z[s] = 0
        self.r[s] = 0
        for i in range(n):
            if self.x[i, a]:
                self._rowsum(s, i + n)
        m = int(self.r[s])
        if forced is not None and int(forced) != m:
            raise ZeroDivisionError("forced outcome has probability 0")
        return m, 1.0


def run_shot(circ, shot: int):
    """Records of a circuit with every crosstalk angle ignored (theta = 0)."""
    sim = CHP(circ.n)
    rec, p0s = [], []
    for op in circ.ops:
        kind = op["op"]
        if kind == "gates":
            for name, q0, q1 in op["gates"]:
                if name == "H":
                    sim.h(q0)
                elif name == "CX":
                    sim.cx(q0, q1)
                else:
                    raise ValueError(name)
        elif kind == "noise":
            xr, zr = op["x"][shot], op["z"][shot]
            for q in np.nonzero(xr | zr)[0]:
                sim.pauli(int(q), int(xr[q]), int(zr[q]))
        elif kind == "measure":
            for mj, q in enumerate(op["qubits"]):
                m, pr = sim.measure(int(q), float(op["u"][shot, mj]))
                rec.append(m)
                p0s.append(pr if pr == 0.5 else float(1 - m))
                if op["reset"] and m == 1:
                    sim.pauli(int(q), 1, 0)
    return rec, p0s

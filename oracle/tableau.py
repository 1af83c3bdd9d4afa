"""Pauli strings and the inverse Clifford tableau of an STN state.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Parity pins:
tests/test_oracle_tableau.py checks every gate rule and frame update against
dense unitaries, and the symplectic invariant.

The STN state is psi = C |MPS> (Sec. IV.A, Eq. 7).  A Clifford gate G acts as
C <- G C (Sec. IV.A), a Pauli P on psi becomes C^dag P C on the MPS (Sec.
IV.A, the commuted sum of Paulis), and a measured Pauli is commuted the same
way (Sec. IV.A, last paragraph).  All three only need the images of the
single-qubit generators, so the oracle stores the inverse tableau

    row X_j :  C^dag X_j C        row Z_j :  C^dag Z_j C       (j = 0..n-1)

each a Pauli string on the MPS qubits.  A Pauli string (x, z, e) means

    i^e * prod_j  i^(x_j z_j) X^(x_j) Z^(z_j)

so that x = z = 1 on a site is Y.  Rows are Hermitian, hence e is 0 or 2.
Every gate rule below is derived numerically from the gate's dense matrix
(conjugate a generator, read off the resulting Pauli), not typed in by hand.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

I2 = np.eye(2, dtype=complex)
X2 = np.array([[0, 1], [1, 0]], dtype=complex)
Z2 = np.array([[1, 0], [0, -1]], dtype=complex)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
H2 = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
S2 = np.diag([1, 1j]).astype(complex)


def site_op(x: int, z: int) -> np.ndarray:
    """i^(xz) X^x Z^z as a 2x2 matrix: I, Z, X or Y."""
    m = I2.copy()
    if x:
        m = m @ X2
    if z:
        m = m @ Z2
    return (1j ** (x * z)) * m


def controlled(u: np.ndarray) -> np.ndarray:
    """|0><0| (x) I + |1><1| (x) u, control first."""
    out = np.zeros((4, 4), complex)
    out[:2, :2] = I2
    out[2:, 2:] = u
    return out


GATES = {
    "I": I2, "X": X2, "Y": Y2, "Z": Z2, "H": H2, "S": S2, "SDG": S2.conj().T,
    "CX": controlled(X2), "CY": controlled(Y2), "CZ": controlled(Z2),
}


@dataclass
class Pauli:
    x: np.ndarray      # bool[n]
    z: np.ndarray      # bool[n]
    e: int             # phase exponent of i, mod 4

    @staticmethod
    def identity(n: int) -> "Pauli":
        return Pauli(np.zeros(n, bool), np.zeros(n, bool), 0)

    @staticmethod
    def single(n: int, q: int, x: int, z: int) -> "Pauli":
        p = Pauli.identity(n)
        p.x[q], p.z[q] = bool(x), bool(z)
        return p

    def copy(self) -> "Pauli":
        return Pauli(self.x.copy(), self.z.copy(), self.e % 4)

    @property
    def n(self) -> int:
        return len(self.x)

    def sign(self) -> int:
        """+1 / -1 for a Hermitian string."""
        if self.e % 2:
            raise ValueError("not Hermitian")
        return 1 if self.e % 4 == 0 else -1

    def support(self):
        return np.nonzero(self.x | self.z)[0]

    def dense(self) -> np.ndarray:
        """2^n x 2^n matrix, qubit 0 most significant (small n only)."""
        m = np.ones((1, 1), complex)
        for j in range(self.n):
            m = np.kron(m, site_op(int(self.x[j]), int(self.z[j])))
        return (1j ** self.e) * m


def mul(a: Pauli, b: Pauli) -> Pauli:
    """Product a*b with its phase.  Per site:
    (i^(x1 z1) X^x1 Z^z1)(i^(x2 z2) X^x2 Z^z2)
      = i^(x1 z1 + x2 z2) (-1)^(z1 x2) X^(x1+x2) Z^(z1+z2)
    and X^(x1+x2) Z^(z1+z2) = i^(-x3 z3) * [i^(x3 z3) X^x3 Z^z3]."""
    x1, z1, x2, z2 = (v.astype(np.int64) for v in (a.x, a.z, b.x, b.z))
    x3, z3 = x1 ^ x2, z1 ^ z2
    e = a.e + b.e + int(np.sum(x1 * z1 + x2 * z2 - x3 * z3 + 2 * z1 * x2))
    return Pauli(x3.astype(bool), z3.astype(bool), e % 4)


def commutes(a: Pauli, b: Pauli) -> bool:
    return int(np.sum(a.x & b.z) + np.sum(a.z & b.x)) % 2 == 0


@lru_cache(maxsize=None)
def _paulis_on(k: int):
    out = []
    for bits in itertools.product((0, 1), repeat=2 * k):
        xs, zs = bits[:k], bits[k:]
        m = np.ones((1, 1), complex)
        for j in range(k):
            m = np.kron(m, site_op(xs[j], zs[j]))
        out.append((xs, zs, m))
    return out


def decompose(m: np.ndarray):
    """Write a dense matrix that equals i^e times a Pauli string as (x, z, e)."""
    k = int(round(np.log2(m.shape[0])))
    for xs, zs, p in _paulis_on(k):
        c = np.trace(p.conj().T @ m) / m.shape[0]
        if abs(c) > 0.5:
            if not np.allclose(m, c * p, atol=1e-12):
                raise ValueError("matrix is not a single Pauli string")
            e = int(round(np.angle(c) / (np.pi / 2))) % 4
            if abs(c - 1j ** e) > 1e-9:
                raise ValueError("phase is not a power of i")
            return xs, zs, e
    raise ValueError("matrix is not a Pauli string")


@lru_cache(maxsize=None)
def conjugation_table(gate: str, dagger_left: bool):
    """For a 1- or 2-qubit gate G, the Pauli g' = G^dag g G (dagger_left) or
    G g G^dag for each local Pauli g, keyed by (xs, zs)."""
    g = GATES[gate]
    k = int(round(np.log2(g.shape[0])))
    table = {}
    for xs, zs, p in _paulis_on(k):
        m = g.conj().T @ p @ g if dagger_left else g @ p @ g.conj().T
        table[(xs, zs)] = decompose(m)
    return table


def conjugate(p: Pauli, gate: str, qubits) -> Pauli:
    """V^dag p V for a gate V on the given qubits (a column operation on an
    MPS-side Pauli string)."""
    qubits = list(qubits)
    xs = tuple(int(p.x[q]) for q in qubits)
    zs = tuple(int(p.z[q]) for q in qubits)
    nx, nz, de = conjugation_table(gate, True)[(xs, zs)]
    out = p.copy()
    for j, q in enumerate(qubits):
        out.x[q], out.z[q] = bool(nx[j]), bool(nz[j])
    out.e = (out.e + de) % 4
    return out


class InverseTableau:
    """Rows C^dag X_j C (index j) and C^dag Z_j C (index n + j)."""

    def __init__(self, n: int):
        self.n = n
        self.x = np.zeros((2 * n, n), bool)
        self.z = np.zeros((2 * n, n), bool)
        self.e = np.zeros(2 * n, np.int64)
        for j in range(n):                      # C = I
            self.x[j, j] = True
            self.z[n + j, j] = True

    def copy(self) -> "InverseTableau":
        t = InverseTableau.__new__(InverseTableau)
        t.n, t.x, t.z, t.e = self.n, self.x.copy(), self.z.copy(), self.e.copy()
        return t

    def row(self, i: int) -> Pauli:
        return Pauli(self.x[i].copy(), self.z[i].copy(), int(self.e[i]) % 4)

    def set_row(self, i: int, p: Pauli) -> None:
        self.x[i], self.z[i], self.e[i] = p.x, p.z, p.e % 4

    def rx(self, q: int) -> Pauli:
        return self.row(q)

    def rz(self, q: int) -> Pauli:
        return self.row(self.n + q)

    def image(self, p: Pauli) -> Pauli:
        """C^dag p C for a physical Pauli p: the product over its sites of
        i^(x z) r(X_q)^x r(Z_q)^z, in site order."""
        out = Pauli.identity(self.n)
        out.e = p.e
        for q in p.support():
            if p.x[q]:
                out = mul(out, self.rx(q))
            if p.z[q]:
                out = mul(out, self.rz(q))
            out.e = (out.e + int(p.x[q] and p.z[q])) % 4
        return out

    def apply_gate(self, gate: str, qubits) -> None:
        """Physical Clifford G on `qubits`: C <- G C, i.e. each generator row
        becomes C^dag (G^dag g G) C, a product of old rows (Sec. IV.A)."""
        qubits = list(qubits)
        table = conjugation_table(gate, True)
        old = self.copy()
        k = len(qubits)
        for j, q in enumerate(qubits):
            for which in ("x", "z"):
                xs = tuple(int(which == "x" and i == j) for i in range(k))
                zs = tuple(int(which == "z" and i == j) for i in range(k))
                nx, nz, de = table[(xs, zs)]
                img = Pauli.identity(self.n)
                for i2, q2 in enumerate(qubits):
                    img.x[q2], img.z[q2] = bool(nx[i2]), bool(nz[i2])
                img.e = de
                self.set_row(q if which == "x" else self.n + q, old.image(img))

    def apply_right(self, gate: str, qubits) -> None:
        """Frame change C <- C V for a Clifford V on MPS qubits: every row r
        becomes V^dag r V."""
        for i in range(2 * self.n):
            self.set_row(i, conjugate(self.row(i), gate, qubits))

    def check_symplectic(self) -> None:
        """Rows of X_i and Z_j anticommute iff i == j; all others commute."""
        n = self.n
        for a in range(2 * n):
            pa = self.row(a)
            if pa.e % 2:
                raise AssertionError(f"row {a} is not Hermitian")
            for b in range(a + 1, 2 * n):
                anti = (a < n <= b and b - n == a)
                if commutes(pa, self.row(b)) == anti:
                    raise AssertionError(f"rows {a},{b} violate the symplectic form")

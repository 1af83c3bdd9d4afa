"""Matrix-product state with two-term operator application and truncation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Parity pins:
tests/test_oracle_mps.py (dense-vector equality without truncation, the
Eckart-Young optimum of a single-bond cut, norms and canonical forms) and
tests/test_oracle_stn.py (statevector agreement of whole circuits).

The MPS of the STN state (Sec. IV.A, Eq. 7) holds one tensor A_j of shape
(left bond, 2, right bond) per qubit, in complex128.  It is kept in
mixed-canonical form around a centre site.

Every non-Clifford step the simulation needs has the form

    phi <- a * (O1_l (x) ... (x) O1_r) phi  +  b * (O2_l (x) ... (x) O2_r) phi

with single-site 2x2 operators on a contiguous span [l, r] (identity
outside).  The crosstalk rotation exp(-i theta P') = cos(theta) I
- i sin(theta) P' is this form with O1 = I and O2 the sites of P' (Sec. IV.A,
the Pauli decomposition of a non-Clifford gate; Eq. 4 for the channel), and
so is a measurement projector (I + s P')/2.  The sum is a bond-2 operator;
applying it doubles the bonds inside the span, after which they are cut back
by the standard two-sweep compression: an exact left-to-right QR sweep, then
a right-to-left SVD sweep that keeps the largest Schmidt values (Sec. IV.B,
Eq. 8: keep at most chi_max terms, largest first).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _apply_site(op: np.ndarray, t: np.ndarray) -> np.ndarray:
    """(op t)[a, s, b] = sum_u op[s, u] t[a, u, b]."""
    return np.matmul(op, t)


def _transfer(e: np.ndarray, bra: np.ndarray, ket: np.ndarray) -> np.ndarray:
    """E'[c, d] = sum_{a,b,s} conj(bra[a, s, c]) E[a, b] ket[b, s, d]."""
    out = 0
    for s in range(2):
        out = out + bra[:, s, :].conj().T @ e @ ket[:, s, :]
    return out


def svd(m: np.ndarray):
    """LAPACK gesdd, falling back to gesvd when it does not converge."""
    try:
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")


def keep_count(s: np.ndarray, chi_max: int, eps_cut: float) -> int:
    """Number of Schmidt values kept: at most chi_max, and only those whose
    squared weight exceeds eps_cut times the total (at least one)."""
    w = s.astype(np.float64) ** 2
    total = float(np.sum(w))
    if total == 0.0:
        return 1
    k = int(np.sum(w > eps_cut * total))
    return max(1, min(chi_max, k))


class MPS:
    def __init__(self, n: int, chi_max: int = 1 << 30, eps_cut: float = 0.0):
        self.n = n
        self.chi_max = chi_max
        self.eps_cut = eps_cut
        self.A = []
        for _ in range(n):
            t = np.zeros((1, 2, 1), complex)
            t[0, 0, 0] = 1.0                   # |0...0>
            self.A.append(t)
        self.center = 0
        self.fidelity = 1.0                    # prod over cuts of (1 - w)
        self.discarded = []                    # per-cut discarded weight w
        # bookkeeping of the last apply_two_term, read by the gradient oracle:
        # whether chi_max dropped a value above the relative cut at some cut,
        # and the norm of the compressed state before renormalisation
        self.last_truncated = False
        self.last_norm = 1.0
        # conditioning of the cuts where chi_max binds: s_k^2 / (s_k^2 - s_{k+1}^2)
        # for the last kept value k (inf for an exact tie).  Eq. 8 keeps the
        # largest values but leaves ties at the cut open; a large value means the
        # kept subspace is ill-conditioned.
        self.max_cut_sensitivity = 0.0
        # the same summed over every binding cut of the run: to first order each
        # binding projector moves by rounding x its sensitivity, and the moves
        # of successive cuts add at worst linearly
        self.sum_cut_sensitivity = 0.0
        # margin of the chi decision at the relative cut: where more than
        # chi_max values exist, chi_max drops weight above the cut iff
        # s_chi^2 > eps sum s^2 (0-based index chi_max); the margin is
        # max(r, 1/r) with r the ratio of the two sides, its smallest value
        # over the run is kept.  A value near 1 means the decision (and with it
        # whether a step counts as truncated) is set by rounding: values near
        # eps sum s^2 are at the noise floor of any Gram-based eigen-solve.
        self.min_flag_margin = float("inf")

    # ------------------------------------------------------------------ basics
    def bonds(self):
        return [self.A[j].shape[2] for j in range(self.n - 1)]

    def copy(self) -> "MPS":
        m = MPS.__new__(MPS)
        m.__dict__.update(self.__dict__)
        m.A = [t.copy() for t in self.A]
        m.discarded = list(self.discarded)
        return m

    def dense(self) -> np.ndarray:
        """Full state vector, qubit 0 most significant (small n only)."""
        v = np.ones((1, 1), complex)
        for t in self.A:
            v = (v @ t.reshape(t.shape[0], -1)).reshape(-1, t.shape[2])
        return v.reshape(-1)

    def overlap(self, other: "MPS") -> complex:
        """<self|other> by plain transfer-matrix contraction."""
        e = np.ones((1, 1), complex)
        for a, b in zip(self.A, other.A):
            e = _transfer(e, a, b)
        return complex(e[0, 0])

    def expect(self, ops: dict) -> complex:
        """<phi| prod_j ops[j] |phi> over all sites (identity where absent),
        by plain transfer-matrix contraction: no canonical form assumed."""
        e = np.ones((1, 1), complex)
        for j, t in enumerate(self.A):
            ot = _apply_site(ops[j], t) if j in ops else t
            e = _transfer(e, t, ot)
        return complex(e[0, 0])

    def norm2(self) -> float:
        return float(self.expect({}).real)

    # ------------------------------------------------------- canonical moves
    def _qr_right(self, j: int) -> None:
        """A_j = Q R with Q left-orthonormal; R moves into A_{j+1}."""
        t = self.A[j]
        dl, _, dr = t.shape
        q, r = np.linalg.qr(t.reshape(dl * 2, dr))
        self.A[j] = q.reshape(dl, 2, q.shape[1])
        nxt = self.A[j + 1]
        self.A[j + 1] = (r @ nxt.reshape(nxt.shape[0], -1)).reshape(r.shape[0], 2, nxt.shape[2])

    def _qr_left(self, j: int) -> None:
        """A_j = L Q with Q right-orthonormal; L moves into A_{j-1}."""
        t = self.A[j]
        dl, _, dr = t.shape
        q, r = np.linalg.qr(t.reshape(dl, 2 * dr).conj().T)
        self.A[j] = q.conj().T.reshape(q.shape[1], 2, dr)
        prv = self.A[j - 1]
        self.A[j - 1] = (prv.reshape(-1, prv.shape[2]) @ r.conj().T).reshape(prv.shape[0], 2, -1)

    def move_center(self, j: int) -> None:
        while self.center < j:
            self._qr_right(self.center)
            self.center += 1
        while self.center > j:
            self._qr_left(self.center)
            self.center -= 1

    def normalize(self) -> float:
        """Scale the centre tensor to unit norm (valid in canonical form)."""
        t = self.A[self.center]
        nrm = float(np.linalg.norm(t))
        if nrm == 0.0:
            raise ZeroDivisionError("state has zero norm")
        self.A[self.center] = t / nrm
        return nrm

    # --------------------------------------------------------- the MPS step
    def apply_two_term(self, l: int, r: int, a: complex, o1: dict, b: complex,
                       o2: dict) -> None:
        """phi <- a * prod O1 phi + b * prod O2 phi on sites [l, r], then
        compress back (QR sweep left to right, SVD truncation right to left)
        and renormalise.  o1/o2 map site -> 2x2 matrix (identity if absent)."""
        eye = np.eye(2, dtype=complex)
        self.move_center(l)
        self.last_truncated = False
        if l == r:
            t = self.A[l]
            self.A[l] = a * _apply_site(o1.get(l, eye), t) + b * _apply_site(o2.get(l, eye), t)
            self.last_norm = self.normalize()
            return
        # bond-2 operator blocks over the span
        B = {}
        t = self.A[l]
        B[l] = np.concatenate([a * _apply_site(o1.get(l, eye), t),
                               b * _apply_site(o2.get(l, eye), t)], axis=2)
        for j in range(l + 1, r):
            t = self.A[j]
            dl, _, dr = t.shape
            blk = np.zeros((2 * dl, 2, 2 * dr), complex)
            blk[:dl, :, :dr] = _apply_site(o1.get(j, eye), t)
            blk[dl:, :, dr:] = _apply_site(o2.get(j, eye), t)
            B[j] = blk
        t = self.A[r]
        B[r] = np.concatenate([_apply_site(o1.get(r, eye), t),
                               _apply_site(o2.get(r, eye), t)], axis=0)
        for j in range(l, r + 1):
            self.A[j] = B[j]
        # left-to-right QR sweep: sites l..r-1 left-orthonormal, centre at r
        for j in range(l, r):
            self._qr_right(j)
        # right-to-left SVD sweep with truncation: centre back at l
        for j in range(r, l, -1):
            t = self.A[j]
            dl, _, dr = t.shape
            u, s, vh = svd(t.reshape(dl, 2 * dr))
            k = keep_count(s, self.chi_max, self.eps_cut)
            tot = float(np.sum(s.astype(np.float64) ** 2))
            if len(s) > self.chi_max and self.eps_cut > 0 and tot > 0:
                r = float(s[self.chi_max]) ** 2 / (self.eps_cut * tot)
                self.min_flag_margin = min(self.min_flag_margin, max(r, 1.0 / r) if r > 0 else float("inf"))
            if k < len(s) and s[k] ** 2 > self.eps_cut * tot:
                self.last_truncated = True
                gap = float(s[k - 1] ** 2 - s[k] ** 2)
                sens = float(s[k - 1] ** 2) / gap if gap > 0 else float("inf")
                self.max_cut_sensitivity = max(self.max_cut_sensitivity, sens)
                self.sum_cut_sensitivity += sens
            w = float(np.sum(s[k:].astype(np.float64) ** 2)) / tot if tot > 0 else 0.0
            self.discarded.append(w)
            self.fidelity *= (1.0 - w)
            self.A[j] = vh[:k].reshape(k, 2, dr)
            prv = self.A[j - 1]
            self.A[j - 1] = (prv.reshape(-1, prv.shape[2]) @ (u[:, :k] * s[:k])).reshape(prv.shape[0], 2, k)
        self.center = l
        self.last_norm = self.normalize()

    def schmidt_values(self, bond: int) -> np.ndarray:
        """Schmidt values across the cut between sites bond and bond+1."""
        self.move_center(bond)
        t = self.A[bond]
        dl, _, dr = t.shape
        return np.linalg.svd(t.reshape(dl * 2, dr), compute_uv=False)

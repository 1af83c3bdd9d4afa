"""Pins of the oracle tableau against dense unitaries (no GPU).

Each inverse-tableau row must equal C^dag X_j C / C^dag Z_j C for the
explicit unitary C, after physical gates (C <- G C) and frame changes
(C <- C V).  This fixes the rowsum phases, every gate rule and the
conjugation tables by brute force, independent of how the oracle derives
them.
"""
import numpy as np
import pytest

from oracle import tableau as T


def _embed(gate, qubits, n):
    """Dense 2^n matrix of a 1/2-qubit gate on `qubits` (qubit 0 most significant)."""
    g = T.GATES[gate]
    k = len(qubits)
    full = np.zeros((2 ** n, 2 ** n), complex)
    for col in range(2 ** n):
        bits = [(col >> (n - 1 - q)) & 1 for q in range(n)]
        sub = 0
        for q in qubits:
            sub = 2 * sub + bits[q]
        for out_sub in range(2 ** k):
            amp = g[out_sub, sub]
            if amp == 0:
                continue
            nb = list(bits)
            for i, q in enumerate(qubits):
                nb[q] = (out_sub >> (k - 1 - i)) & 1
            row = 0
            for b in nb:
                row = 2 * row + b
            full[row, col] += amp
    return full


def _gen(n, q, which):
    return T.Pauli.single(n, q, which == "x", which == "z").dense()


def _check_rows(tab, U, n):
    for q in range(n):
        for which, idx in (("x", q), ("z", n + q)):
            want = U.conj().T @ _gen(n, q, which) @ U
            got = tab.row(idx).dense()
            assert np.allclose(got, want, atol=1e-12), (q, which)


@pytest.mark.parametrize("seed", range(12))
def test_rows_match_dense_unitary(seed):
    rng = np.random.default_rng(seed)
    n = 4
    tab = T.InverseTableau(n)
    U = np.eye(2 ** n, dtype=complex)
    one = ["H", "S", "SDG", "X", "Y", "Z"]
    two = ["CX", "CY", "CZ"]
    for step in range(40):
        right = rng.random() < 0.4
        if rng.random() < 0.5:
            g, qs = one[rng.integers(len(one))], [int(rng.integers(n))]
        else:
            g = two[rng.integers(len(two))]
            qs = [int(v) for v in rng.choice(n, 2, replace=False)]
        G = _embed(g, qs, n)
        if right:
            tab.apply_right(g, qs)
            U = U @ G
        else:
            tab.apply_gate(g, qs)
            U = G @ U
        _check_rows(tab, U, n)
        tab.check_symplectic()


def test_product_phase_by_brute_force():
    rng = np.random.default_rng(3)
    n = 3
    for _ in range(200):
        a = T.Pauli(rng.random(n) < 0.5, rng.random(n) < 0.5, int(rng.integers(4)))
        b = T.Pauli(rng.random(n) < 0.5, rng.random(n) < 0.5, int(rng.integers(4)))
        assert np.allclose(T.mul(a, b).dense(), a.dense() @ b.dense(), atol=1e-12)
        assert T.commutes(a, b) == np.allclose(a.dense() @ b.dense(), b.dense() @ a.dense())


def test_image_of_physical_pauli():
    rng = np.random.default_rng(5)
    n = 3
    tab = T.InverseTableau(n)
    U = np.eye(2 ** n, dtype=complex)
    for _ in range(25):
        g = ["H", "S", "CX", "CZ"][rng.integers(4)]
        qs = [int(rng.integers(n))] if g in ("H", "S") else [int(v) for v in rng.choice(n, 2, replace=False)]
        tab.apply_gate(g, qs)
        U = _embed(g, qs, n) @ U
    for _ in range(50):
        p = T.Pauli(rng.random(n) < 0.5, rng.random(n) < 0.5, 0)
        assert np.allclose(tab.image(p).dense(), U.conj().T @ p.dense() @ U, atol=1e-12)


def test_symplectic_catches_a_broken_row():
    tab = T.InverseTableau(3)
    tab.apply_gate("H", [0])
    tab.apply_gate("CX", [0, 1])
    tab.check_symplectic()
    tab.z[3 + 1, 2] ^= True          # plant a wrong bit
    with pytest.raises(AssertionError):
        tab.check_symplectic()

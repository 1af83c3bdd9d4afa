"""Pins of the oracle MPS (no GPU): dense equality without truncation, the
Eckart-Young optimum of a single cut (Eq. 8), canonical moves and norms."""
import numpy as np
import pytest

from oracle import mps as M
from oracle.tableau import site_op


def random_mps(n, chi, rng):
    m = M.MPS(n, chi_max=1 << 20, eps_cut=0.0)
    dims = [1] + [min(chi, 2 ** min(j, n - j)) for j in range(1, n)] + [1]
    for j in range(n):
        t = rng.normal(size=(dims[j], 2, dims[j + 1])) + 1j * rng.normal(size=(dims[j], 2, dims[j + 1]))
        m.A[j] = t
    m.center = 0
    m.move_center(n - 1)
    m.move_center(0)
    m.normalize()
    return m


def dense_op(n, ops):
    out = np.ones((1, 1), complex)
    for j in range(n):
        out = np.kron(out, ops.get(j, np.eye(2)))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_two_term_matches_dense_without_truncation(seed):
    rng = np.random.default_rng(seed)
    n = 7
    m = random_mps(n, 4, rng)
    v = m.dense()
    l, r = sorted(rng.choice(n, 2, replace=False))
    o2 = {j: site_op(int(rng.integers(2)), int(rng.integers(2))) for j in range(l, r + 1)}
    th = 0.3
    a, b = np.cos(th), -1j * np.sin(th)
    m.eps_cut = 1e-28
    m.apply_two_term(int(l), int(r), a, {}, b, o2)
    want = a * v + b * dense_op(n, o2) @ v
    want /= np.linalg.norm(want)
    got = m.dense()
    assert abs(abs(np.vdot(got, want)) - 1) < 1e-12
    assert abs(np.linalg.norm(got) - 1) < 1e-12
    assert 1 - m.fidelity < 1e-15


def test_center_moves_preserve_state():
    rng = np.random.default_rng(1)
    m = random_mps(8, 6, rng)
    v = m.dense()
    for c in (5, 2, 7, 0, 4):
        m.move_center(c)
        assert np.allclose(m.dense(), v, atol=1e-12)
        for j in range(c):          # left-orthonormal
            t = m.A[j].reshape(-1, m.A[j].shape[2])
            assert np.allclose(t.conj().T @ t, np.eye(t.shape[1]), atol=1e-12)
        for j in range(c + 1, 8):   # right-orthonormal
            t = m.A[j].reshape(m.A[j].shape[0], -1)
            assert np.allclose(t @ t.conj().T, np.eye(t.shape[0]), atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_single_cut_truncation_is_eckart_young(k):
    """A two-site operator doubles one bond; cutting it back to k must give the
    best rank-k approximation of the dense state across that cut (Eq. 8)."""
    rng = np.random.default_rng(k)
    n = 6
    m = random_mps(n, 4, rng)
    v = m.dense()
    o2 = {2: site_op(1, 0), 3: site_op(1, 1)}
    a, b = 0.8, 0.6j
    w = a * v + b * dense_op(n, o2) @ v
    mat = w.reshape(2 ** 3, 2 ** 3)
    u, s, vh = np.linalg.svd(mat)
    best = (u[:, :k] * s[:k]) @ vh[:k]
    best = best.reshape(-1) / np.linalg.norm(best)
    discarded = np.sum(s[k:] ** 2) / np.sum(s ** 2)
    m.chi_max = k
    m.eps_cut = 1e-28
    m.apply_two_term(2, 3, a, {}, b, o2)
    got = m.dense()
    assert abs(abs(np.vdot(got, best)) - 1) < 1e-10
    assert abs((1 - m.fidelity) - discarded) < 1e-12


def test_keep_rule():
    s = np.array([1.0, 1e-3, 1e-8, 1e-9])
    # squared weights 1, 1e-6, 1e-16, 1e-18 (total ~1)
    assert M.keep_count(s, 10, 1e-14) == 2
    assert M.keep_count(s, 10, 1e-17) == 3
    assert M.keep_count(s, 1, 1e-17) == 1
    assert M.keep_count(np.zeros(3), 4, 1e-14) == 1


def test_expect_and_norm():
    rng = np.random.default_rng(7)
    m = random_mps(6, 4, rng)
    v = m.dense()
    ops = {1: site_op(1, 0), 4: site_op(1, 1)}
    assert abs(m.expect(ops) - np.vdot(v, dense_op(6, ops) @ v)) < 1e-12
    assert abs(m.norm2() - 1) < 1e-12

"""Crosstalk models of the workload generator beside the coherent one (CPU):
the Pauli-twirled approximation (Eq. 6) and random-sign angles (Eq. 9)."""
import numpy as np

from paper_2605_29514_amd import workload as W


def test_pta_flip_statistics():
    """Each coupling fires Z..Z with probability sin^2(theta) (Eq. 6), so a
    qubit's Z flip in a layer is the parity of its couplings' firings:
    P(flip) = (1 - prod_c (1 - 2 sin^2 theta_c)) / 2."""
    S, th = 20000, 0.3
    circ = W.memory_circuit(3, 1, S, seed=7, theta_nn=th, nnn=True, p=0.0, crosstalk="pta",
                            final_readout=False)
    assert circ.count("rotate") == 0
    lay = W.rotated_layout(3)
    couplings = W.nn_couplings(lay) + W.nnn_couplings(lay)
    angle = [th] * len(W.nn_couplings(lay)) + [th / 2] * len(W.nnn_couplings(lay))
    expect = np.zeros(circ.n)
    prod = np.ones(circ.n)
    for c, a in zip(couplings, angle):
        for q in c:
            prod[q] *= 1 - 2 * np.sin(a) ** 2
    expect = (1 - prod) / 2
    noise = [o for o in circ.ops if o["op"] == "noise"]
    assert len(noise) == 4                      # one per CNOT layer (p = 0: no other noise)
    for o in noise:
        assert not o["x"].any()
        freq = o["z"].mean(axis=0)
        sigma = np.sqrt(expect * (1 - expect) / S) + 1e-12
        assert np.all(np.abs(freq - expect) <= 5 * sigma + 1e-9), np.max(np.abs(freq - expect) / sigma)


def test_random_sign_angles():
    """theta_i in {theta, -theta} with probability 1/2 each (Eq. 9), drawn
    per rotation instance and shot; magnitudes unchanged."""
    S = 4000
    a = W.memory_circuit(3, 1, S, seed=9, theta_nn=0.05, nnn=True, random_sign=True)
    b = W.memory_circuit(3, 1, S, seed=9, theta_nn=0.05, nnn=True, random_sign=False)
    ra = [o["theta"] for o in a.ops if o["op"] == "rotate"]
    rb = [o["theta"] for o in b.ops if o["op"] == "rotate"]
    assert len(ra) == len(rb) == 4
    for x, y in zip(ra, rb):
        assert np.array_equal(np.abs(x), y)
        neg = (x < 0).mean()
        assert abs(neg - 0.5) < 5 * np.sqrt(0.25 / x.size)
    assert not np.array_equal(ra[0], ra[1])     # fresh signs in every layer

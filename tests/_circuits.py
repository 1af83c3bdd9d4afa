"""Small random circuits shared by the oracle and GPU tests."""
import numpy as np

from paper_2605_29514_amd import workload as W


def random_circuit(n, n_layers, n_shots, seed):
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(n_layers):
        gates = []
        for _ in range(3):
            g = ["H", "S", "CX", "CZ"][rng.integers(4)]
            if g in ("H", "S"):
                gates.append((g, int(rng.integers(n)), -1))
            else:
                a, b = rng.choice(n, 2, replace=False)
                gates.append((g, int(a), int(b)))
        ops.append({"op": "gates", "gates": gates})
        x = rng.random((n_shots, n)) < 0.1
        z = rng.random((n_shots, n)) < 0.1
        ops.append({"op": "noise", "x": x, "z": z})
        R = 3
        paulis = np.full((R, 3), -1, np.int32)
        for r in range(R):
            k = int(rng.integers(2, 4))
            paulis[r, :k] = rng.choice(n, k, replace=False)
        ops.append({"op": "rotate", "paulis": paulis,
                    "theta": rng.uniform(-0.6, 0.6, (n_shots, R)), "param": np.arange(R)})
        qs = rng.choice(n, 2, replace=False).astype(np.int32)
        ops.append({"op": "measure", "qubits": qs, "reset": bool(rng.random() < 0.5),
                    "u": rng.random((n_shots, 2))})
    return W.Circuit(n, n_shots, ops)


def entangling_circuit(n, layers, n_shots, seed, meas_every=2, phase_gates=True):
    """Denser entanglers (3 H, 3 CNOT and an S per layer, four 2-3 body Z
    rotations) and two measurements every other layer, so that small
    chi_max truncates often and the rotations move the probabilities."""
    rng = np.random.default_rng(seed)
    ops = []
    for L in range(layers):
        gates = [("H", int(q), -1) for q in rng.choice(n, 3, replace=False)]
        for _ in range(3):
            a, b = rng.choice(n, 2, replace=False)
            gates.append(("CX", int(a), int(b)))
        sq = int(rng.integers(n))
        if phase_gates:                       # S is complex: breaks the theta -> -theta symmetry
            gates.append(("S", sq, -1))
        ops.append({"op": "gates", "gates": gates})
        R = 4
        paulis = np.full((R, 3), -1, np.int32)
        for r in range(R):
            k = int(rng.integers(2, 4))
            paulis[r, :k] = rng.choice(n, k, replace=False)
        ops.append({"op": "rotate", "paulis": paulis, "theta": rng.uniform(-0.8, 0.8, (n_shots, R)),
                    "param": np.arange(R)})
        if L % meas_every == meas_every - 1:
            qs = rng.choice(n, 2, replace=False).astype(np.int32)
            ops.append({"op": "measure", "qubits": qs, "reset": True, "u": rng.random((n_shots, 2))})
    ops.append({"op": "measure", "qubits": np.arange(3, dtype=np.int32), "reset": False,
                "u": rng.random((n_shots, 3))})
    return W.Circuit(n, n_shots, ops)

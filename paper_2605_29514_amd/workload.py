"""Seeded synthetic workloads: rotated-surface-code memory experiments.

This module only builds inputs.  It lays out the rotated surface code
(Fig. 1a), emits the syndrome-extraction circuit (Fig. 1b/1c, repeated for
the memory experiment of Sec. II), places the crosstalk couplings (Sec. III.B,
Eq. 4) and draws every random number the simulation consumes (depolarising
locations of Eqs. 2-3 with the Table I ratios, crosstalk angles, measurement
uniforms).  It contains none of the simulation arithmetic: no tableau, no
state, no probability.  Both the HIP path and the CPU oracle read the same
arrays produced here.

Conventions (each a reading of a point the paper leaves open):
  * qubit coordinates (y, x): data at (2r+1, 2c+1), faces at (2r, 2c);
    a face is X-type when r+c is even; interior faces are kept, plus X faces
    on the top/bottom edges and Z faces on the left/right edges (d^2-1
    ancillas);
  * qubit index = row-major order of (y, x) over data and ancillas together;
    the MPS site of a qubit is its index;
  * CNOT order: X ancillas NW, NE, SW, SE; Z ancillas NW, SW, NE, SE;
  * crosstalk after each of the four CNOT layers on every coupling, order:
    nearest-neighbour (data-ancilla diagonal) pairs sorted by (min, max)
    index, then next-nearest (same-kind pairs two lattice units apart), then
    ancilla-centred diagonal triples;
  * depolarising noise (when p > 0): after each H (p1 = 0.1p, 3 Paulis),
    after each CNOT (p2 = p, 15 Pauli pairs), X after reset (pR = 2p), X
    before each measurement (pM = 5p); a location fires when u1 < p and its
    Pauli is floor(u2 * K) in lexicographic order over {X, Y, Z} (pairs:
    first qubit major, identity-identity skipped);
  * measurement outcome m = 0 iff u < p(0), with u a 53-bit uniform in [0, 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Pauli codes used in noise arrays: bit 0 = X component, bit 1 = Z component.
PAULI_I, PAULI_X, PAULI_Z, PAULI_Y = 0, 1, 2, 3
_ONE_Q = [PAULI_X, PAULI_Y, PAULI_Z]          # lexicographic X < Y < Z
_TWO_Q = [(a, b) for a in (0, 1, 3, 2) for b in (0, 1, 3, 2) if (a, b) != (0, 0)]
# (0,1,3,2) = I, X, Y, Z in code space so that the 15 pairs run I X, I Y, I Z, X I, ...

NW, NE, SW, SE = (-1, -1), (-1, +1), (+1, -1), (+1, +1)
X_ORDER = (NW, NE, SW, SE)
Z_ORDER = (NW, SW, NE, SE)


@dataclass
class Layout:
    d: int
    coords: List[tuple]            # (y, x) per qubit index
    kind: List[str]                # 'D', 'X' or 'Z' per qubit index
    data: List[int]
    x_anc: List[int]
    z_anc: List[int]
    index: dict                    # (y, x) -> qubit index

    @property
    def n(self) -> int:
        return len(self.coords)

    @property
    def ancillas(self) -> List[int]:
        return sorted(self.x_anc + self.z_anc)


def rotated_layout(d: int) -> Layout:
    """Rotated surface code of distance d (Fig. 1a): 2d^2-1 qubits."""
    if d < 2:
        raise ValueError("distance must be >= 2")
    pts = []
    for r in range(d):
        for c in range(d):
            pts.append((2 * r + 1, 2 * c + 1, 'D'))
    for r in range(d + 1):
        for c in range(d + 1):
            typ = 'X' if (r + c) % 2 == 0 else 'Z'
            interior = 1 <= r <= d - 1 and 1 <= c <= d - 1
            top_bottom = (r == 0 or r == d) and 1 <= c <= d - 1 and typ == 'X'
            left_right = (c == 0 or c == d) and 1 <= r <= d - 1 and typ == 'Z'
            if interior or top_bottom or left_right:
                pts.append((2 * r, 2 * c, typ))
    pts.sort(key=lambda p: (p[0], p[1]))
    coords = [(p[0], p[1]) for p in pts]
    kind = [p[2] for p in pts]
    index = {c: i for i, c in enumerate(coords)}
    data = [i for i, k in enumerate(kind) if k == 'D']
    xa = [i for i, k in enumerate(kind) if k == 'X']
    za = [i for i, k in enumerate(kind) if k == 'Z']
    return Layout(d, coords, kind, data, xa, za, index)


def cnot_layers(lay: Layout) -> List[List[tuple]]:
    """Four CNOT layers as (control, target) pairs (Fig. 1b/1c)."""
    layers = []
    for t in range(4):
        layer = []
        for a in lay.x_anc:                      # X check: ancilla controls data
            y, x = lay.coords[a]
            dy, dx = X_ORDER[t]
            q = lay.index.get((y + dy, x + dx))
            if q is not None:
                layer.append((a, q))
        for a in lay.z_anc:                      # Z check: data controls ancilla
            y, x = lay.coords[a]
            dy, dx = Z_ORDER[t]
            q = lay.index.get((y + dy, x + dx))
            if q is not None:
                layer.append((q, a))
        layers.append(layer)
    return layers


def nn_couplings(lay: Layout) -> List[tuple]:
    """Nearest-neighbour data-ancilla pairs (diagonal lattice edges)."""
    out = set()
    for a in lay.x_anc + lay.z_anc:
        y, x = lay.coords[a]
        for dy, dx in (NW, NE, SW, SE):
            q = lay.index.get((y + dy, x + dx))
            if q is not None:
                out.add((min(a, q), max(a, q)))
    return sorted(out)


def nnn_couplings(lay: Layout) -> List[tuple]:
    """Next-nearest pairs: same-kind qubits (data-data or ancilla-ancilla)
    two lattice units apart horizontally or vertically."""
    out = set()
    for i, (y, x) in enumerate(lay.coords):
        for dy, dx in ((0, 2), (2, 0)):
            j = lay.index.get((y + dy, x + dx))
            if j is not None and (lay.kind[i] == 'D') == (lay.kind[j] == 'D'):
                out.add((min(i, j), max(i, j)))
    return sorted(out)


def ancilla_triples(lay: Layout) -> List[tuple]:
    """Ancilla-centred collinear triples {NW, a, SE} and {NE, a, SW} for each
    ancilla with all four data neighbours."""
    out = []
    for a in sorted(lay.x_anc + lay.z_anc):
        y, x = lay.coords[a]
        nb = {dd: lay.index.get((y + dd[0], x + dd[1])) for dd in (NW, NE, SW, SE)}
        if any(v is None for v in nb.values()):
            continue
        out.append(tuple(sorted((nb[NW], a, nb[SE]))))
        out.append(tuple(sorted((nb[NE], a, nb[SW]))))
    return out


# --------------------------------------------------------------------------
# Circuit IR.  Ops are dicts; every per-shot array has the shot as axis 0.
#   {"op": "gates",   "gates": [("H", q, -1) | ("CX", c, t)]}
#   {"op": "noise",   "x": bool[S, n], "z": bool[S, n]}      Pauli flips
#   {"op": "rotate",  "paulis": int32[R, 3] (-1 padded), "theta": f64[S, R],
#                     "param": int32[R] (index into the angle parameter
#                     vector, for gradients)}
#   {"op": "measure", "qubits": int32[M], "reset": bool, "u": f64[S, M]}
# --------------------------------------------------------------------------


@dataclass
class Circuit:
    n: int
    n_shots: int
    ops: list
    layout: Optional[Layout] = None
    n_params: int = 0
    meta: dict = field(default_factory=dict)

    def count(self, op: str) -> int:
        return sum(1 for o in self.ops if o["op"] == op)

    @property
    def n_rotations(self) -> int:
        return sum(len(o["paulis"]) for o in self.ops if o["op"] == "rotate")

    @property
    def n_measurements(self) -> int:
        return sum(len(o["qubits"]) for o in self.ops if o["op"] == "measure")

    def shot_slice(self, s0: int, s1: int) -> "Circuit":
        """Same circuit restricted to shots [s0, s1)."""
        return self.shot_select(np.arange(s0, s1))

    def shot_select(self, idx) -> "Circuit":
        """Same circuit with the per-shot inputs of shots idx (in that order,
        repeats allowed)."""
        idx = np.asarray(idx, dtype=np.int64)
        ops = []
        for o in self.ops:
            o2 = dict(o)
            for key in ("x", "z", "theta", "u"):
                if key in o2:
                    o2[key] = o2[key][idx]
            ops.append(o2)
        return Circuit(self.n, len(idx), ops, self.layout, self.n_params, dict(self.meta))


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed, stream]))


def _uniform53(g: np.random.Generator, shape) -> np.ndarray:
    """53-bit uniforms in [0, 1): k * 2^-53 with k uniform on [0, 2^53)."""
    k = g.integers(0, 1 << 53, size=shape, dtype=np.int64)
    return k.astype(np.float64) * (1.0 / (1 << 53))


class _Noise:
    """Draws depolarising events; fire uniform then Pauli-choice uniform."""

    def __init__(self, seed: int, n_shots: int, n: int, p: float):
        self.g = _rng(seed, 2)
        self.S, self.n, self.p = n_shots, n, p

    def empty(self):
        return np.zeros((self.S, self.n), bool), np.zeros((self.S, self.n), bool)

    def _fire(self, rate, count):
        u1 = _uniform53(self.g, (self.S, count))
        u2 = _uniform53(self.g, (self.S, count))
        return u1 < rate, u2

    def one_qubit(self, qubits, rate):
        x, z = self.empty()
        if rate <= 0 or not qubits:
            return x, z
        fire, u2 = self._fire(rate, len(qubits))
        k = np.minimum((u2 * 3).astype(np.int64), 2)
        codes = np.array(_ONE_Q)[k]
        for j, q in enumerate(qubits):
            c = np.where(fire[:, j], codes[:, j], 0)
            x[:, q] ^= (c & 1).astype(bool)
            z[:, q] ^= (c >> 1 & 1).astype(bool)
        return x, z

    def two_qubit(self, pairs, rate):
        x, z = self.empty()
        if rate <= 0 or not pairs:
            return x, z
        fire, u2 = self._fire(rate, len(pairs))
        k = np.minimum((u2 * 15).astype(np.int64), 14)
        ca = np.array([a for a, _ in _TWO_Q])[k]
        cb = np.array([b for _, b in _TWO_Q])[k]
        for j, (q0, q1) in enumerate(pairs):
            c0 = np.where(fire[:, j], ca[:, j], 0)
            c1 = np.where(fire[:, j], cb[:, j], 0)
            x[:, q0] ^= (c0 & 1).astype(bool)
            z[:, q0] ^= (c0 >> 1 & 1).astype(bool)
            x[:, q1] ^= (c1 & 1).astype(bool)
            z[:, q1] ^= (c1 >> 1 & 1).astype(bool)
        return x, z

    def x_flip(self, qubits, rate):
        x, z = self.empty()
        if rate <= 0 or not qubits:
            return x, z
        u1 = _uniform53(self.g, (self.S, len(qubits)))
        for j, q in enumerate(qubits):
            x[:, q] = u1[:, j] < rate
        return x, z


def memory_circuit(d: int, rounds: int, n_shots: int, *, seed: int = 1,
                   theta_nn=0.05, nnn: bool = False, theta_triple=None,
                   theta_law: str = "fixed", theta_range=(0.02, 0.10),
                   p: float = 0.0, per_layer_params: bool = False,
                   random_sign: bool = False, final_readout: bool = True,
                   dense_noise: bool = False, crosstalk: str = "coherent", basis: str = "Z") -> Circuit:
    """Memory-Z experiment on the rotated code with ZZ(Z) crosstalk.

    dense_noise: emit a noise op at every noise location even when no shot
    fires there, so that the op sequence does not depend on the seed (one
    captured graph then serves every batch of shots).

    theta_law:
      "fixed"        every NN coupling gets theta_nn, NNN theta_nn/2, triples theta_triple
      "per_coupling" one U[theta_range] draw per NN coupling shared by shots and
                     layers; NNN get their own draw halved
      "per_shot"     independent U[theta_range] per shot and coupling; NNN halved
    per_layer_params: each rotation instance (coupling x layer x round) gets
      its own angle parameter index (used for gradients).
    random_sign: each rotation instance and shot flips the sign of its angle
      with probability 1/2 (Eq. 9).
    basis: "Z" (memory-Z: data start in |0> and are read out in Z) or "X"
      (memory-X: H on every data qubit after the first reset and before the
      final readout, so the X checks are the deterministic ones and the
      readout is in X; ZZ crosstalk then acts on the protected observable).
    crosstalk:
      "coherent"  rotations exp(-i theta Z..Z) (Eq. 4)
      "pta"       their Pauli-twirled approximation (Eq. 6): each coupling
                  and shot applies Z..Z with probability sin^2(theta), drawn
                  from its own stream, as a Pauli noise op (no rotation, so
                  the run is Clifford-only)
    """
    if crosstalk not in ("coherent", "pta"):
        raise ValueError(crosstalk)
    if basis not in ("Z", "X"):
        raise ValueError(basis)
    lay = rotated_layout(d)
    n = lay.n
    S = n_shots
    layers = cnot_layers(lay)
    nn = nn_couplings(lay)
    nnn = nnn_couplings(lay) if nnn else []
    tri = ancilla_triples(lay) if theta_triple else []
    paulis = [list(c) + [-1] * (3 - len(c)) for c in nn + nnn + tri]
    paulis = np.array(paulis, dtype=np.int32).reshape(-1, 3)
    R = len(paulis)
    g_theta = _rng(seed, 1)
    if theta_law == "fixed":
        base = np.array([theta_nn] * len(nn) + [theta_nn / 2] * len(nnn)
                        + [theta_triple or 0.0] * len(tri), dtype=np.float64)
        theta_layer = np.broadcast_to(base, (S, R)).copy()
    elif theta_law == "per_coupling":
        lo, hi = theta_range
        t_nn = lo + (hi - lo) * _uniform53(g_theta, (len(nn),))
        t_nnn = (lo + (hi - lo) * _uniform53(g_theta, (len(nnn),))) / 2
        t_tri = np.full(len(tri), theta_triple or 0.0)
        base = np.concatenate([t_nn, t_nnn, t_tri])
        theta_layer = np.broadcast_to(base, (S, R)).copy()
    elif theta_law == "per_shot":
        lo, hi = theta_range
        t_nn = lo + (hi - lo) * _uniform53(g_theta, (S, len(nn)))
        t_nnn = (lo + (hi - lo) * _uniform53(g_theta, (S, len(nnn)))) / 2
        t_tri = np.full((S, len(tri)), theta_triple or 0.0)
        theta_layer = np.concatenate([t_nn, t_nnn, t_tri], axis=1)
    else:
        raise ValueError(theta_law)
    g_sign = _rng(seed, 4)
    g_pta = _rng(seed, 5)
    noise = _Noise(seed, S, n, p)
    g_meas = _rng(seed, 3)
    ops = []
    anc = lay.ancillas
    n_params = 0

    def add_noise(xz):
        x, z = xz
        if dense_noise or x.any() or z.any():
            ops.append({"op": "noise", "x": x, "z": z})

    for rnd in range(rounds):
        add_noise(noise.x_flip(anc + (lay.data if rnd == 0 else []), 2 * p))
        if rnd == 0 and basis == "X":
            ops.append({"op": "gates", "gates": [("H", q, -1) for q in lay.data]})
            add_noise(noise.one_qubit(lay.data, 0.1 * p))
        if lay.x_anc:
            ops.append({"op": "gates", "gates": [("H", a, -1) for a in lay.x_anc]})
            add_noise(noise.one_qubit(lay.x_anc, 0.1 * p))
        for t in range(4):
            ops.append({"op": "gates", "gates": [("CX", c, q) for c, q in layers[t]]})
            add_noise(noise.two_qubit(layers[t], p))
            if R:
                th = theta_layer.copy()
                if random_sign:
                    flip = _uniform53(g_sign, (S, R)) < 0.5
                    th = np.where(flip, -th, th)
                if crosstalk == "pta":
                    fire = _uniform53(g_pta, (S, R)) < np.sin(th) ** 2
                    z = np.zeros((S, n), dtype=bool)
                    for c in range(R):
                        for q in paulis[c]:
                            if q >= 0:
                                z[:, q] ^= fire[:, c]
                    add_noise((np.zeros((S, n), dtype=bool), z))
                    continue
                if per_layer_params:
                    param = np.arange(n_params, n_params + R, dtype=np.int32)
                    n_params += R
                else:
                    param = np.arange(R, dtype=np.int32)
                    n_params = R
                ops.append({"op": "rotate", "paulis": paulis.copy(), "theta": th,
                            "param": param})
        if lay.x_anc:
            ops.append({"op": "gates", "gates": [("H", a, -1) for a in lay.x_anc]})
            add_noise(noise.one_qubit(lay.x_anc, 0.1 * p))
        add_noise(noise.x_flip(anc, 5 * p))
        ops.append({"op": "measure", "qubits": np.array(anc, np.int32), "reset": True,
                    "u": _uniform53(g_meas, (S, len(anc)))})
    if final_readout:
        if basis == "X":
            ops.append({"op": "gates", "gates": [("H", q, -1) for q in lay.data]})
            add_noise(noise.one_qubit(lay.data, 0.1 * p))
        add_noise(noise.x_flip(lay.data, 5 * p))
        ops.append({"op": "measure", "qubits": np.array(lay.data, np.int32), "reset": False,
                    "u": _uniform53(g_meas, (S, len(lay.data)))})
    meta = {"d": d, "rounds": rounds, "p": p, "theta_law": theta_law, "crosstalk": crosstalk, "basis": basis,
            "n_nn": len(nn), "n_nnn": len(nnn), "n_tri": len(tri)}
    return Circuit(n, S, ops, lay, n_params, meta)


# --------------------------------------------------------------------------
# Named workloads.  Sizes follow the five configurations this project is
# measured on; seeds are fixed so that every run draws the same inputs.
# --------------------------------------------------------------------------

CONFIGS = {
    # d=3, 3 rounds, theta=0.05 on NN pairs, no depolarising, complex128, chi 64
    "d3_nn_chi64": dict(d=3, rounds=3, n_shots=100, theta_nn=0.05, p=0.0,
                        chi_max=64, precision="fp64", seed=11),
    # d=5, 5 rounds, per-coupling theta in [0.02, 0.10], NNN at half, p=1e-3,
    # chi 256, FP32 contractions with FP64 truncation, 1024 shots
    "d5_nnn_chi256": dict(d=5, rounds=5, n_shots=1024, theta_law="per_coupling", nnn=True,
                          theta_range=(0.02, 0.10), p=1e-3, chi_max=256,
                          precision="fp32", seed=21),
    # the d=5 workload at the bond cap the paper uses for all its results
    # (chi 32, Sec. IV.B): chi binds from the second round on
    "d5_nnn_chi32": dict(d=5, rounds=5, n_shots=1024, theta_law="per_coupling", nnn=True,
                         theta_range=(0.02, 0.10), p=1e-3, chi_max=32,
                         precision="fp32", seed=21),
    # d=7, 7 rounds, per-shot theta in [0.01, 0.08], NNN at half, chi 512
    "d7_nnn_chi512": dict(d=7, rounds=7, n_shots=4096, theta_law="per_shot", nnn=True,
                          theta_range=(0.01, 0.08), p=0.0, chi_max=512,
                          precision="fp32", seed=31),
    # d=5 gradient: one parameter per NN coupling per layer, theta=0.05, chi 128
    "d5_grad_chi128": dict(d=5, rounds=5, n_shots=1, theta_nn=0.05, p=0.0,
                           per_layer_params=True, chi_max=128, precision="fp64", seed=41),
    # d=9, 9 rounds, theta=0.04 NN plus ancilla-centred ZZZ at 0.01, chi 1024
    "d9_tri_chi1024": dict(d=9, rounds=9, n_shots=512, theta_nn=0.04, theta_triple=0.01,
                           p=0.0, chi_max=1024, precision="fp32", seed=51),
}


def make_config(name: str, **override) -> tuple:
    """Returns (Circuit, run options) for a named workload."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    opts = {k: cfg.pop(k) for k in ("chi_max", "precision") if k in cfg}
    circ = memory_circuit(**cfg)
    circ.meta["name"] = name
    return circ, opts

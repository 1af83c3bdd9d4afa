"""Decoding of memory experiments and the logical error rate P_L (Eq. 1).

The decoder itself is native (stn_decode in libstn: union-find over a
detector graph, host code).  This module builds its inputs from a workload
circuit and a run's records:

* detector_graph: the detectors of a memory-B experiment (B = Z or X, the
  circuit's basis) are the checks of type B in every syndrome round plus a
  final layer formed from the data readout.  Edges are the error mechanisms
  of a Pauli model of the circuit: a flip of data qubit j in a round (the
  type-B checks that contain j, or one check and the boundary when j sits
  on the boundary; it flips the observable when j is on the logical
  operator) and a flip of check a's outcome (between consecutive layers).
  Their probabilities come from the Pauli-twirled noise (Sec. III.D): the
  depolarising rates of Eqs. 2-3 with the Table I ratios, and for memory-X
  the crosstalk flips of Eq. 6 (sin^2 theta per ZZ coupling per CNOT layer;
  ZZ commutes with the Z observable of memory-Z).  The weights are
  log((1 - p) / p).  Hook and diagonal mechanisms of the circuit-level
  model are left out.
* detection_events: d(0, a) = m(0, a) (the first outcome of a type-B check
  is deterministic), d(r, a) = m(r, a) xor m(r-1, a), and the final layer
  compares the check's value recomputed from the data readout with its last
  measured outcome.
* logical_error_rate: P_L of Eq. 1 with theta_i in {0, pi}, i.e. the
  fraction of shots whose decoded observable is flipped (the Pauli case in
  which Eq. 1 is the ordinary logical error rate).  The per-syndrome
  logical rotation angle of a coherent run is not given by the paper; this
  estimator averages sin^2(theta_i / 2) over the sampled readouts instead of
  |sin(theta_i / 2)|.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Tuple

import numpy as np

from . import workload as W


class DemEdge(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("weight", ctypes.c_double),
                ("obs", ctypes.c_uint8), ("pad", ctypes.c_uint8 * 7)]


def _lib():
    from . import stn
    lib = stn.load()
    lib.stn_decode.restype = ctypes.c_int
    lib.stn_decode.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p]
    return lib


def checks(lay: W.Layout, basis: str) -> Tuple[List[int], Dict[int, List[int]]]:
    """The type-`basis` ancillas and, for each, its data qubits."""
    anc = lay.z_anc if basis == "Z" else lay.x_anc
    sup = {}
    for a in anc:
        y, x = lay.coords[a]
        sup[a] = [lay.index[(y + dy, x + dx)] for dy, dx in (W.NW, W.NE, W.SW, W.SE)
                  if (y + dy, x + dx) in lay.index]
    return sorted(anc), sup


def logical_support(lay: W.Layout, basis: str) -> List[int]:
    """Data qubits of a logical operator of type `basis`: a row or column of
    data whose overlap with every check of the other type is even."""
    _, other = checks(lay, "X" if basis == "Z" else "Z")
    d = lay.d
    cands = [[lay.index[(2 * r + 1, 2 * c + 1)] for c in range(d)] for r in range(d)]
    cands += [[lay.index[(2 * r + 1, 2 * c + 1)] for r in range(d)] for c in range(d)]
    for cand in cands:
        s = set(cand)
        if all(len(s.intersection(q)) % 2 == 0 for q in other.values()):
            return sorted(cand)
    raise RuntimeError("no logical operator found")


def _coupling_flip_rates(circ) -> np.ndarray:
    """Per qubit, the summed Pauli-twirled flip probability sin^2(theta) of
    its crosstalk couplings in one CNOT layer (Eq. 6), averaged over shots."""
    rot = next((o for o in circ.ops if o["op"] == "rotate"), None)
    out = np.zeros(circ.n)
    if rot is None:
        return out
    s2 = np.mean(np.sin(rot["theta"]) ** 2, axis=0)
    for c, qs in enumerate(rot["paulis"]):
        for q in qs:
            if q >= 0:
                out[q] += s2[c]
    return out


def detector_graph(circ, p: float = None) -> Tuple[List[DemEdge], int, dict]:
    """Edges of the memory experiment's detector graph (see module doc),
    the number of detectors, and the node map {(layer, ancilla): index}."""
    lay = circ.layout
    basis = circ.meta.get("basis", "Z")
    p = circ.meta.get("p", 0.0) if p is None else p
    R = circ.meta["rounds"]
    anc, sup = checks(lay, basis)
    L = set(logical_support(lay, basis))
    node = {(r, a): r * len(anc) + i for r in range(R + 1) for i, a in enumerate(anc)}
    n_nodes = (R + 1) * len(anc)
    bnd = n_nodes
    xt = _coupling_flip_rates(circ) if basis == "X" else np.zeros(circ.n)
    # per round: four CNOTs per data qubit (two-qubit depolarising, 8 of the
    # 15 Paulis act on a given qubit with the flipping component), four
    # crosstalk layers; an ancilla outcome also flips on reset (2p) and
    # readout (5p)
    def clip(q):
        return float(min(max(q, 1e-12), 0.49))
    p_data = {j: clip(4 * 8 * p / 15 + 4 * xt[j]) for j in lay.data}
    p_anc = {a: clip(4 * 8 * p / 15 + 2 * p + 5 * p + 4 * xt[a]) for a in anc}
    where: Dict[int, List[int]] = {j: [] for j in lay.data}
    for a in anc:
        for j in sup[a]:
            where[j].append(a)
    edges = []
    for r in range(R + 1):
        for j in lay.data:
            ends = [node[(r, a)] for a in where[j]]
            if not ends:
                continue
            b = ends[1] if len(ends) > 1 else bnd
            w = float(np.log((1 - p_data[j]) / p_data[j]))
            edges.append(DemEdge(ends[0], b, w, 1 if j in L else 0))
        if r < R:
            for a in anc:
                w = float(np.log((1 - p_anc[a]) / p_anc[a]))
                edges.append(DemEdge(node[(r, a)], node[(r + 1, a)], w, 0))
    return edges, n_nodes, node


def _final_readout(circ, records) -> Tuple[np.ndarray, np.ndarray]:
    """(ancilla outcomes [S, R, n_checks] of the type-B checks, data
    outcomes [S, n_data] of the final readout) from the records."""
    lay = circ.layout
    basis = circ.meta.get("basis", "Z")
    anc, _ = checks(lay, basis)
    rounds, col = [], 0
    data = None
    for o in circ.ops:
        if o["op"] != "measure":
            continue
        qs = list(o["qubits"])
        m = np.asarray(records[:, col:col + len(qs)], np.uint8)
        col += len(qs)
        if o["reset"]:
            rounds.append(m[:, [qs.index(a) for a in anc]])
        else:
            data = m[:, [qs.index(j) for j in lay.data]]
    return np.stack(rounds, axis=1), data


def detection_events(circ, records) -> np.ndarray:
    """uint8 [S, n_nodes] detection events of a run's records."""
    lay = circ.layout
    basis = circ.meta.get("basis", "Z")
    anc, sup = checks(lay, basis)
    m, data = _final_readout(circ, records)
    pos = {j: i for i, j in enumerate(lay.data)}
    final = np.stack([np.bitwise_xor.reduce(data[:, [pos[j] for j in sup[a]]], axis=1) for a in anc], axis=1)
    layers = [m[:, 0]]
    for r in range(1, m.shape[1]):
        layers.append(m[:, r] ^ m[:, r - 1])
    layers.append(final ^ m[:, -1])
    return np.ascontiguousarray(np.concatenate(layers, axis=1), np.uint8)


def observed_flip(circ, records) -> np.ndarray:
    """The logical observable read out at the end (0 = unchanged), per shot."""
    lay = circ.layout
    _, data = _final_readout(circ, records)
    pos = {j: i for i, j in enumerate(lay.data)}
    L = logical_support(lay, circ.meta.get("basis", "Z"))
    return np.bitwise_xor.reduce(data[:, [pos[j] for j in L]], axis=1).astype(np.uint8)


def decode(edges: List[DemEdge], n_nodes: int, events: np.ndarray, corrections: bool = False):
    """Predicted observable flip per shot (and the corrections, uint8
    [S, n_edges], when asked) from stn_decode."""
    lib = _lib()
    arr = (DemEdge * len(edges))(*edges)
    ev = np.ascontiguousarray(events, np.uint8)
    S = ev.shape[0]
    pred = np.zeros(S, np.uint8)
    corr = np.zeros((S, len(edges)), np.uint8) if corrections else None
    st = lib.stn_decode(ctypes.cast(arr, ctypes.c_void_p), len(edges), n_nodes, ev.ctypes.data_as(ctypes.c_void_p),
                        S, pred.ctypes.data_as(ctypes.c_void_p),
                        corr.ctypes.data_as(ctypes.c_void_p) if corrections else None)
    if st != 0:
        raise ValueError(f"stn_decode failed with status {st}")
    return (pred, corr) if corrections else pred


def logical_error_rate(circ, records) -> dict:
    """P_L (Eq. 1, Pauli case) of a run: decoded failures / shots."""
    edges, n_nodes, _ = detector_graph(circ)
    ev = detection_events(circ, records)
    pred = decode(edges, n_nodes, ev)
    fail = (pred ^ observed_flip(circ, records)).astype(bool)
    S = len(fail)
    pl = float(fail.mean()) if S else 0.0
    return {"P_L": pl, "failures": int(fail.sum()), "shots": S,
            "stderr": float(np.sqrt(pl * (1 - pl) / S)) if S else 0.0,
            "detection_fraction": float(ev.mean()) if ev.size else 0.0}

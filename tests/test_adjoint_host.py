"""Host logic of the checkpointed gradient driver (CPU only)."""
import numpy as np

from paper_2605_29514_amd import adjoint
from paper_2605_29514_amd import workload as W


def test_stretches_end_with_measurements():
    ops = [("gates",), ("rotate", [1, 2]), ("measure", [0]), ("noise",), ("rotate", [3]), ("measure", [1, 2]),
           ("gates",)]
    assert adjoint.stretches(ops) == [(0, 3), (3, 6), (6, 7)]
    assert adjoint.stretches([("measure", [0])]) == [(0, 1)]


def test_step_and_rotation_counts():
    ops = [("gates",), ("rotate", [[0, 1, -1], [1, 2, -1]]), ("measure", [0, 1]), ("rotate", [[2, 3, -1]])]
    assert adjoint._rots_in(ops, 0, 4) == 3
    assert adjoint._steps_in(ops, 0, 4) == 5
    assert adjoint._steps_in(ops, 0, 1) == 0


def test_rotation_count_matches_parameters():
    circ = W.memory_circuit(3, 2, 1, seed=5, theta_nn=0.1, p=0.02, per_layer_params=True)
    assert adjoint.rotation_count(circ) == circ.n_params == 2 * 4 * 24

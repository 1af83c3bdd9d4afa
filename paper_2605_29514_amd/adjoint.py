"""d log P(record) / d theta through libstn's adjoint pass, with per-stretch
checkpoints, and a torch.autograd.Function around it.

Forward: the circuit runs once with a checkpoint (stn_checkpoint_save) at
the start of every stretch (by default each syndrome round, i.e. each run
of ops ending in a measurement).  Backward: stretches are replayed last
first -- checkpoint restored, the stretch re-run with its recorded outcomes
forced while the library records a tape, then stn_backward carries the
adjoint state back through it and writes the gradient of every rotation of
the stretch.  Memory: one checkpoint per stretch plus one tape (a state
snapshot per non-Clifford step of one stretch).

The angles are per shot: theta[s, i] is the angle of the i-th rotation (in
circuit order) of shot s; the gradient has the same layout.  The truncation
reading (projectors held fixed where chi_max dropped weight, exact
elsewhere) is the library's; see include/stn.h.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import stn


def rotation_count(circ) -> int:
    return sum(len(op["paulis"]) for op in circ.ops if op["op"] == "rotate")


def stretches(ops) -> List[Tuple[int, int]]:
    """[start, stop) op ranges, each ending with a measurement op."""
    out, start = [], 0
    for i, op in enumerate(ops):
        if op[0] == "measure":
            out.append((start, i + 1))
            start = i + 1
    if start < len(ops):
        out.append((start, len(ops)))
    return out


def _steps_in(ops, a, b) -> int:
    return sum(len(op[1]) for op in ops[a:b] if op[0] in ("rotate", "measure"))


def _rots_in(ops, a, b) -> int:
    return sum(len(op[1]) for op in ops[a:b] if op[0] == "rotate")


class GradientRun:
    """One checkpointed forward over a circuit with a fixed record, and its
    adjoint pass.  records: uint8 [S, n_measurements] (the outcomes to
    condition on); theta: optional float64 [S, R] angles replacing the
    circuit's."""

    def __init__(self, circ, chi_max: int, records: np.ndarray, precision: str = "fp64",
                 eps_cut: Optional[float] = None, chi_adj: Optional[int] = None, device: str = "cuda:0",
                 segments: Optional[Sequence[Tuple[int, int]]] = None, static_tape: bool = False):
        import torch
        self.torch = torch
        self.circ = circ
        self.sim = stn.Simulator(circ.n, circ.n_shots, chi_max, precision, eps_cut, device, layer_mode=1)
        self.ops = stn.prepare(circ, device, forced=np.asarray(records, np.uint8), per_shot_theta=True)
        self.R = rotation_count(circ)
        self.segments = list(segments) if segments is not None else stretches(self.ops)
        self.chi_adj = chi_adj or min(512, max(8 * chi_max, 64))
        self.checkpoints = []
        self.device = device
        # record into the library's static per-GPU tape instead of a torch buffer
        self.static_tape = static_tape

    def set_theta(self, theta) -> None:
        """theta: [S, R] tensor of per-shot angles in circuit rotation order."""
        col = 0
        for op in self.ops:
            if op[0] == "rotate":
                k = len(op[1])
                op[2].copy_(theta[:, col:col + k])
                col += k

    def forward(self):
        """Runs the circuit with checkpoints; returns log P per shot."""
        self.sim.reset()
        self.checkpoints = []
        for a, b in self.segments:
            self.checkpoints.append(self.sim.checkpoint_save())
            stn.run_prepared(self.sim, self.ops, a, b)
        lp, _ = self.sim.logprob()
        return lp

    def backward(self):
        """dJ/dtheta per shot and rotation, [S, R] float64 (device)."""
        torch = self.torch
        sim = self.sim
        grad = torch.zeros((self.circ.n_shots, self.R), dtype=torch.float64, device=sim.device)
        if not hasattr(sim, "_adj"):
            sim.adjoint_init(self.chi_adj)
        sim.adjoint_zero()
        col_end = self.R
        for (a, b), ck in reversed(list(zip(self.segments, self.checkpoints))):
            nrot = _rots_in(self.ops, a, b)
            col = col_end - nrot
            sim.checkpoint_load(ck)
            if self.static_tape:
                sim.tape_begin_static(max(1, _steps_in(self.ops, a, b)))
            else:
                sim.tape_begin(max(1, _steps_in(self.ops, a, b)))
            stn.run_prepared(sim, self.ops, a, b)
            got = sim.tape_end()
            assert got == nrot, (got, nrot)
            if _steps_in(self.ops, a, b):
                sim.backward(grad, col)
            col_end = col
        self.adjoint_truncated = sim.adjoint_truncated()
        return grad


class CircuitLogProb:
    """torch.autograd.Function factory: logp = CircuitLogProb(run)(theta)
    with theta [S, R] float64 on the device; backward returns
    grad_output[s] * dJ_s/dtheta[s, :]."""

    def __new__(cls, run: GradientRun):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta):
                run.set_theta(theta.detach())
                return run.forward().clone()

            @staticmethod
            def backward(ctx, grad_out):
                g = run.backward()
                return g * grad_out.to(g.dtype)[:, None]

        return _Fn.apply

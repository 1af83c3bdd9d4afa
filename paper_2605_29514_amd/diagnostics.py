"""Truncation diagnostics of a run: what chi_max does to the state and to the
syndromes (Sec. IV.B, Figs. 2-3), from the MPS and the records only.

* the Schmidt spectrum across a cut comes from the library (stn_spectrum:
  FP64 Gram of the centre tensor and Jacobi eigen-solve on the device, every
  shot at once); nothing here recomputes it from returned tensors.
* detection_rates: per syndrome round, the fraction of detection events
  (an ancilla outcome that differs from the same ancilla's previous one; in
  the first round only the Z checks, whose noiseless outcome is 0).
* chi_sweep: runs one circuit at several chi_max and collects, per chi_max,
  the per-shot truncation error and log P, the detection rates and the
  Schmidt spectrum of a chosen shot at the centre cut just before every
  round's ancilla measurement.

CLI: python -m paper_2605_29514_amd.diagnostics --config d5_nnn_chi32 --shots 64 --rounds 2 --chis 8,16,32
"""
from __future__ import annotations

import argparse
import json
from typing import Dict, List, Optional, Sequence

import numpy as np


def measurement_rounds(circ) -> List[np.ndarray]:
    """Qubits measured by each ancilla round (reset) of a workload circuit, in
    record order."""
    return [np.asarray(o["qubits"]) for o in circ.ops if o["op"] == "measure" and o["reset"]]


def detection_rates(circ, records: np.ndarray) -> List[float]:
    """Fraction of detection events per syndrome round over all shots."""
    rounds = measurement_rounds(circ)
    z_anc = set(circ.layout.z_anc) if circ.layout is not None else set()
    out, col, prev = [], 0, None
    for qs in rounds:
        m = np.asarray(records[:, col:col + len(qs)], dtype=np.uint8)
        col += len(qs)
        if prev is None:
            keep = np.array([q in z_anc for q in qs])
            ev = m[:, keep]
        else:
            ev = m ^ prev
        out.append(float(ev.mean()) if ev.size else 0.0)
        prev = m
    return out


def chi_sweep(circ, chis: Sequence[int], precision: str = "fp32", shot: int = 0,
              cut: Optional[int] = None, device: str = "cuda:0", layer_mode: int = 0,
              top: int = 64) -> Dict[int, dict]:
    """Runs circ at every chi_max in chis (same inputs, sampled records);
    `cut` names the bond between sites cut and cut + 1 (default: the centre),
    and the spectra (the largest `top` squared Schmidt values of `shot`) come
    from the device before every round's ancilla measurement."""
    from . import stn
    import torch
    cut = circ.n // 2 - 1 if cut is None else cut
    out = {}
    for chi in chis:
        sim = stn.Simulator(circ.n, circ.n_shots, chi, precision, None, device, layer_mode=layer_mode)
        ops = stn.prepare(circ, device)
        res, spectra, start = [], [], 0
        for i, op in enumerate(ops):
            if op[0] == "measure" and op[2]:            # an ancilla round ends here
                stn.run_prepared(sim, ops, start, i, records=res)
                sim.sync()
                vals, _ = sim.spectrum(cut + 1)
                spectra.append(vals[shot, :top].cpu().numpy().tolist())
                start = i
        stn.run_prepared(sim, ops, start, None, records=res)
        lp, te = sim.logprob()
        rec = torch.cat([r[0] for r in res], dim=1).cpu().numpy()
        out[chi] = {"trunc_err": te.cpu().numpy().tolist(), "logp": lp.cpu().numpy().tolist(),
                    "detection_rate": detection_rates(circ, rec), "spectra": spectra,
                    "max_bond": int(sim.bonds().max())}
        del sim
    return out


def main(argv=None):
    from . import workload
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--config", default="d5_nnn_chi32")
    ap.add_argument("--shots", type=int, default=64)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--chis", default="8,16,32")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--json", action="store_true", help="print the full result as JSON")
    a = ap.parse_args(argv)
    circ, opts = workload.make_config(a.config, n_shots=a.shots, rounds=a.rounds)
    prec = a.precision or opts["precision"]
    chis = [int(c) for c in a.chis.split(",")]
    res = chi_sweep(circ, chis, prec)
    if a.json:
        print(json.dumps(res))
        return
    for chi, r in res.items():
        te = np.array(r["trunc_err"])
        head = ", ".join(f"{x:.2e}" for x in r["spectra"][-1][:4]) if r["spectra"] else ""
        print(f"chi_max {chi:4d}: max bond {r['max_bond']:4d}, truncation error mean {te.mean():.3e} "
              f"max {te.max():.3e}, mean log P {np.mean(r['logp']):.4f}, detection rate per round "
              f"{[round(x, 4) for x in r['detection_rate']]}, last centre-cut spectrum [{head}, ...]")


if __name__ == "__main__":
    main()

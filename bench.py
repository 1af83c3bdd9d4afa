"""Throughput benchmark of the STN crosstalk step on one MI355X.

Workload: rotated surface code d=5 memory-Z experiment (49 qubits, 5
syndrome rounds), ZZ crosstalk after each of the 4 CNOT layers on the 80
nearest-neighbour pairs (theta ~ U[0.02, 0.10] per coupling) and the 72
next-nearest pairs (own draw, halved), depolarising p = 1e-3 (Table I
ratios), chi_max = 256, FP32 complex contractions with FP64 Gram, eigen-solve
and norms, 1024 shots batched.  All inputs are seeded and synthetic and are
resident in device memory before the timed region starts.

A step is one syndrome-extraction round over every shot: Clifford layers and
noise (tableau), 608 crosstalk rotations (rewrite, bond-2 update, QR sweep,
Gram/eigen truncation) and 24 ancilla measurements (projection, frame change,
reset); the last round also reads out the data qubits.  --warmup W rounds run
untimed first (they are the circuit's own first rounds), then --steps K rounds
are timed.

Prints one JSON line.  value = (shots x rotations in the timed rounds) / time.
roofline: the kernel class with the largest time in the timed region, its
algorithmic work (counted on the device from the realised bond dimensions,
in a replay of the same rounds: the counters slow the kernels they count)
over its own launch time (HIP events on the library stream, timed pass).
plain_fp64: the plain per-shot FP64 GPU form (per-step kernels, one shot at a
time) of the same rounds on the first shots, with the batched records
forced, within a time budget (--plain-seconds): its rotation rate and the
largest relative difference of the batched FP32 probabilities from it.
cpu_baseline: the FP64 oracle timed on the host cores over a bounded sample
of the same rounds (see --cpu-seconds).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp32_vector_TFs": 157.3,
    "fp64_vector_TFs": 78.6,
    "fp32_mfma_TFs": 157.3,
    "fp64_mfma_TFs": 78.6,
}
# which unit bounds each kernel class of the current kernels
CLASS_BOUND = {
    "eigen": ("alu", "fp64_vector_TFs"),    # FP64 Jacobi rotations on vector ALUs
    "gram": ("alu", "fp64_vector_TFs"),     # FP64-accumulated FMA tiles
    "expect": ("alu", "fp64_vector_TFs"),
    "qr": ("alu", None),                    # precision-dependent
    "gemm": ("alu", None),
    "build": ("hbm", "hbm_GBs"),
    "select": ("hbm", "hbm_GBs"),
    "tableau": ("hbm", "hbm_GBs"),
    "layer": ("alu", None),                 # fused layer kernel: mixed FP32 / FP64 work
}


def kernel_source_hash():
    """sha256 (first 16 hex) of the kernel sources, in a fixed order; a
    stored traffic figure counts only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "linalg.h", "mps.hip", "layer.hip"):
        with open(os.path.join(ROOT, "paper_2605_29514_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 PMC
    summary (profiles/traffic_*.json), or None when no summary matches the
    class or the kernel source changed since the counters were taken."""
    import glob
    sha = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as f:
            t = json.load(f)
        if t.get("kernel_class") == kernel_class and t.get("source_sha256_16") == sha:
            return float(t["traffic_bytes_per_launch"])
    return None


def split_rounds(ops):
    """Indices [start, stop) of each syndrome round in prepared ops; a round
    ends with an ancilla measurement (the final data readout joins the last)."""
    bounds, start = [], 0
    for i, op in enumerate(ops):
        if op[0] == "measure" and op[2]:          # reset=True: ancilla round end
            bounds.append([start, i + 1])
            start = i + 1
    if start < len(ops):
        bounds[-1][1] = len(ops)
    return bounds


def rotations_in(circ_ops, lo, hi):
    return sum(len(o[1]) for o in circ_ops[lo:hi] if o[0] == "rotate")


# ----------------------------------------------------------------- CPU leg
def _oracle_worker(args):
    """Runs shots of the workload on the FP64 oracle, one after the other,
    timing only the rotations of the timed rounds, until the time budget is
    used; returns (rotations timed, seconds timed)."""
    name, shots, shots_total, t_lo, t_hi, budget, chi, eps = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import stn as ostn
    from paper_2605_29514_amd import workload
    circ, _ = workload.make_config(name, n_shots=shots_total)
    done, busy = 0, 0.0
    for shot in shots:
        if busy > budget:
            break
        st = ostn.Shot(circ.n, chi, eps)
        for oi, op in enumerate(circ.ops[:t_hi]):
            timed = oi >= t_lo
            k = op["op"]
            if k == "gates":
                for g in op["gates"]:
                    st.gate(g[0], [g[1], g[2]])
            elif k == "noise":
                st.pauli_noise(op["x"][shot], op["z"][shot])
            elif k == "rotate":
                for ri, qs in enumerate(op["paulis"]):
                    t0 = time.perf_counter()
                    st.rotate([int(q) for q in qs], float(op["theta"][shot, ri]))
                    if timed:
                        busy += time.perf_counter() - t0
                        done += 1
            elif k == "measure":
                for mj, q in enumerate(op["qubits"]):
                    st.measure(int(q), float(op["u"][shot, mj]), None, bool(op["reset"]))
    return done, busy


def plain_fp64_form(circ, chi, rounds, W, K, batched, n, dev, budget_s):
    """The plain per-shot FP64 GPU form of the same rounds: per-step kernels,
    one shot at a time, FP64 throughout, on up to the first n shots with the
    batched run's records forced, until budget_s seconds are spent (at least
    one timed round).  Returns its rotation rate over the timed rounds it ran
    and the largest relative difference of the batched FP32 probabilities
    from it over the measurements it ran."""
    import torch
    from paper_2605_29514_amd import stn
    rec = torch.cat([r[0] for r in batched], dim=1)[:n].cpu().numpy()
    prob = torch.cat([r[1] for r in batched], dim=1)[:n].cpu().numpy()
    full = np.zeros((n, circ.n_measurements), np.uint8)
    full[:, :rec.shape[1]] = rec
    ms_total, rot_total, worst, shots_used = 0.0, 0, 0.0, 0
    t_start = time.perf_counter()
    for s in range(n):
        c1 = circ.shot_slice(s, s + 1)
        sim = stn.Simulator(c1.n, 1, chi, "fp64", None, dev, layer_mode=1)
        ops1 = stn.prepare(c1, dev, forced=full[s:s + 1])
        r1 = split_rounds(ops1)
        res = []
        for r in range(W + K):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(sim.stream)
            stn.run_prepared(sim, ops1, *r1[r], records=res)
            b.record(sim.stream)
            sim.sync()
            if r >= W:
                ms_total += a.elapsed_time(b)
                rot_total += rotations_in(ops1, *r1[r])
            print(f"# plain FP64 form: shot {s + 1}, round {r + 1} done", file=sys.stderr, flush=True)
            if r >= W and time.perf_counter() - t_start > budget_s:
                break
        p64 = torch.cat([x[1] for x in res], dim=1).cpu().numpy()[0]
        worst = max(worst, float(np.max(np.abs(prob[s, :p64.shape[0]] - p64) / p64)))
        shots_used += 1
        del sim
        if time.perf_counter() - t_start > budget_s:
            break
    return {"value": rot_total / (ms_total / 1e3), "unit": "rotations/s", "shots": shots_used,
            "timed_rotations": rot_total, "per_step_kernels": True, "precision": "fp64",
            "max_rel_prob_diff_batched_fp32": worst}


def cpu_baseline(name, circ, ops_bounds, t_lo_round, t_hi_round, chi, eps, budget, cores):
    """Oracle rotations/s over the same rounds: `cores` worker processes (BLAS
    1 thread each) take shots 0, 1, 2, ... round-robin and time the
    rotations of the timed rounds until each has spent `budget` seconds."""
    # prepared ops mirror the circuit ops one to one
    t_lo, t_hi = ops_bounds[t_lo_round][0], ops_bounds[t_hi_round - 1][1]
    per = [list(range(w, circ.n_shots, cores)) for w in range(cores)]
    args = [(name, per[w], circ.n_shots, t_lo, t_hi, budget, chi, eps) for w in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, args)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": done / busy if busy > 0 else 0.0, "unit": "rotations/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} worker processes (FP64 numpy oracle, BLAS 1 thread each) taking shots "
                      f"round-robin, each timing the rotations of the timed rounds until {budget:.0f} s were "
                      f"spent; {done} rotations, slowest worker {busy:.1f} s (wall incl. replays {wall:.1f} s)"}


# ----------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="d5_nnn_chi256")
    ap.add_argument("--shots", type=int, default=None, help="override the shot count (testing only)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-all", action="store_true")
    ap.add_argument("--layer-mode", type=int, default=0, help="0 automatic, 1 per-step kernels, 2 fused")
    ap.add_argument("--layer-threads", type=int, default=0, help="threads per shot of the fused kernel")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-shot FP64 GPU form (per-step kernels, one shot at a time)")
    ap.add_argument("--plain-shots", type=int, default=8)
    ap.add_argument("--plain-seconds", type=float, default=60.0,
                    help="time budget of the plain FP64 form (whole rounds; at least one)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scales HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "read_bytes": n, "write_bytes": n}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(shots would shard across GPUs with one final gather).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_29514_amd import stn, workload

    cfg = dict(workload.CONFIGS[args.config])
    over = {} if args.shots is None else {"n_shots": args.shots}
    circ, opts = workload.make_config(args.config, **over)
    chi, prec = opts["chi_max"], opts["precision"]
    eps = stn.DEFAULT_EPS[stn.STN_FP64 if prec == "fp64" else stn.STN_FP32]
    dev = "cuda:0"
    print(f"# building inputs: {args.config} shots={circ.n_shots}", file=sys.stderr, flush=True)
    sim = stn.Simulator(circ.n, circ.n_shots, chi, prec, eps, dev, layer_mode=args.layer_mode,
                        layer_threads=args.layer_threads)
    ops = stn.prepare(circ, dev)
    rounds = split_rounds(ops)
    schedule = {"layer_mode": args.layer_mode, "layer_threads": args.layer_threads, "tuned": False}
    W, K = args.warmup, args.steps
    if args.layer_mode == 0 and args.layer_threads == 0 and not args.no_tune and W + K <= len(rounds):
        from paper_2605_29514_amd import tune
        # tuning window: with one timed round, that whole round (its early
        # layers, where bonds are small, favour other block sizes than the
        # rest); with several, the first two crosstalk layers of the second
        # timed round (saturated rounds cost the most, a whole one per
        # candidate would take minutes).  Reached once, restored from a
        # checkpoint per candidate when that fits in memory.
        r0 = W + 1 if K >= 2 else W
        start = rounds[r0][0]
        if start > 0 and sim.lib.stn_checkpoint_bytes(sim.ctx) > (16 << 30):
            start = 0
        stop = rounds[r0][1] if K == 1 else tune.layers_stop(ops, 2, start)
        key = tune.problem_key(torch.cuda.get_device_name(0), circ.n, circ.n_shots, chi, prec, args.config)
        t = tune.autotune(sim, ops, stop, start=start, key=f"{key}|window@{start}:{stop}",
                          log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        schedule = {"layer_mode": t["choice"][0], "layer_threads": t["choice"][1], "tuned": True,
                    "cached": t["cached"], "candidates_ms": t["ms"], "tuning_window_ops": [start, stop]}
        print(f"# autotuned schedule {t['choice']}", file=sys.stderr, flush=True)
    if W + K > len(rounds):
        print(f"warmup + steps exceeds the {len(rounds)} rounds of the circuit", file=sys.stderr)
        sys.exit(2)
    torch.cuda.synchronize()
    batched = []                      # (outcomes, prob) device tensors of every measurement op run
    for r in range(W):
        t = time.perf_counter()
        stn.run_prepared(sim, ops, *rounds[r], records=batched)
        sim.sync()
        print(f"# warmup round {r + 1}: {time.perf_counter() - t:.2f} s, max bond "
              f"{int(sim.bonds().max())}", file=sys.stderr, flush=True)
    # Timed region: launch events per kernel class only.  The device work
    # counters (atomics from every block, per-phase clocks) slow the kernels
    # they count, so the work per launch comes from a counted replay below.
    prof_classes = None if args.profile_all else ["eigen", "qr", "gemm", "gram", "layer"]
    sim.profile(prof_classes, counters=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    round_ev = []
    for r in range(W, W + K):
        stn.run_prepared(sim, ops, *rounds[r], records=batched)
        round_ev.append(torch.cuda.Event())
        round_ev[-1].record(sim.stream)
    ev1.record(sim.stream)
    # progress: poll the per-round events (host side only; the GPU timeline
    # is what ev0 / ev1 measure)
    for i, e in enumerate(round_ev):
        while not e.query():
            time.sleep(0.05)
        print(f"# timed round {W + i + 1} done at {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    sim.sync()
    prof = sim.profile_read()
    lo, hi = rounds[W][0], rounds[W + K - 1][1]
    n_rot = rotations_in(ops, lo, hi) * circ.n_shots
    bonds = sim.bonds()
    value = n_rot / (ms / 1e3)
    # counted replay of the same rounds from the initial state (deterministic:
    # same launches, same bonds): algorithmic work per class, phase shares
    sim.profile([])
    sim.reset()
    for r in range(W):
        stn.run_prepared(sim, ops, *rounds[r])
    sim.profile(prof_classes, counters=True)
    for r in range(W, W + K):
        stn.run_prepared(sim, ops, *rounds[r])
        sim.sync()
        print(f"# counted replay of round {r + 1} done", file=sys.stderr, flush=True)
    work = sim.profile_read()
    phases = sim.profile_phases()
    sim.profile([])
    for c in stn.K_CLASSES:
        prof[c]["flops"], prof[c]["bytes"] = work[c]["flops"], work[c]["bytes"]
        if work[c]["launches"] != prof[c]["launches"]:
            print(f"# warning: class {c}: {prof[c]['launches']} timed launches, {work[c]['launches']} counted",
                  file=sys.stderr, flush=True)
    prof["layer_fp64_flops"], prof["eigen_sweeps"] = work["layer_fp64_flops"], work["eigen_sweeps"]
    # dominant kernel class by measured time
    classes = [c for c in stn.K_CLASSES if prof[c]["launches"] > 0]
    dom = max(classes, key=lambda c: prof[c]["ms"]) if classes else None
    roof = None
    if dom:
        bound, peak_key = CLASS_BOUND[dom]
        if peak_key is None:
            peak_key = "fp64_vector_TFs" if prec == "fp64" else "fp32_vector_TFs"
        d = prof[dom]
        per_launch_ms = d["ms"] / d["launches"]
        if bound == "hbm":
            achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9
            unit = "GB/s"
        else:
            achieved = d["flops"] / (d["ms"] / 1e3) / 1e12
            unit = "TFLOP/s"
        peak = PEAKS[peak_key]
        if dom == "layer" and prec == "fp32" and d["flops"] > 0:
            # FP64 Gram + eigen-solve at the FP64 peak, the rest at the FP32 peak
            f64 = prof["layer_fp64_flops"]
            f32 = d["flops"] - f64
            peak = d["flops"] / (f32 / PEAKS["fp32_vector_TFs"] + f64 / PEAKS["fp64_vector_TFs"])
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": measured_traffic(dom), "kernel_class": dom,
                "launches": d["launches"], "avg_launch_ms": per_launch_ms,
                "algorithmic_flops_per_launch": d["flops"] / d["launches"],
                "fp64_flops_share": (prof["layer_fp64_flops"] / d["flops"]) if dom == "layer" and d["flops"] else None,
                "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
                "share_of_step_time": d["ms"] / ms if ms > 0 else None}
    plain = None
    if not args.no_plain and prec == "fp32":
        plain = plain_fp64_form(circ, chi, rounds, W, K, batched, min(args.plain_shots, circ.n_shots), dev,
                                args.plain_seconds)
        plain["batched_fp32_speedup"] = value / plain["value"]
    cpu = None
    if not args.no_cpu:
        cores = min(os.cpu_count() or 1, 16)
        print(f"# cpu baseline on {cores} cores", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.config, circ, rounds, W, W + K, chi, eps,
                           args.cpu_seconds, cores)
    out = {
        "metric": f"crosstalk rotations/sec (shots x gates) at d={cfg['d']}, chi={chi}",
        "value": value, "unit": "rotations/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 contractions + f64 gram/eigen/norms" if prec == "fp32" else "c128",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: rotated surface code d={cfg['d']} memory-Z, "
                               f"{circ.n} qubits, rounds {W + 1}-{W + K} of {cfg['rounds']}",
                   "shots": circ.n_shots, "chi_max": chi, "rotations_timed": n_rot,
                   "max_bond_after": int(bonds.max()), "mean_bond_after": float(bonds.mean()),
                   "wall_s": wall, "eigen_sweeps": prof["eigen_sweeps"], "schedule": schedule,
                   "class_ms": {c: prof[c]["ms"] for c in classes},
                   "layer_phase_share": ({k: v / sum(phases.values()) for k, v in phases.items()}
                                         if sum(phases.values()) > 0 else None)},
        "roofline": roof,
        "plain_fp64": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

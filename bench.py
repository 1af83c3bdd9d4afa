"""Throughput benchmark of the STN crosstalk step on one MI355X.

Workload: rotated surface code d=5 memory-Z experiment (49 qubits),
ZZ crosstalk after each of the 4 CNOT layers on the 80 nearest-neighbour
pairs (theta ~ U[0.02, 0.10] per coupling) and the 72 next-nearest pairs
(own draw, halved), depolarising p = 1e-3 (Table I ratios), chi_max = 256,
FP32 complex contractions with FP64 Gram, eigen-solve and norms, 1024 shots
batched.  All inputs are seeded and synthetic and are resident in device
memory before the timed region starts.

A step is one pass of the hot path over every shot from the initial state:
stn_reset, syndrome round 1 (Clifford layers and noise on the tableau, 608
crosstalk rotations -- rewrite, bond-2 update, compression and Gram/eigen
truncation -- and 24 ancilla measurements with projection, frame change and
reset), then round 2 up to and including its first crosstalk layer (152
rotations), where the bonds grow from 16 to 64: 760 rotations per shot.  The
circuit has only five rounds and a saturated round takes minutes, so the
steps replay this window rather than walking on through the circuit.
--warmup W steps run untimed, then --steps K steps are timed (HIP events on
the library stream around all K).

Prints one JSON line.  value = (shots x rotations per step x K) / time.
roofline: the kernel class with the largest time in the timed region, its
algorithmic work per step (counted on the device from the realised bond
dimensions in a separate replay of one step: the counters slow the kernels
they count; each truncation eigen-solve of order nn at a fixed 107/8 nn^3
FP64 flops, whatever route ran) over its own launch time in the timed region
(HIP events around each of its launches on the library stream); `executed`
beside it recounts the solves at the flops they executed.  graph: the same step captured
once as a HIP graph and replayed (time per replay, records bit-identical to
the eager step).  plain_fp64: the plain per-shot FP64 GPU form (per-step
kernels, one shot at a time) of the window on the first shots with the
batched records forced, within a time budget, and the largest relative
difference of the batched FP32 probabilities from it.  cpu_baseline: the
FP64 oracle timed on the host cores over a bounded sample of the window.
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
# the machine's CPU share for one GPU: worker pools stay within it whatever the
# host reports
HOST_CPU_SHARE = 16
# autotuner candidates of the bench window: (layer mode, threads per shot, LDS tile)
BENCH_CANDIDATES = ((2, 256, 32), (2, 256, 64), (2, 512, 32), (2, 512, 64))


def kernel_source_hash():
    """sha256 (first 16 hex) of the kernel sources, in a fixed order; a
    stored traffic figure counts only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "linalg.h", "mps.hip", "layer.hip"):
        with open(os.path.join(ROOT, "paper_2605_29514_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class, window):
    """HBM bytes per launch of a kernel class on this window from the
    committed rocprofv3 PMC summary (profiles/traffic_*.json), or None when
    no summary matches or the kernel source changed since the counters were
    taken."""
    import glob
    sha = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as f:
            t = json.load(f)
        if (t.get("kernel_class") == kernel_class and t.get("source_sha256_16") == sha
                and t.get("window") == window):
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


def window_stop(ops, window):
    """End (exclusive) of the op window a step replays from the initial state."""
    rounds = split_rounds(ops)
    if window == "round1":
        return rounds[0][1]
    if window in ("r2l1", "r2l2"):
        r2 = rounds[1][0]
        rot = [i for i in range(r2, rounds[1][1]) if ops[i][0] == "rotate"]
        return rot[0 if window == "r2l1" else 1] + 1
    raise ValueError(window)


WINDOW_TEXT = {
    "r2l1": "syndrome round 1 + round 2 through its first crosstalk layer",
    "r2l2": "syndrome round 1 + round 2 through its second crosstalk layer",
    "round1": "syndrome round 1",
}


def rotations_in(circ_ops, lo, hi):
    return sum(len(o[1]) for o in circ_ops[lo:hi] if o[0] == "rotate")


def records_of(res):
    import torch
    if not res:
        return None, None
    return (torch.cat([r[0] for r in res], dim=1).cpu().numpy(),
            torch.cat([r[1] for r in res], dim=1).cpu().numpy())


# ----------------------------------------------------------------- CPU leg
def _oracle_worker(args):
    """Runs shots of the workload on the FP64 oracle through the window, one
    after the other, timing every rotation, until the time budget is used;
    returns (rotations timed, seconds timed, complete windows)."""
    name, shots, shots_total, stop_op, budget, chi, eps = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    from oracle import stn as ostn
    from paper_2605_29514_amd import workload
    circ, _ = workload.make_config(name, n_shots=shots_total)
    per_window = sum(len(op["paulis"]) for op in circ.ops[:stop_op] if op["op"] == "rotate")
    done, busy, whole = 0, 0.0, 0
    for shot in shots:
        if busy > budget:
            break
        st = ostn.Shot(circ.n, chi, eps)
        start = done
        for op in circ.ops[:stop_op]:
            if busy > budget:
                break
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
                    busy += time.perf_counter() - t0
                    done += 1
                    if busy > budget:
                        break
            elif k == "measure":
                for mj, q in enumerate(op["qubits"]):
                    st.measure(int(q), float(op["u"][shot, mj]), None, bool(op["reset"]))
        whole += done - start == per_window
    return done, busy, whole


def cpu_baseline(name, circ, stop_op, chi, eps, budget, cores):
    """Oracle rotations/s over the window: `cores` worker processes (BLAS 1
    thread each) take shots 0, 1, 2, ... round-robin and time every rotation
    until each has spent `budget` seconds."""
    per = [list(range(w, circ.n_shots, cores)) for w in range(cores)]
    args = [(name, per[w], circ.n_shots, stop_op, budget, chi, eps) for w in range(cores)]
    ctx = mp.get_context("spawn")
    # one BLAS thread per worker: the spawned children read these before
    # numpy starts its thread pool (threadpool_limits in the worker as well)
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    t0 = time.perf_counter()
    try:
        with ctx.Pool(cores) as pool:
            res = pool.map(_oracle_worker, args)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    whole = sum(r[2] for r in res)
    return {"value": done / busy if busy > 0 else 0.0, "unit": "rotations/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} worker processes (FP64 numpy oracle, one BLAS thread each), each running "
                      f"its shots (round-robin from shot 0) through the window from the start and timing "
                      f"every rotation until {budget:.0f} s were spent; {done} rotations in total, {whole} "
                      f"complete windows, slowest worker {busy:.1f} s (wall {wall:.1f} s).  A worker stopped "
                      f"inside a window has timed its cheaper first part, so the rate may overstate the "
                      f"oracle slightly"}


def plain_fp64_form(circ, chi, stop_op, rec, prob, n, dev, budget_s):
    """The plain per-shot FP64 GPU form of the window: per-step kernels, one
    shot at a time, FP64 throughout, on up to the first n shots with the
    batched run's records forced, op by op until budget_s seconds are spent.
    Returns its rotation rate over the rotation ops it ran and the largest
    relative difference of the batched FP32 probabilities from it."""
    import torch
    from paper_2605_29514_amd import stn
    full = np.zeros((n, circ.n_measurements), np.uint8)
    full[:, :rec.shape[1]] = rec[:n]
    ms_total, rot_total, worst, shots_used = 0.0, 0, 0.0, 0
    t_start = time.perf_counter()
    for s in range(n):
        c1 = circ.shot_slice(s, s + 1)
        sim = stn.Simulator(c1.n, 1, chi, "fp64", None, dev, layer_mode=1)
        ops1 = stn.prepare(c1, dev, forced=full[s:s + 1])
        res = []
        for i in range(stop_op):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(sim.stream)
            stn.run_prepared(sim, ops1, i, i + 1, records=res)
            b.record(sim.stream)
            sim.sync()
            if ops1[i][0] == "rotate":
                ms_total += a.elapsed_time(b)
                rot_total += len(ops1[i][1])
                print(f"# plain FP64 form: shot {s + 1}, op {i + 1}/{stop_op}", file=sys.stderr, flush=True)
            if time.perf_counter() - t_start > budget_s:
                break
        if res:
            p64 = torch.cat([x[1] for x in res], dim=1).cpu().numpy()[0]
            worst = max(worst, float(np.max(np.abs(prob[s, :p64.shape[0]] - p64) / p64)))
        shots_used += 1
        del sim
        if time.perf_counter() - t_start > budget_s:
            break
    return {"value": rot_total / (ms_total / 1e3) if ms_total else None, "unit": "rotations/s",
            "shots": shots_used, "timed_rotations": rot_total, "per_step_kernels": True, "precision": "fp64",
            "max_rel_prob_diff_batched_fp32": worst}


def graph_leg(args, circ, chi, prec, eps, dev, ops_stop, tuned, ref_rec, ref_prob, reps=1):
    """Captures stn_reset + the window once on a side stream and replays it;
    returns the time per replay and whether the records and probabilities
    equal the eager step's."""
    import torch
    from paper_2605_29514_amd import stn
    side = torch.cuda.Stream()
    sim = stn.Simulator(circ.n, circ.n_shots, chi, prec, eps, dev, layer_mode=tuned[0],
                        layer_threads=tuned[1], layer_lds=tuned[2], stream=side)
    ops = stn.prepare(circ, dev)[:ops_stop]
    t0 = time.perf_counter()
    graph, res = stn.capture(sim, ops)
    cap_s = time.perf_counter() - t0
    times = []
    same = True
    for _ in range(reps):
        side.wait_stream(torch.cuda.current_stream())
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(side):             # a replay goes to the current stream
            a.record(side)
            graph.replay()
            b.record(side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
        rec, prob = records_of(res)
        same = same and bool(np.array_equal(rec, ref_rec) and np.array_equal(prob, ref_prob))
        print(f"# graph replay {len(times)}: {times[-1]:.1f} ms", file=sys.stderr, flush=True)
    del graph, res, sim
    torch.cuda.synchronize()
    return {"ms_per_replay": float(np.mean(times)), "capture_s": cap_s, "replays": reps,
            "bit_identical_to_eager": same}


# ----------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="d5_nnn_chi256")
    ap.add_argument("--window", default="r2l1", choices=sorted(WINDOW_TEXT))
    ap.add_argument("--shots", type=int, default=None, help="override the shot count (testing only)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-all", action="store_true")
    ap.add_argument("--layer-mode", type=int, default=0, help="0 automatic, 1 per-step kernels, 2 fused")
    ap.add_argument("--layer-threads", type=int, default=0, help="threads per shot of the fused kernel")
    ap.add_argument("--layer-lds", type=int, default=0, help="eigen-solve LDS order of the fused kernel")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the step")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-shot FP64 GPU form (per-step kernels, one shot at a time)")
    ap.add_argument("--plain-shots", type=int, default=4)
    ap.add_argument("--plain-seconds", type=float, default=30.0,
                    help="time budget of the plain FP64 form")
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
        print("bench.py measures one GPU: this build has no multi-GPU path (shots would shard "
              "across GPUs with one final gather of records, log P and truncation errors).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_29514_amd import stn, workload

    cfg = dict(workload.CONFIGS[args.config])
    over = {} if args.shots is None else {"n_shots": args.shots}
    circ, opts = workload.make_config(args.config, **over)
    chi, prec = opts["chi_max"], opts["precision"]
    eps = stn.DEFAULT_EPS[stn.STN_FP64 if prec == "fp64" else stn.STN_FP32]
    dev = "cuda:0"
    print(f"# building inputs: {args.config} shots={circ.n_shots} window {args.window}", file=sys.stderr, flush=True)
    sim = stn.Simulator(circ.n, circ.n_shots, chi, prec, eps, dev, layer_mode=args.layer_mode,
                        layer_threads=args.layer_threads, layer_lds=args.layer_lds)
    ops = stn.prepare(circ, dev)
    stop = window_stop(ops, args.window)
    rot_per_shot = rotations_in(ops, 0, stop)
    W, K = max(0, args.warmup), max(1, args.steps)
    chosen = (args.layer_mode or 2, args.layer_threads or 128, args.layer_lds)
    schedule = {"layer_mode": chosen[0], "layer_threads": chosen[1], "layer_lds": chosen[2], "tuned": False}
    if args.layer_mode == 0 and args.layer_threads == 0 and not args.no_tune:
        from paper_2605_29514_amd import tune
        key = tune.problem_key(torch.cuda.get_device_name(0), circ.n, circ.n_shots, chi, prec, args.config)
        # the fused shapes with 256 or 512 threads per shot: at this shot
        # count the per-step schedule is slower by orders of magnitude, and
        # 64 / 128 threads by about 2x on this window (measured); each
        # candidate runs one whole step
        t = tune.autotune(sim, ops, stop, key=f"{key}|window {args.window}", candidates=BENCH_CANDIDATES,
                          log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        chosen = tuple(t["choice"])
        schedule = {"layer_mode": chosen[0], "layer_threads": chosen[1], "layer_lds": chosen[2], "tuned": True,
                    "cached": t["cached"], "candidates_ms": t["ms"]}
        print(f"# autotuned schedule {chosen}", file=sys.stderr, flush=True)
    else:
        stn_mode = args.layer_mode
        if stn_mode:
            sim.set_layer_mode(stn_mode)
    torch.cuda.synchronize()
    for w in range(W):
        t = time.perf_counter()
        sim.reset()
        stn.run_prepared(sim, ops, 0, stop)
        sim.sync()
        print(f"# warmup step {w + 1}: {time.perf_counter() - t:.2f} s, max bond {int(sim.bonds().max())}",
              file=sys.stderr, flush=True)
    # Timed region: launch events per kernel class only.  The device work
    # counters (atomics from every block, per-phase clocks) slow the kernels
    # they count, so the work per step comes from a counted replay below.
    prof_classes = None if args.profile_all else ["eigen", "qr", "gemm", "gram", "layer", "expect"]
    sim.profile(prof_classes, counters=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    last = []
    for k in range(K):
        last = []
        sim.reset()
        stn.run_prepared(sim, ops, 0, stop, records=last)
        e = torch.cuda.Event()
        e.record(sim.stream)
        # progress (host side only; the GPU timeline is what ev0 / ev1 measure)
        while not e.query():
            time.sleep(0.02)
        print(f"# timed step {k + 1} done at {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    sim.sync()
    prof = sim.profile_read()
    bonds = sim.bonds()
    rec, prob = records_of(last)
    n_rot = rot_per_shot * circ.n_shots * K
    value = n_rot / (ms / 1e3)
    # counted replay of one step (deterministic: same launches, same bonds):
    # algorithmic work per class, phase shares and branch counts
    sim.profile(prof_classes, counters=True)
    sim.reset()
    stn.run_prepared(sim, ops, 0, stop)
    sim.sync()
    work = sim.profile_read()
    phases = sim.profile_phases()
    paths = sim.profile_paths()
    sim.profile([])
    print("# counted replay done", file=sys.stderr, flush=True)
    for c in stn.K_CLASSES:
        prof[c]["flops"], prof[c]["bytes"] = work[c]["flops"] * K, work[c]["bytes"] * K
        if work[c]["launches"] * K != prof[c]["launches"]:
            print(f"# warning: class {c}: {prof[c]['launches']} timed launches, {work[c]['launches']} per "
                  f"counted step", file=sys.stderr, flush=True)
    prof["layer_fp64_flops"], prof["eigen_sweeps"] = work["layer_fp64_flops"] * K, work["eigen_sweeps"]
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
        if dom in ("layer", "expect") and prec == "fp32" and d["flops"] > 0 and dom == "layer":
            # FP64 Gram + eigen-solve at the FP64 peak, the rest at the FP32 peak
            f64 = prof["layer_fp64_flops"]
            f32 = d["flops"] - f64
            peak = d["flops"] / (f32 / PEAKS["fp32_vector_TFs"] + f64 / PEAKS["fp64_vector_TFs"])
        executed = None
        if dom == "layer" and d["flops"] > 0:
            # the same work with the eigen-solves at their executed flop count
            # (route and sweeps as run) instead of the fixed nominal cost
            dn = (paths.get("eig_nominal_flops", 0.0) - paths.get("eig_exec_flops", 0.0)) * K
            fx = d["flops"] - dn
            f64x = prof["layer_fp64_flops"] - dn
            px = fx / ((fx - f64x) / PEAKS["fp32_vector_TFs"] + f64x / PEAKS["fp64_vector_TFs"])
            ax = fx / (d["ms"] / 1e3) / 1e12
            executed = {"flops_per_launch": fx / d["launches"], "achieved": ax, "peak": px, "frac": ax / px,
                        "eigen_nominal_flops_per_launch": paths.get("eig_nominal_flops", 0.0) * K / d["launches"],
                        "eigen_executed_flops_per_launch": paths.get("eig_exec_flops", 0.0) * K / d["launches"]}
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": measured_traffic(dom, args.window), "kernel_class": dom,
                "launches": d["launches"], "avg_launch_ms": per_launch_ms,
                "algorithmic_flops_per_launch": d["flops"] / d["launches"],
                "fp64_flops_share": (prof["layer_fp64_flops"] / d["flops"]) if dom == "layer" and d["flops"] else None,
                "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
                "share_of_step_time": d["ms"] / ms if ms > 0 else None,
                "executed": executed}
    graph = None
    if not args.no_graph:
        del sim
        torch.cuda.synchronize()
        graph = graph_leg(args, circ, chi, prec, eps, dev, stop, chosen, rec, prob)
    plain = None
    if not args.no_plain and prec == "fp32":
        plain = plain_fp64_form(circ, chi, stop, rec, prob, min(args.plain_shots, circ.n_shots), dev,
                                args.plain_seconds)
        if plain["value"]:
            plain["batched_fp32_speedup"] = value / plain["value"]
    cpu = None
    if not args.no_cpu:
        try:
            avail = len(os.sched_getaffinity(0))
        except AttributeError:
            avail = os.cpu_count() or 1
        cores = max(1, min(avail, HOST_CPU_SHARE))
        print(f"# cpu baseline on {cores} cores ({avail} available to this process)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.config, circ, stop, chi, eps, args.cpu_seconds, cores)
    ph_tot = sum(phases.values())
    out = {
        "metric": f"crosstalk rotations/sec (shots x gates) at d={cfg['d']}, chi={chi}",
        "value": value, "unit": "rotations/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 contractions + f64 gram/eigen/norms" if prec == "fp32" else "c128",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: rotated surface code d={cfg['d']} memory-Z, {circ.n} qubits, "
                               f"{circ.n_shots} shots; step = stn_reset + {WINDOW_TEXT[args.window]} "
                               f"({rot_per_shot} rotations per shot); bonds after the step: max "
                               f"{int(bonds.max())}, mean {float(bonds.mean()):.1f}",
                   "window": args.window, "shots": circ.n_shots, "chi_max": chi,
                   "rotations_per_step": rot_per_shot * circ.n_shots,
                   "max_bond_after": int(bonds.max()), "mean_bond_after": float(bonds.mean()),
                   "fp32_cut": eps, "wall_s": wall, "eigen_sweeps_per_step": prof["eigen_sweeps"],
                   "schedule": schedule,
                   "class_ms": {c: prof[c]["ms"] for c in classes},
                   "layer_phase_share": ({k: v / ph_tot for k, v in phases.items()} if ph_tot > 0 else None),
                   "layer_branches_per_step": paths},
        "roofline": roof,
        "graph": graph,
        "plain_fp64": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

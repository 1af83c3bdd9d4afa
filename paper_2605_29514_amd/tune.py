"""Launch-shape autotuner for the rotation layers.

The library offers two schedules for a chunk of rotations -- per-step
kernels with many blocks per product, or the fused per-shot layer kernel --
four block sizes for the fused kernel (64, 128, 256, 512 threads per shot) and
two LDS tiles for its FP32-path eigen-solve (factors of order up to 32 or up
to 64 held in LDS; the larger tile leaves room for fewer blocks per compute
unit).
Which one is fastest depends on the shot count, the bond dimensions the
circuit reaches and the precision, so it is measured, not guessed: each
candidate runs the same window of the real workload on the real Simulator,
timed with HIP events on the Simulator's stream, and the fastest is kept.
The window starts either at the initial state (stn_reset before and after,
no second workspace) or at a later point of the circuit -- the bonds of a
saturated round differ from those of the first one -- reached once and
restored for every candidate from a checkpoint (stn_checkpoint_save /
stn_checkpoint_load).  Results are cached per (device, problem) key in a
JSON file.

All candidates compute the same results up to rounding order and, where
the LDS tile changes a step's route, up to directions of weight below the
truncation cut (the GPU parity tests run every one of them against the
oracle).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

# (layer mode, threads per shot, eigen-solve LDS order): 1 = per-step
# kernels, 2 = fused kernel; LDS order 0 = chosen by the library (from chi_max
# and the threads per shot)
CANDIDATES: Tuple[Tuple[int, int, int], ...] = ((1, 0, 0), (2, 64, 0), (2, 128, 0), (2, 128, 64),
                                                (2, 256, 32), (2, 256, 64), (2, 512, 32), (2, 512, 64))
# the fused-kernel shapes alone (many shots: the per-step schedule is far slower)
FUSED: Tuple[Tuple[int, int, int], ...] = tuple(c for c in CANDIDATES if c[0] == 2)


def cache_path() -> str:
    return os.environ.get("STN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2605_29514_amd", "tune.json"))


def problem_key(device_name: str, n: int, shots: int, chi: int, precision: str, workload: str) -> str:
    return f"{device_name}|n={n}|S={shots}|chi={chi}|{precision}|{workload}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(timings: Dict[Tuple[int, ...], float]) -> Tuple[int, ...]:
    """Fastest candidate; ties go to the earlier entry of CANDIDATES."""
    order = {c: i for i, c in enumerate(CANDIDATES)}
    return min(timings, key=lambda c: (timings[c], order.get(c, len(order))))


def apply(sim, choice: Sequence[int]) -> None:
    mode, threads = int(choice[0]), int(choice[1])
    sim.set_layer_mode(mode)
    if threads:
        sim.set_layer_threads(threads)
    sim.set_layer_lds(int(choice[2]) if len(choice) > 2 else 0)


def autotune(sim, ops, stop: int, *, start: int = 0, key: Optional[str] = None, candidates: Iterable = CANDIDATES,
             use_cache: bool = True, log=None) -> dict:
    """Times ops[start:stop] for every candidate on `sim` (ops[:start] run
    once beforehand, the state there restored for each candidate from a
    checkpoint), leaves `sim` reset to the initial state with the fastest
    candidate applied, and returns {"choice", "ms", "cached"}."""
    import torch
    from . import stn
    if use_cache and key:
        hit = load_cache().get(key)
        if hit and tuple(hit.get("choice", ())) in set(map(tuple, candidates)):
            apply(sim, hit["choice"])
            sim.reset()
            return {"choice": tuple(hit["choice"]), "ms": hit.get("ms"), "cached": True}
    ck = None
    if start > 0:
        sim.reset()
        stn.run_prepared(sim, ops, 0, start)
        sim.sync()
        ck = sim.checkpoint_save()
    timings: Dict[Tuple[int, ...], float] = {}
    for cand in candidates:
        cand = tuple(cand)
        apply(sim, cand)
        if ck is None:
            sim.reset()
        else:
            sim.checkpoint_load(ck)
        sim.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(sim.stream)
        stn.run_prepared(sim, ops, start, stop)
        b.record(sim.stream)
        sim.sync()
        timings[cand] = a.elapsed_time(b)
        if log:
            log(f"autotune {cand}: {timings[cand]:.1f} ms")
    del ck
    best = pick(timings)
    apply(sim, best)
    sim.reset()
    sim.sync()
    ms = {"/".join(map(str, c)): v for c, v in timings.items()}
    if key:
        store_cache(key, {"choice": list(best), "ms": ms})
    return {"choice": best, "ms": ms, "cached": False}


def layers_stop(ops, layers: int = 2, start: int = 0) -> int:
    """Index just past the `layers`-th rotation op of a prepared op list at or
    after `start` (the end of an autotuning window of crosstalk layers)."""
    seen = 0
    for i, op in enumerate(ops):
        if i < start:
            continue
        if op[0] == "rotate":
            seen += 1
            if seen == layers:
                return i + 1
    return len(ops)

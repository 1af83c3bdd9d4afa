"""Host-side parts of bench.py: the replayed window and the CPU baseline leg
(the FP64 oracle timed in worker processes with one BLAS thread each)."""
import os

import bench
from paper_2605_29514_amd import workload


def _ops(circ):
    # the (kind, _, reset) shape of prepared ops that the window logic reads
    return [(op["op"], None, op.get("reset")) for op in circ.ops]


def test_window_r2l1_ends_after_first_layer_of_round_two():
    circ, _ = workload.make_config("d3_nn_chi64")
    ops = _ops(circ)
    rounds = bench.split_rounds(ops)
    stop = bench.window_stop(ops, "r2l1")
    assert ops[stop - 1][0] == "rotate"
    assert rounds[1][0] < stop < rounds[1][1]
    # no rotation of round 2 before the one that closes the window
    assert not any(ops[i][0] == "rotate" for i in range(rounds[1][0], stop - 1))
    assert bench.window_stop(ops, "round1") == rounds[0][1]


def test_cpu_baseline_counts_whole_windows_and_restores_env():
    circ, _ = workload.make_config("d3_nn_chi64", n_shots=4)
    stop = bench.window_stop(_ops(circ), "r2l1")
    before = os.environ.get("OMP_NUM_THREADS")
    r = bench.cpu_baseline("d3_nn_chi64", circ, stop, 64, 1e-12, 1.0, 2)
    assert os.environ.get("OMP_NUM_THREADS") == before
    assert r["kind"] == "oracle" and r["cores"] == 2 and r["unit"] == "rotations/s"
    assert r["value"] > 0
    per_window = sum(len(op["paulis"]) for op in circ.ops[:stop] if op["op"] == "rotate")
    # the d=3 window takes well under a second on one core: each worker
    # finishes at least its first window
    assert "complete windows" in r["sample"]
    whole = int(r["sample"].split(" complete windows")[0].rsplit(" ", 1)[1])
    done = int(r["sample"].split(" rotations in total")[0].rsplit(" ", 1)[1])
    assert whole >= 2 and done >= whole * per_window

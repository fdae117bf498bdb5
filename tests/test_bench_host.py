"""bench.py's host-side bookkeeping, without a GPU."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_traffic_only_for_the_recorded_workload():
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_sp2_step_counters.json")))
    for prec, r in rec.items():
        got = bench.counter_traffic(prec, dict(r["match"]))
        # None only if the kernel sources changed after the counters were taken
        assert got in (None, r["traffic_bytes_per_launch"])
        other = dict(r["match"], tau=1e-3)
        assert bench.counter_traffic(prec, other) is None
        assert bench.counter_traffic(prec, dict(r["match"], sum_s3=r["match"]["sum_s3"] + 1)) is None
    assert bench.counter_traffic("no-such-precision", {}) is None
    for prec, r in rec.items():
        other = "k_sp2_step" if r["kernel"] == "k_sp2_wide" else "k_sp2_wide"
        assert bench.counter_traffic(prec, dict(r["match"]), other) is None

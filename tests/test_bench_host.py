"""bench.py's host-side bookkeeping, without a GPU."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_traffic_only_for_the_recorded_workload():
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_sp2_step_counters.json")))
    kernels = {r["kernel"] for r in rec.values()}
    for key, r in rec.items():
        prec, kern = key.split("/")
        assert (r["precision"], r["kernel"]) == (prec, kern)
        got = bench.counter_traffic(prec, dict(r["match"]), kern)
        # None only if the kernel sources changed after the counters were taken
        assert got in (None, r["traffic_bytes_per_launch"])
        other = dict(r["match"], tau=1e-3)
        assert bench.counter_traffic(prec, other, kern) is None
        assert bench.counter_traffic(prec, dict(r["match"], sum_s3=r["match"]["sum_s3"] + 1), kern) is None
        for k in kernels - {kern}:
            if f"{prec}/{k}" not in rec:
                assert bench.counter_traffic(prec, dict(r["match"]), k) is None
    assert bench.counter_traffic("no-such-precision", {}, "k_sp2_step") is None

"""Write the stored expectations of the full-size G-SP2 parity test.

Calls only the FP64 oracle and the seeded input generators.  Workload:
3,500 water molecules (21,000 orbitals), 128 uneven spatial parts (cores
U[60, 300] orbitals), graph from the distance-based stand-in for the
previous P thresholded at tau = 1e-5 (the oracle cannot afford the dense
previous P at this size).  Stores the oracle's branch sequence, traces and
idempotency errors, and per part its size, core size, core trace and the
Frobenius norm of its core columns.

    python tests/golden/make_full_size_golden.py        (about 15 min on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth.locality import surrogate_prev_density  # noqa: E402
from synth.partition import uneven_spatial_partition  # noqa: E402
from synth.water import make_water  # noqa: E402

SPEC = {"n_mol": 3500, "seed": 0, "n_parts": 128, "core_lo": 60.0, "core_hi": 300.0, "tau": 1e-5,
        "q_floor": 5e-6, "max_iter": 60}
OUT = os.path.join(HERE, "gsp2_water3500_tau1e-5.json")


def main():
    t0 = time.time()
    s = make_water(SPEC["n_mol"], SPEC["seed"])
    part = uneven_spatial_partition(s, SPEC["n_parts"], SPEC["core_lo"], SPEC["core_hi"], seed=SPEC["seed"])
    Q = surrogate_prev_density(s, SPEC["q_floor"])
    res = oracle.gsp2(s.H, Q, SPEC["tau"], part, SPEC["n_parts"], s.n_occ, max_iter=SPEC["max_iter"])
    r = res.sp2
    per_part = []
    for k in range(SPEC["n_parts"]):
        blk = res.core_columns[k]
        c = len(res.cores[k])
        per_part.append({"s": int(len(res.index[k])), "c": int(c),
                         "core_trace": float(np.trace(blk[:c, :c])),
                         "fro": float(np.linalg.norm(blk))})
    out = {
        "source": "FP64 oracle (oracle.gsp2), written by tests/golden/make_full_size_golden.py",
        "spec": SPEC, "n": s.n, "n_occ": s.n_occ, "eps": list(res.eps),
        "status": r.status, "converged": r.converged, "n_products": r.n_products,
        "alphas": [int(a) for a in r.alphas], "traces": [float(x) for x in r.traces],
        "errors": [float(x) for x in r.errors], "parts": per_part,
        "fro_total": float(np.sqrt(sum(p["fro"] ** 2 for p in per_part))),
        "seconds": round(time.time() - t0, 1),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}: {r.n_products} products, {out['seconds']} s")


if __name__ == "__main__":
    main()

"""Write the stored expectations of the full-size G-SP2 parity tests.

Calls only the FP64 oracle and the seeded input generators (synth/).
Workload: 3,500 water molecules (21,000 orbitals), 128 uneven spatial parts
(cores U[60, 300] orbitals), tau = 1e-5, with the graph taken from one of
two previous density matrices:

  dense    the oracle's own FP64 dense SP2 P of the same H (Methods, "Graph
           Theory": the graph comes from a P computed by ordinary SP2).  This
           is the benchmark's workload.  About 25 min for the dense P and
           20 min for G-SP2 on 8 cores, 20 GB of memory.
  standin  the distance-based stand-in for the previous P (about 15 min).

For each it stores the oracle's branch sequence, traces and idempotency
errors, the graph's size and digest, and per part its size, core size, core
trace, Frobenius norm of its core columns, the SHA-256 of its index list and
a Gaussian sketch S B R of its core-column block B (rows in ascending global
order, core columns ascending; probes from synth.sketch), plus the full
index lists of three parts (smallest, median, largest), which the tests
recompute with the oracle.  For the dense graph it also stores the dense
run's branch sequence, a sketch of the dense P and every entry whose
magnitude lies within 1e-7 relative of tau (pairs whose side of the
threshold a rounding-level difference could change).

    python tests/golden/make_full_size_golden.py [dense|standin|both]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import sketch  # noqa: E402
from synth.locality import surrogate_prev_density  # noqa: E402
from synth.partition import uneven_spatial_partition  # noqa: E402
from synth.water import make_water  # noqa: E402

SPEC = {"n_mol": 3500, "seed": 0, "n_parts": 128, "core_lo": 60.0, "core_hi": 300.0, "tau": 1e-5,
        "q_floor": 5e-6, "max_iter": 60}
OUT = {"standin": os.path.join(HERE, "gsp2_water3500_tau1e-5"),
       "dense": os.path.join(HERE, "gsp2_water3500_densep_tau1e-5")}


def log(msg):
    print(f"[golden] {msg}", flush=True)


def graph_digest(adj: sp.csr_matrix) -> str:
    """SHA-256 of the symmetric adjacency in canonical CSR form (sorted columns)."""
    a = sp.csr_matrix(adj, dtype=np.int8)
    a.sort_indices()
    h = hashlib.sha256()
    h.update(np.asarray(a.indptr, dtype="<i8").tobytes())
    h.update(np.asarray(a.indices, dtype="<i4").tobytes())
    return h.hexdigest()


def index_digest(idx) -> str:
    return hashlib.sha256(np.asarray(idx, dtype="<i4").tobytes()).hexdigest()


def part_sketch(k, index, core_block):
    """S B R of a part's core columns, rows in ascending global order."""
    order = np.argsort(index, kind="stable")
    B = core_block[order, :]
    S, R = sketch.probes(k, B.shape[0], B.shape[1])
    return S @ B @ R


def run_gsp2(s, part, adj, label):
    t = time.time()
    res = oracle.gsp2(s.H, None, SPEC["tau"], part, SPEC["n_parts"], s.n_occ, max_iter=SPEC["max_iter"],
                      adjacency=adj)
    log(f"{label}: oracle G-SP2 {res.sp2.n_products} products, {time.time() - t:.0f} s")
    return res


def summarise(res, adj, label, extra, arrays):
    r = res.sp2
    per_part, sketches = [], []
    for k in range(SPEC["n_parts"]):
        blk = res.core_columns[k]
        c = len(res.cores[k])
        per_part.append({"s": int(len(res.index[k])), "c": int(c),
                         "core_trace": float(np.trace(blk[:c, :c])),
                         "fro": float(np.linalg.norm(blk)),
                         "idx_sha256": index_digest(res.index[k])})
        sketches.append(part_sketch(k, res.index[k], blk))
    sizes = np.array([p["s"] for p in per_part])
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    out = {
        "source": f"FP64 oracle (oracle.gsp2), written by tests/golden/make_full_size_golden.py ({label})",
        "spec": SPEC, "graph_source": label, "n": int(res.n), "n_occ": float(extra.pop("n_occ")),
        "eps": list(res.eps), "status": r.status, "converged": r.converged, "n_products": r.n_products,
        "alphas": [int(a) for a in r.alphas], "traces": [float(x) for x in r.traces],
        "errors": [float(x) for x in r.errors], "parts": per_part,
        "fro_total": float(np.sqrt(sum(p["fro"] ** 2 for p in per_part))),
        "graph": {"nnz_sym": int(adj.nnz), "sha256": graph_digest(adj)},
        "sketch": {"m": sketch.SKETCH_M, "r": sketch.SKETCH_R, "seed": sketch.SKETCH_SEED,
                   "rows": "ascending global id", "cols": "core vertices ascending"},
        "sample_parts": pick,
    }
    out.update(extra)
    arrays = dict(arrays)
    arrays["part_sketch"] = np.stack(sketches)
    for k in pick:
        arrays[f"index_{k}"] = np.asarray(res.index[k], dtype=np.int32)
    return out, arrays


def write(label, out, arrays, t0):
    out["seconds"] = round(time.time() - t0, 1)
    with open(OUT[label] + ".json", "w") as f:
        json.dump(out, f, indent=1)
    np.savez_compressed(OUT[label] + ".npz", **arrays)
    log(f"wrote {OUT[label]}.json/.npz: {out['n_products']} products, {out['seconds']} s")


def standin(s, part):
    t0 = time.time()
    Q = surrogate_prev_density(s, SPEC["q_floor"])
    adj = oracle.threshold_graph(Q, SPEC["tau"])
    res = run_gsp2(s, part, adj, "standin")
    out, arrays = summarise(res, adj, "standin", {"n_occ": s.n_occ}, {})
    write("standin", out, arrays, t0)


def dense(s, part):
    t0 = time.time()
    tau = SPEC["tau"]
    P, dres = oracle.dense_sp2(s.H, s.n_occ, max_iter=SPEC["max_iter"])
    log(f"dense: oracle dense SP2 {dres.n_products} products ({dres.status}), {time.time() - t0:.0f} s")
    S, R = sketch.probes(-1, s.n, s.n)
    dense_sketch = S @ P @ R
    absP = np.abs(P)
    np.fill_diagonal(absP, 0.0)
    near = np.argwhere(np.abs(absP - tau) <= 1e-7 * tau)
    near_list = [[int(u), int(v), float(P[u, v])] for u, v in near]
    # entries at or below tau / 2 cannot be edges; dropping them first is exact
    Pf = sp.csr_matrix(np.where(absP > 0.5 * tau, P, 0.0))
    del absP
    adj = oracle.threshold_graph(Pf, tau)
    del Pf
    tr = float(np.trace(P))
    idem = float(np.linalg.norm(P @ P - P) / np.linalg.norm(P))
    del P
    log(f"dense: graph nnz {adj.nnz}, {len(near_list)} entries within 1e-7 relative of tau")
    res = run_gsp2(s, part, adj, "dense")
    extra = {"n_occ": s.n_occ,
             "dense_run": {"n_products": dres.n_products, "status": dres.status,
                           "alphas": [int(a) for a in dres.alphas], "traces": [float(x) for x in dres.traces],
                           "errors": [float(x) for x in dres.errors], "trace_P": tr, "idempotency_rel": idem},
             "near_tau": near_list}
    out, arrays = summarise(res, adj, "dense", extra, {"dense_sketch": dense_sketch})
    write("dense", out, arrays, t0)


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "both"
    s = make_water(SPEC["n_mol"], SPEC["seed"])
    part = uneven_spatial_partition(s, SPEC["n_parts"], SPEC["core_lo"], SPEC["core_hi"], seed=SPEC["seed"])
    if which in ("dense", "both"):
        dense(s, part)
    if which in ("standin", "both"):
        standin(s, part)


if __name__ == "__main__":
    main()

"""Helpers of the full-size GPU tests (3,500 water molecules, 21,000
orbitals, 128 uneven parts, tau = 1e-5): the stored oracle expectations, the
GPU's FP64 regular-SP2 previous P, and part-by-part comparisons.

Every expected value comes from tests/golden/, written by
tests/golden/make_full_size_golden.py from the FP64 oracle alone; the
oracle's recomputation of sampled parts below takes its index lists from
those files too, never from the GPU."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import scipy.sparse as sp

import oracle
from synth import sketch

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def load_golden(stem: str):
    with open(os.path.join(GOLDEN, stem + ".json")) as f:
        gold = json.load(f)
    arrays = dict(np.load(os.path.join(GOLDEN, stem + ".npz")))
    return gold, arrays


def graph_digest(adj_ptr, adj_col, n) -> tuple[str, int]:
    """SHA-256 of the undirected graph (union of both orientations of the
    directed adjacency) in canonical CSR form, and its entry count; the
    golden script hashes the oracle's threshold graph the same way."""
    A = sp.csr_matrix((np.ones(len(adj_col), dtype=np.int8), adj_col, adj_ptr), shape=(n, n))
    A = ((A + A.T) > 0).astype(np.int8).tocsr()
    A.sort_indices()
    h = hashlib.sha256()
    h.update(np.asarray(A.indptr, dtype="<i8").tobytes())
    h.update(np.asarray(A.indices, dtype="<i4").tobytes())
    return h.hexdigest(), int(A.nnz)


def index_digest(idx) -> str:
    return hashlib.sha256(np.asarray(idx, dtype="<i4").tobytes()).hexdigest()


def fp64_previous_p(g, torch, Hd, n, n_occ, stream):
    """Regular SP2 of the whole H (one part) on the GPU with FP64 products:
    the previous P whose threshold is the graph, as a device CSR (the one-part
    plan stores every column in full, rows ascending), and its run info."""
    part = np.zeros(n, dtype=np.int32)
    with torch.cuda.stream(stream):
        with g.gsp2_plan_create(Hd, 0.0, part, 1, stream=stream) as plan:
            P = torch.empty(n * n, dtype=torch.float64, device="cuda")
            run = g.gsp2_density(plan, Hd, n_occ, P, precision="fp64")
            torch.cuda.synchronize()
    col_ptr = torch.arange(0, n * n + 1, n, dtype=torch.int64, device="cuda")
    row_idx = torch.arange(n, dtype=torch.int32, device="cuda").repeat(n)
    return g.DeviceCSR(n, col_ptr, row_idx, P), run


def dense_sketch(torch, P_dev, n):
    """S P R of the dense previous P (probes of key -1), on the GPU in FP64."""
    S, R = sketch.probes(-1, n, n)
    Pm = P_dev.view(n, n)                  # column-major P: its transpose, equal for this symmetric iterate
    St = torch.as_tensor(S, device="cuda")
    Rt = torch.as_tensor(R, device="cuda")
    return (St @ (Pm.T @ Rt)).cpu().numpy()


def core_block(vals, col_ptr, core, s):
    """A part's core columns from P's values (CSC in the plan's pattern):
    rows in ascending global order, core columns ascending."""
    starts = col_ptr[np.asarray(core)]
    return vals[starts[None, :] + np.arange(s)[:, None]].astype(np.float64)


def part_errors(gold, arrays, vals, col_ptr, part):
    """Relative sketch error of every part's core columns against the stored
    oracle sketches: ||S (B_gpu - B_oracle) R|| / ||S B_oracle R||."""
    errs = []
    for k, p in enumerate(gold["parts"]):
        core = np.flatnonzero(part == k)
        B = core_block(vals, col_ptr, core, p["s"])
        S, R = sketch.probes(k, p["s"], p["c"])
        want = arrays["part_sketch"][k]
        errs.append(float(np.linalg.norm(S @ B @ R - want) / np.linalg.norm(want)))
    return np.array(errs)


def oracle_sampled_parts(gold, arrays, system, alphas):
    """The oracle recomputes the sampled parts by replaying `alphas` on their
    stored index lists: {k: (index in local order, core columns)}."""
    emin, emax = oracle.gershgorin_bounds(system.H)
    ks = gold["sample_parts"]
    idx = [arrays[f"index_{k}"] for k in ks]
    X0 = [oracle.initial_guess(system.H[ix][:, ix].toarray(), emin, emax) for ix in idx]
    cores = [gold["parts"][k]["c"] for k in ks]
    res = oracle.sp2_blocks(X0, cores, system.n_occ, alpha_seq=alphas, trace_tol=1e30)
    return {k: (ix, X[:, :c]) for k, ix, X, c in zip(ks, idx, res.blocks, cores)}


def sampled_errors(samples, vals, col_ptr, part):
    """Element-by-element relative Frobenius error of the sampled parts."""
    out = {}
    for k, (ix, ref) in samples.items():
        core = np.flatnonzero(part == k)
        order = np.argsort(ix, kind="stable")
        B = core_block(vals, col_ptr, core, len(ix))
        want = ref[order, :]
        out[k] = float(np.linalg.norm(B - want) / np.linalg.norm(want))
    return out

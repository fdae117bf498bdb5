"""Helpers for the GPU tests: run the library through the C ABI and bring
its P back as a scipy matrix."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import paper_1801_10016_amd as g


def run_gsp2(H, P_prev, tau, part, n_parts, n_occ, h_dtype=None, p_dtype=None, tile16=0, tune=None, **kw):
    """One plan and one gsp2_density; tile16 fixes the 16-bit tile edge, tune
    (a precision) runs the tile autotuner first and stores its record in
    run["tune"]."""
    import torch
    Hd = g.csr_to_device(H, dtype=h_dtype or torch.float64)
    Pd = g.csr_to_device(sp.csr_matrix(P_prev), dtype=p_dtype or torch.float64)
    with g.gsp2_plan_create(Pd, tau, part, n_parts, tile16=tile16) as plan:
        rec = g.gsp2_plan_tune(plan, Hd, n_occ, tune, n_products=4) if tune else None
        info, cs, ss = g.gsp2_plan_query(plan)
        col_ptr, row_idx = g.gsp2_plan_pattern(plan)
        p64 = kw.get("precision") == "fp64"
        P_val = torch.full((info["nnz_P"],), float("nan"), dtype=torch.float64 if p64 else torch.float32,
                           device="cuda")
        run = g.gsp2_density(plan, Hd, n_occ, P_val, **kw)
        torch.cuda.synchronize()
        if rec is not None:
            run["tune"] = rec
        vals = P_val.cpu().numpy()
        index = [g.gsp2_plan_part_index(plan, k) for k in range(n_parts)]
    P = sp.csc_matrix((vals.astype(np.float64), row_idx, col_ptr), shape=(H.shape[0], H.shape[0]))
    return P, run, info, index, vals


def rel_fro(a, b) -> float:
    a = a.toarray() if sp.issparse(a) else a
    b = b.toarray() if sp.issparse(b) else b
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))

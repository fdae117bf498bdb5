"""gsp2_density_noalloc (per-run buffers in the library's static device
scratch, no allocation) against gsp2_density (buffers in the plan's
workspace), through the C ABI: the same kernels on the same inputs, so the
two give the same bits.  Two calls in a row, the second on a smaller plan,
then other precisions, and a plan too large for the scratch."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth.partition import uneven_spatial_partition
from tests import _pins as pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(n_mol, seed, n_parts, tau, **kw):
    import torch

    import paper_1801_10016_amd as g
    s = pins.water(n_mol, seed)
    Pp = pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    part = uneven_spatial_partition(s, n_parts, seed=0)
    Hd = g.csr_to_device(s.H)
    Pd = g.csr_to_device(sp.csr_matrix(Pp))
    dt = torch.float64 if kw.get("precision") == "fp64" else torch.float32
    print(f"noalloc: N={s.n} parts={n_parts} tau={tau} {kw}", flush=True)
    with g.gsp2_plan_create(Pd, tau, part, n_parts) as plan:
        info, _, _ = g.gsp2_plan_query(plan)
        col_ptr, row_idx = g.gsp2_plan_pattern(plan)
        P1 = torch.full((info["nnz_P"],), float("nan"), dtype=dt, device="cuda")
        P2 = torch.full((info["nnz_P"],), float("nan"), dtype=dt, device="cuda")
        r1 = g.gsp2_density(plan, Hd, s.n_occ, P1, **kw)
        r2 = g.gsp2_density_noalloc(plan, Hd, s.n_occ, P2, **kw)
        torch.cuda.synchronize()
        v1, v2 = P1.cpu().numpy(), P2.cpu().numpy()
    P = sp.csc_matrix((v2.astype(np.float64), row_idx, col_ptr), shape=(s.n, s.n))
    return s, Pp, part, P, v1, v2, r1, r2


def _same(v1, v2, r1, r2):
    assert np.isfinite(v2).all()
    assert np.array_equal(v1, v2)
    for key in ("status", "n_products", "n_alpha", "result_iterate", "alpha"):
        assert r1[key] == r2[key], key
    for key in ("traces", "errors"):                 # slots a run leaves unwritten hold NaN
        assert np.array_equal(np.array(r1[key]), np.array(r2[key]), equal_nan=True), key


def test_noalloc_equals_density_two_calls():
    from tests._gpu import rel_fro
    for n_mol, seed, n_parts, tau in ((64, 0, 8, 1e-5), (24, 1, 3, 1e-3)):
        s, Pp, part, P, v1, v2, r1, r2 = _both(n_mol, seed, n_parts, tau)
        _same(v1, v2, r1, r2)
        ref = oracle.gsp2(s.H, Pp, tau, part, n_parts, s.n_occ)
        err = rel_fro(P, ref.csc())
        print(f"  {r2['n_products']} products, rel_err vs oracle {err:.2e}", flush=True)
        assert r2["status"] == 0 and err <= 1e-5


@pytest.mark.parametrize("kw", [{"precision": "fp64"}, {"precision": "fp16", "refine": 2},
                                {"precision": "bf16", "refine": 2, "refine_precision": "fp16x3"},
                                {"alpha_seq": [1, -1, 1, -1, -1], "trace_tol": 1e9, "symmetrize": True}])
def test_noalloc_other_options(kw):
    _, _, _, _, v1, v2, r1, r2 = _both(32, 2, 4, 1e-3, **kw)
    _same(v1, v2, r1, r2)


def test_noalloc_rejects_a_run_larger_than_the_scratch():
    import torch

    import paper_1801_10016_amd as g
    s = pins.water(600, 0)                 # one part of 3,600 orbitals: 2 x 3,712^2 floats > 64 MiB
    part = np.zeros(s.n, dtype=np.int32)
    Hd = g.csr_to_device(s.H)
    with g.gsp2_plan_create(Hd, 0.0, part, 1) as plan:
        P = torch.empty(plan.nnz_P, dtype=torch.float32, device="cuda")
        with pytest.raises(g.Gsp2Error) as e:
            g.gsp2_density_noalloc(plan, Hd, s.n_occ, P)
    assert e.value.status == 6 and "static scratch" in str(e.value)

"""The boundary's precision and assembly options and its failure statuses,
through the C ABI, against the FP64 oracle.

* GSP2_PREC_FP64: every step in FP64 on v_mfma_f64_16x16x4_f64, the
  arithmetic of the paper's dgemm runs; bar 1e-10 against the oracle.
* symmetrize: mirrored stored pairs of P become their mean (the oracle's
  csc(symmetrize=True)).
* Failure handling (Methods, SP2: a wrong final trace is a failed run; the
  stop rule ends the iteration): max_iter too small and a switched-off stop
  rule give GSP2_E_NOT_CONVERGED with a finite P, a trace bound the result
  misses gives GSP2_E_WRONG_TRACE, an occupation above n is rejected."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth.partition import uneven_spatial_partition
from tests import _pins as pins

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _prev(s):
    return pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])


@pytest.mark.parametrize("n_mol,seed,n_parts,tau", [(64, 0, 8, 1e-5), (200, 1, 6, 1e-4), (100, 2, 3, 1e-2)])
def test_fp64_products_match_the_oracle(n_mol, seed, n_parts, tau):
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(n_mol, seed)
    Pp = _prev(s)
    part = uneven_spatial_partition(s, n_parts, seed=0)
    ref = oracle.gsp2(s.H, Pp, tau, part, n_parts, s.n_occ)
    P, run, info, index, vals = run_gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, precision="fp64")
    assert run["status"] == 0 and run["precision"] == 4 and np.isfinite(vals).all()
    for k in range(n_parts):
        assert np.array_equal(index[k], ref.index[k])
    err = rel_fro(P, ref.csc())
    print(f"fp64: N={s.n} parts={n_parts} tau={tau} products {run['n_products']} / {ref.sp2.n_products}, "
          f"rel_err={err:.2e}", flush=True)
    # FP64 traces leave no near-tie at this size: the branch sequences agree;
    # where the stop fires can differ by a product or two, since it compares
    # idempotency errors at the rounding level once both runs have converged
    m = min(len(run["alpha"]), len(ref.sp2.alphas))
    assert run["alpha"][:m] == ref.sp2.alphas[:m] and abs(run["n_products"] - ref.sp2.n_products) <= 2
    assert err <= TOL64
    assert abs(run["trace"] - ref.sp2.traces[-1]) <= 1e-9 * s.n


def test_fp64_one_part_is_the_eigen_projector():
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(64, 1)
    part = np.zeros(s.n, dtype=np.int32)
    P, run, _, _, _ = run_gsp2(s.H, s.H, 0.0, part, 1, s.n_occ, precision="fp64")
    Pstar = oracle.eig_projector(s.H, s.n_occ)
    D, _ = oracle.dense_sp2(s.H, s.n_occ)
    e_star, e_dense = rel_fro(P, Pstar), rel_fro(P, D)
    print(f"fp64 dense: vs eigh {e_star:.2e}, vs oracle dense SP2 {e_dense:.2e}", flush=True)
    assert run["status"] == 0 and e_dense <= TOL64 and e_star <= TOL64


def test_fp64_replay_and_refinement():
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(48, 0)
    Pp = _prev(s)
    part = uneven_spatial_partition(s, 4, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 4, s.n_occ)
    P, run, _, _, _ = run_gsp2(s.H, Pp, 1e-3, part, 4, s.n_occ, precision="fp64", alpha_seq=ref.sp2.alphas)
    assert run["status"] == 0 and rel_fro(P, ref.csc()) <= TOL64
    # two FP64 refinement products after the stop keep the converged result
    P2, run2, _, _, _ = run_gsp2(s.H, Pp, 1e-3, part, 4, s.n_occ, precision="fp64", refine=2)
    assert run2["status"] == 0 and run2["n_refine"] == 2
    assert rel_fro(P2, ref.csc()) <= 1e3 * TOL64


@pytest.mark.parametrize("precision,tol", [("fp32", TOL), ("fp64", TOL64)])
def test_symmetrize_matches_the_oracle(precision, tol):
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(64, 0)
    Pp = _prev(s)
    part = uneven_spatial_partition(s, 8, seed=0)
    tau = 1e-2
    ref = oracle.gsp2(s.H, Pp, tau, part, 8, s.n_occ)
    P0, _, _, _, v0 = run_gsp2(s.H, Pp, tau, part, 8, s.n_occ, precision=precision, alpha_seq=ref.sp2.alphas,
                               trace_tol=1e9)
    P1, run, _, _, v1 = run_gsp2(s.H, Pp, tau, part, 8, s.n_occ, precision=precision, alpha_seq=ref.sp2.alphas,
                                 trace_tol=1e9, symmetrize=True)
    err = rel_fro(P1, ref.csc(symmetrize=True))
    print(f"{precision} symmetrize: rel_err={err:.2e}", flush=True)
    assert err <= tol
    # mirrored stored pairs hold one value; the others are the plain assembly's
    A, B = P0.tocsr(), P1.tocsr()
    Bt = B.T.tocsr()
    pattern = A.copy()
    pattern.data = np.ones_like(pattern.data)
    both = pattern.multiply(pattern.T).tocsr()
    r, c = both.nonzero()
    assert np.array_equal(np.asarray(B[r, c]).ravel(), np.asarray(Bt[r, c]).ravel())
    only = pattern - both
    r, c = only.nonzero()
    assert len(r) > 0 and np.array_equal(np.asarray(B[r, c]).ravel(), np.asarray(A[r, c]).ravel())


def test_not_converged_statuses_keep_p_finite():
    from tests._gpu import run_gsp2
    s = pins.water(64, 0)
    Pp = _prev(s)
    part = uneven_spatial_partition(s, 8, seed=0)
    # a budget the stop rule cannot meet
    _, run, _, _, vals = run_gsp2(s.H, Pp, 1e-5, part, 8, s.n_occ, max_iter=5, check=False)
    assert run["status"] == 4 and run["n_products"] == 5 and np.isfinite(vals).all(), run
    # the stop rule switched off: 60 products run past convergence, where
    # eigenvalues a rounding above 1 grow under squaring; P stays finite and
    # the run is not reported as converged
    _, run, _, _, vals = run_gsp2(s.H, Pp, 1e-5, part, 8, s.n_occ, max_iter=60, stop_rule=False, check=False)
    print(f"stop rule off: status {run['status_name']}, {run['n_products']} products, "
          f"max |P| = {np.abs(vals).max():.3e}", flush=True)
    assert run["status"] == 4 and np.isfinite(vals).all()


def test_wrong_trace_status_in_trace_mode():
    from tests._gpu import run_gsp2
    s = pins.water(64, 0)
    Pp = _prev(s)
    part = uneven_spatial_partition(s, 8, seed=0)
    _, ok, _, _, _ = run_gsp2(s.H, Pp, 1e-2, part, 8, s.n_occ)
    miss = abs(ok["trace"] - s.n_occ)
    assert ok["status"] == 0 and miss > 0.0
    _, bad, _, _, vals = run_gsp2(s.H, Pp, 1e-2, part, 8, s.n_occ, trace_tol=0.5 * miss, check=False)
    assert bad["status"] == 5 and bad["n_products"] == ok["n_products"] and np.isfinite(vals).all()


def test_occupation_above_n_is_rejected():
    import paper_1801_10016_amd as g
    from tests._gpu import run_gsp2
    s = pins.water(16, 0)
    part = np.zeros(s.n, dtype=np.int32)
    for occ in (s.n + 1, -1.0):
        with pytest.raises(g.Gsp2Error) as e:
            run_gsp2(s.H, s.H, 1e-5, part, 1, occ)
        assert e.value.status == 1

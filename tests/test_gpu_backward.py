"""Reverse mode (gsp2_backward, FP32 products, checkpointed iterates) against
the FP64 oracle's adjoint, which is itself pinned to central differences,
the closed-form projector derivative and Hellmann-Feynman.

Bar: ||dH_gpu - dH_oracle||_F / ||dH_oracle||_F <= 1e-4.  FP32 rounding in
the ~30 forward products (relative 1e-6 each) is amplified by the reverse
products, whose norms grow with the branch polynomial's derivative near the
crossover; the measured gaps are printed."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth.partition import uneven_spatial_partition
from synth.water import hopping_derivatives
from tests import _pins as pins

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(n_mol, seed, n_parts, tau):
    s = pins.water(n_mol, seed)
    Pp = pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    part = uneven_spatial_partition(s, n_parts, seed=0)
    fw = oracle.gsp2(s.H, Pp, tau, part, n_parts, s.n_occ)
    return s, Pp, part, fw


def _gpu_grad(s, Pp, tau, part, n_parts, alphas, W):
    import torch
    import paper_1801_10016_amd as g
    Hd = g.csr_to_device(s.H)
    with g.gsp2_plan_create(g.csr_to_device(sp.csr_matrix(Pp)), tau, part, n_parts) as plan:
        col_ptr, row_idx = g.gsp2_plan_pattern(plan)
        cols = np.repeat(np.arange(s.n), np.diff(col_ptr))
        dLdP = torch.as_tensor(W[row_idx, cols].astype(np.float32)).cuda()
        dH, info = g.gsp2_backward(plan, Hd, alphas, dLdP)
        torch.cuda.synchronize()
    Hc = s.H.tocsr()
    dense = np.zeros((s.n, s.n))
    rows = np.repeat(np.arange(s.n), np.diff(Hc.indptr))
    dense[rows, Hc.indices] = dH.cpu().numpy()
    return dense, info


@pytest.mark.parametrize("n_mol,seed,n_parts,tau", [(16, 0, 3, 1e-2), (64, 0, 8, 1e-3), (64, 1, 4, 1e-5)])
def test_backward_matches_oracle_adjoint(n_mol, seed, n_parts, tau):
    s, Pp, part, fw = _setup(n_mol, seed, n_parts, tau)
    rng = np.random.default_rng(7)
    W = rng.normal(size=(s.n, s.n))
    W = W + W.T
    ref = oracle.gsp2_grad(s.H, Pp, tau, part, n_parts, fw.sp2.alphas, W)
    got, info = _gpu_grad(s, Pp, tau, part, n_parts, fw.sp2.alphas, W)
    err = np.linalg.norm(got - ref.dH) / np.linalg.norm(ref.dH)
    print(f"backward N={s.n} parts={n_parts} tau={tau}: {len(fw.sp2.alphas)} products, "
          f"checkpoint every {info['checkpoint_every']}, rel_err={err:.2e}; "
          f"rows ({info['row_min']},{info['row_max']}) vs oracle {ref.rows}; "
          f"d_eps ({info['d_eps_min']:.4e},{info['d_eps_max']:.4e}) vs {ref.d_eps[0]:.4e},{ref.d_eps[1]:.4e}",
          flush=True)
    assert (info["row_min"], info["row_max"]) == ref.rows
    # once converged, P hardly depends on the bounds and both derivatives are at
    # rounding level: compare them on the scale of the whole gradient
    scale = 1e-5 * np.linalg.norm(ref.dH)
    assert np.allclose([info["d_eps_min"], info["d_eps_max"]], ref.d_eps, rtol=1e-3, atol=scale)
    assert err <= TOL


def test_backward_band_energy_and_hopping_parameters():
    """L = Tr(P H) (band energy) and the chain rule to the hopping prefactor
    and decay length, through torch.autograd with H's values as a function of
    (A, lam)."""
    import torch
    import paper_1801_10016_amd as g
    from paper_1801_10016_amd.autograd import gsp2_density_autograd
    s, Pp, part, fw = _setup(64, 2, 6, 1e-3)
    tau, n_parts = 1e-3, 6
    DA, DL = hopping_derivatives(s)
    Hc = s.H.tocsr()
    # H's stored values as H_fixed + A * f(lam): intermolecular entries are -A exp(-(r - 2.5)/lam)
    rows = np.repeat(np.arange(s.n), np.diff(Hc.indptr))
    fA = np.asarray(DA[rows, Hc.indices]).ravel()              # = -exp(-(r - 2.5)/lam) on those entries
    inter = fA != 0.0
    r_minus = np.zeros_like(fA)
    r_minus[inter] = -np.log(-fA[inter]) * s.hop_lam          # r - 2.5
    fixed = Hc.data - np.where(inter, s.hop_a * fA, 0.0)
    dev = "cuda"
    A = torch.tensor(s.hop_a, dtype=torch.float64, device=dev, requires_grad=True)
    lam = torch.tensor(s.hop_lam, dtype=torch.float64, device=dev, requires_grad=True)
    rm = torch.as_tensor(r_minus, device=dev)
    mask = torch.as_tensor(inter, device=dev)
    H_val = torch.as_tensor(fixed, device=dev) + torch.where(mask, -A * torch.exp(-rm / lam),
                                                             torch.zeros_like(rm))
    assert np.allclose(H_val.detach().cpu().numpy(), Hc.data, rtol=0, atol=1e-12)
    pattern = g.csr_to_device(s.H)
    with g.gsp2_plan_create(g.csr_to_device(sp.csr_matrix(Pp)), tau, part, n_parts) as plan:
        col_ptr, row_idx = g.gsp2_plan_pattern(plan)
        cols = np.repeat(np.arange(s.n), np.diff(col_ptr))
        # H on P's stored entries, gathered from H_val so both appearances of H are differentiated
        where = sp.csr_matrix((np.arange(1, Hc.nnz + 1, dtype=np.float64), Hc.indices, Hc.indptr), shape=Hc.shape)
        hpos = np.asarray(where[row_idx, cols]).ravel().astype(np.int64) - 1
        has = torch.as_tensor(hpos >= 0, device=dev)
        hidx = torch.as_tensor(np.maximum(hpos, 0), device=dev)
        Hvals_on_P = torch.where(has, H_val[hidx], torch.zeros((), dtype=torch.float64, device=dev))
        P_val = gsp2_density_autograd(H_val, plan, pattern, s.n_occ)
        L = torch.sum(P_val.double() * Hvals_on_P)          # Tr(P H) over P's stored entries
        L.backward()
        gA, gl = float(A.grad), float(lam.grad)
    # oracle: dL/dH through P (W = H on P's pattern) plus the explicit H in Tr(P H)
    W = s.H.toarray()
    ref = oracle.gsp2_grad(s.H, Pp, tau, part, n_parts, fw.sp2.alphas, W)
    Pd = ref.P
    total = ref.dH + np.where(s.H.toarray() != 0, Pd, 0.0)   # explicit part: dTr(PH)/dH = P on H's pattern
    rA = float(np.sum(total * DA.toarray()))
    rl = float(np.sum(total * DL.toarray()))
    print(f"dL/dA gpu {gA:.6e} oracle {rA:.6e}; dL/dlam gpu {gl:.6e} oracle {rl:.6e}", flush=True)
    assert abs(gA - rA) <= 1e-3 * abs(rA)
    assert abs(gl - rl) <= 1e-3 * abs(rl)


def test_backward_water1000_two_losses():
    """1,000 molecules (6,000 orbitals), 32 parts, tau = 1e-3 (at 1e-5 every
    sub-problem is the whole system): L = Tr(P W) with W random symmetric on
    P's pattern, and the band energy Tr(P H); GPU gradient against the
    oracle's, and dL/dA against central differences of the FP64 oracle
    (h = 1e-4, branches replayed).  For the band energy the gradient through
    P nearly cancels (it vanishes for an exact projector), so the gap is
    measured on the scale of the whole gradient, explicit term P included."""
    import time
    s, Pp, part, fw = _setup(1000, 0, 32, 1e-3)
    tau, n_parts = 1e-3, 32
    adj = oracle.threshold_graph(Pp, tau)
    rng = np.random.default_rng(11)
    Ppat = fw.dense() != 0
    W = rng.normal(size=(s.n, s.n))
    W = np.where(Ppat | Ppat.T, W + W.T, 0.0)
    DA, _ = hopping_derivatives(s)
    Hd = s.H.toarray()
    from synth.water import make_water
    h = 1e-4
    for name in ("Tr(PW)", "Tr(PH)"):
        band = name == "Tr(PH)"
        Wl = Hd if band else W
        t0 = time.perf_counter()
        ref = oracle.gsp2_grad(s.H, Pp, tau, part, n_parts, fw.sp2.alphas, Wl, adjacency=adj)
        t_or = time.perf_counter() - t0
        got, info = _gpu_grad(s, Pp, tau, part, n_parts, fw.sp2.alphas, Wl)
        explicit = np.where(Hd != 0, ref.P, 0.0) if band else 0.0   # dTr(PH)/dH at fixed P
        total_ref = ref.dH + explicit
        err_total = np.linalg.norm(got - ref.dH) / np.linalg.norm(total_ref)
        err_through_p = np.linalg.norm(got - ref.dH) / np.linalg.norm(ref.dH)
        print(f"water1000 {name}: {len(fw.sp2.alphas)} products, gap on the whole gradient {err_total:.2e}, "
              f"on the part through P alone {err_through_p:.2e} "
              f"(oracle {t_or:.1f} s, GPU pass workspace {info['workspace_bytes'] / 2**30:.2f} GiB)", flush=True)
        if band:
            # the part through P nearly cancels (Hellmann-Feynman: it vanishes for
            # an exact projector), so FP32 rounding is large relative to it: it is
            # held to the bar on the scale of the whole gradient, and on its own
            # scale to 5e-4 (2.0e-4 measured)
            assert err_total <= TOL and err_through_p <= 5e-4
        else:
            assert err_through_p <= TOL

        def L_of(hop_a):
            Hh = make_water(1000, 0, hop_a=hop_a).H
            g = oracle.gsp2(Hh, Pp, tau, part, n_parts, s.n_occ, alpha_seq=fw.sp2.alphas,
                            trace_tol=1e9, adjacency=adj)
            Pd = g.dense()
            return float(np.sum((Hh.toarray() if band else Wl) * Pd))
        fd = (L_of(s.hop_a + h) - L_of(s.hop_a - h)) / (2 * h)
        an = float(np.sum((got + explicit) * DA.toarray()))
        print(f"  dL/dA: GPU adjoint {an:.6e}, central difference {fd:.6e}", flush=True)
        assert abs(an - fd) <= 1e-4 * abs(fd)

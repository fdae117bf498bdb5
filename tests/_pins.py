"""Checks that tie the FP64 oracle to facts fixed by the paper and by
mathematics (not to the oracle itself).  Each check raises AssertionError.
The planted-mistake test runs them against deliberately broken copies of
the oracle and expects at least one to fail."""
from __future__ import annotations

import json
import os

import numpy as np
import scipy.sparse as sp

import oracle
from synth.partition import molecule_partition, uneven_spatial_partition
from synth.water import make_water

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_cache: dict = {}


def water(n_mol, seed=0, **kw):
    key = (n_mol, seed, tuple(sorted(kw.items())))
    if key not in _cache:
        _cache[key] = make_water(n_mol, seed, **kw)
    return _cache[key]


def cached(key, make):
    if key not in _cache:
        _cache[key] = make()
    return _cache[key]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# -- Gershgorin (Methods, SP2: bounds from the circle theorem) ---------------

def check_gershgorin_textbook():
    # discrete 1-D Laplacian tridiag(-1, 2, -1): discs centred at 2 with
    # radius 2 inside and 1 at the two ends, so the bounds are [0, 4]; its
    # eigenvalues 2 - 2 cos(k pi / (n + 1)) lie strictly inside.
    n = 12
    L = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lo, hi = oracle.gershgorin_bounds(L)
    assert (lo, hi) == (0.0, 4.0), (lo, hi)
    lam = 2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    assert lo < lam.min() and lam.max() < hi
    # a diagonal matrix has zero radii: the bounds are its extreme entries
    d = np.array([3.5, -7.25, 0.0, 11.0])
    assert oracle.gershgorin_bounds(np.diag(d)) == (-7.25, 11.0)
    # sparse and dense inputs agree, signs of off-diagonals do not matter
    A = np.array([[1.0, -2.0, 0.5], [-2.0, -3.0, 1.0], [0.5, 1.0, 4.0]])
    assert oracle.gershgorin_bounds(A) == (-6.0, 5.5)
    assert oracle.gershgorin_bounds(sp.csr_matrix(A)) == (-6.0, 5.5)


def check_gershgorin_contains(H):
    lo, hi = oracle.gershgorin_bounds(H)
    w = np.linalg.eigvalsh(H.toarray() if sp.issparse(H) else H)
    assert lo <= w[0] + 1e-12 and w[-1] <= hi + 1e-12, (lo, hi, w[0], w[-1])


# -- eq. (1): X0 maps the spectrum into [0, 1] in reverse order ---------------

def check_initial_guess(H):
    Hd = H.toarray()
    lo, hi = oracle.gershgorin_bounds(Hd)
    X0 = oracle.initial_guess(Hd, lo, hi)
    w, V = np.linalg.eigh(Hd)
    x = np.diag(V.T @ X0 @ V)
    assert np.all(x >= -1e-12) and np.all(x <= 1 + 1e-12)
    # the lowest eigenvalue of H becomes the largest of X0, and vice versa
    assert np.allclose(x, (hi - w) / (hi - lo), atol=1e-12)
    assert np.all(np.diff(x) <= 1e-12)


# -- the limit of eq. (3) is the projector on the occupied states ------------

def check_dense_projector(sys_, tol=1e-12):
    P, res = oracle.dense_sp2(sys_.H, sys_.n_occ)
    assert res.converged, res.status
    Ps = oracle.eig_projector(sys_.H, sys_.n_occ)
    Hd = sys_.H.toarray()
    assert rel(P, Ps) <= tol, rel(P, Ps)
    assert np.linalg.norm(P @ P - P) / np.linalg.norm(P) <= tol
    assert abs(np.trace(P) - sys_.n_occ) <= 1e-9 * sys_.n
    assert np.linalg.norm(Hd @ P - P @ Hd) / np.linalg.norm(Hd) <= tol
    # tens of products, the range the paper reports for systems of this kind
    assert 15 <= res.n_products <= 60
    return P, res


def check_iterates_are_polynomials(sys_):
    """Every iterate X_t equals the branch maps applied to the eigenvalues of
    X0 (functional calculus); checks every step, not only the limit."""
    Hd = sys_.H.toarray()
    lo, hi = oracle.gershgorin_bounds(Hd)
    X0 = oracle.initial_guess(Hd, lo, hi)
    w, V = np.linalg.eigh(Hd)
    _, res = oracle.dense_sp2(sys_.H, sys_.n_occ)
    for t in range(len(res.alphas) + 1):
        x = (hi - w) / (hi - lo)
        for a in res.alphas[:t]:
            x = (2 * x - x * x) if a > 0 else (x * x)
        Xt = oracle.sp2_blocks([X0], [Hd.shape[0]], sys_.n_occ, alpha_seq=res.alphas[:t]).blocks[0]
        D = V.T @ Xt @ V
        assert np.linalg.norm(D - np.diag(np.diag(D))) <= 1e-10 * max(1.0, np.linalg.norm(D)), t
        assert np.allclose(np.diag(D), x, atol=1e-9), t


def check_branch_direction(sys_):
    """The trace rule picks 2X - X^2 while the trace is at or below N_occ."""
    _, res = oracle.dense_sp2(sys_.H, sys_.n_occ)
    for tr, a in zip(res.traces, res.alphas):
        assert a == (1 if tr <= sys_.n_occ else -1)
    # x -> 2x - x^2 raises and x -> x^2 lowers every eigenvalue in [0, 1], so
    # the chosen branch moves the trace toward N_occ
    for t, a in enumerate(res.alphas):
        step = res.traces[t + 1] - res.traces[t]
        assert (step >= -1e-9) if a > 0 else (step <= 1e-9), (t, a, step)


def check_diagonal_step():
    d = np.array([-3.0, 1.5, -8.0, 0.25, 4.0, -1.0, 2.0])
    P, res = oracle.dense_sp2(np.diag(d), 3)
    expect = np.zeros(7)
    expect[np.argsort(d)[:3]] = 1.0
    assert np.allclose(P, np.diag(expect), atol=1e-12)


# -- A = 0 monomer: closed form ------------------------------------------------

def monomer_eigenvalues():
    """Monomer spectrum from the model, worked by hand: the two O p
    combinations orthogonal to (1,1,1)/sqrt(3) stay at -10 eV and the
    antisymmetric H combination stays at -5 eV; s, the symmetric p
    combination and the symmetric H combination couple through -4 sqrt(2)
    and -4 sqrt(6), giving the cubic
        (l+20)(l+10)(l+5) - 96 (l+20) - 32 (l+10) = 0
      = l^3 + 35 l^2 + 222 l - 1240 = 0 ."""
    cubic = np.sort(np.roots([1.0, 35.0, 222.0, -1240.0]).real)
    return np.sort(np.concatenate([cubic, [-10.0, -10.0, -5.0]]))


def check_monomer():
    s = water(8, seed=3, hop_a=0.0)
    w = np.linalg.eigvalsh(s.H.toarray())
    mono = monomer_eigenvalues()
    assert np.allclose(w, np.repeat(mono, 8), atol=1e-10)
    assert np.allclose(mono[[0, 1, 5]], [-23.010, -15.473, 3.483], atol=1e-3)
    # four occupied states per molecule: the highest is the flat -10 eV band,
    # the lowest empty one the -5 eV H combination, so the gap is 5 eV
    assert abs(oracle.spectral_gap(s.H, s.n_occ) - 5.0) <= 1e-10
    # textbook: a diagonal matrix with two states occupied
    assert oracle.spectral_gap(np.diag([7.0, 1.0, 3.0, 2.0]), 2) == 1.0
    # one part per molecule: the halo is empty and G-SP2 is exact
    Pprev = s.H  # block diagonal pattern, no intermolecular entries
    part = molecule_partition(s)
    g = oracle.gsp2(s.H, Pprev, 1e-5, part, s.n_mol, s.n_occ)
    assert all(len(h) == 0 for h in g.halos)
    assert rel(g.dense(), oracle.eig_projector(s.H, s.n_occ)) <= 1e-12


# -- graph: Fig. 2 worked example, threshold rule, halo definition ------------

def check_fig2():
    with open(os.path.join(GOLDEN, "fig2_corehalo.json")) as f:
        fx = json.load(f)
    names = fx["vertices"]
    ix = {v: i for i, v in enumerate(names)}
    n = len(names)
    Pp = np.eye(n)
    for a, b in fx["edges"]:
        Pp[ix[a], ix[b]] = Pp[ix[b], ix[a]] = 0.5
    A = oracle.threshold_graph(sp.csr_matrix(Pp), 0.1)
    for key in ("a", "b"):
        case = fx["partitions"][key]
        part = np.empty(n, dtype=np.int32)
        for k, members in enumerate(case["parts"]):
            part[[ix[v] for v in members]] = k
        cores, halos = oracle.core_halo(A, part, len(case["parts"]))
        for k in range(len(case["parts"])):
            assert sorted(names[i] for i in halos[k]) == sorted(case["halos"][k])
        sizes = [len(c) + len(h) for c, h in zip(cores, halos)]
        assert sizes == case["sizes"]
        assert oracle.ch_cost(sizes) == case["cost"]
        cut = sum(1 for a, b in fx["edges"] if part[ix[a]] != part[ix[b]])
        assert cut == case["edge_cut"]


def check_threshold_rule():
    tau = 0.25
    P = np.array([[9.0, 0.25, 0.0, -0.3],
                  [0.25, 9.0, 0.2500001, 0.0],
                  [0.0, 0.1, 9.0, 0.0],
                  [-0.3, 0.0, 0.0, 9.0]])
    A = oracle.threshold_graph(sp.csr_matrix(P), tau).toarray()
    expect = np.zeros((4, 4), dtype=np.int8)
    # |0.25| is not > 0.25; |-0.3| is; 0.2500001 above (1,2) only, union makes it symmetric
    for u, v in ((0, 3), (1, 2)):
        expect[u, v] = expect[v, u] = 1
    assert (A == expect).all(), A


def check_halo_brute_force(seed=0):
    rng = np.random.default_rng(seed)
    n, k = 40, 5
    M = (rng.random((n, n)) < 0.08).astype(float)
    M = np.maximum(M, M.T)
    np.fill_diagonal(M, 1.0)
    part = rng.integers(0, k, n).astype(np.int32)
    part[:k] = np.arange(k)
    A = oracle.threshold_graph(sp.csr_matrix(M), 0.5)
    cores, halos = oracle.core_halo(A, part, k)
    for p in range(k):
        core = [v for v in range(n) if part[v] == p]
        halo = sorted({u for v in core for u in range(n) if u != v and M[v, u] > 0.5 and part[u] != p})
        assert list(cores[p]) == core
        assert list(halos[p]) == halo


# -- G-SP2 special cases -------------------------------------------------------

def check_gsp2_one_part_is_dense(sys_):
    P, res = oracle.dense_sp2(sys_.H, sys_.n_occ)
    part = np.zeros(sys_.n, dtype=np.int32)
    g = oracle.gsp2(sys_.H, P, 1e-5, part, 1, sys_.n_occ)
    # equal up to the summation order of the sparse vs dense Gershgorin row
    # sums; that rounding can move the stop by one product, so the branch
    # sequences need only agree on their common prefix
    m = min(len(g.sp2.alphas), len(res.alphas))
    assert g.sp2.alphas[:m] == res.alphas[:m] and abs(len(g.sp2.alphas) - len(res.alphas)) <= 2
    assert rel(g.dense(), P) <= 1e-13


def check_gsp2_full_halo_is_dense(sys_):
    P, res = oracle.dense_sp2(sys_.H, sys_.n_occ)
    part = uneven_spatial_partition(sys_, 4, seed=1)
    full = np.ones((sys_.n, sys_.n))
    g = oracle.gsp2(sys_.H, sp.csr_matrix(full), 0.5, part, 4, sys_.n_occ)
    assert all(s == sys_.n for s in g.sizes)
    assert rel(g.dense(), P) <= 1e-12


def check_symmetrize(sys_, tau=1e-2, n_parts=8):
    """P assembled from core columns, symmetrised on its own pattern: every
    stored entry whose mirror is stored becomes the mean of the two, others
    stay (brute force over the stored entries); with complete halos the
    pattern is full and the result is (P + P^T) / 2."""
    P0, _ = oracle.dense_sp2(sys_.H, sys_.n_occ)
    part = uneven_spatial_partition(sys_, n_parts, seed=0)
    g = oracle.gsp2(sys_.H, P0, tau, part, n_parts, sys_.n_occ)
    A = g.csc().toarray()
    stored = np.zeros(A.shape, dtype=bool)
    for idx, core in zip(g.index, g.cores):
        stored[np.ix_(idx, core)] = True
    B = g.csc(symmetrize=True).toarray()
    assert g.csc(symmetrize=True).nnz == g.csc().nnz
    n_mirrored = 0
    for i, j in zip(*np.nonzero(stored)):
        if stored[j, i]:
            assert B[i, j] == 0.5 * (A[i, j] + A[j, i])
            n_mirrored += 1
        else:
            assert B[i, j] == A[i, j]
    assert 0 < n_mirrored < stored.sum()          # both kinds occur at this tau
    assert np.array_equal(g.dense(symmetrize=True), B)
    full = oracle.gsp2(sys_.H, sp.csr_matrix(np.ones(A.shape)), 0.5, part, n_parts, sys_.n_occ)
    F = full.dense()
    assert np.allclose(full.dense(symmetrize=True), 0.5 * (F + F.T), rtol=0, atol=1e-15)


def check_occupation_status(sys_, tau=1e-2, n_parts=4):
    """A stop whose result misses N_occ by more than trace_tol is a failed
    run; the same run with a bound above its miss succeeds.  Truncated halos
    leave the G-SP2 trace a little off N_occ."""
    P, _ = oracle.dense_sp2(sys_.H, sys_.n_occ)
    part = uneven_spatial_partition(sys_, n_parts, seed=0)
    ok = oracle.gsp2(sys_.H, P, tau, part, n_parts, sys_.n_occ).sp2
    miss = abs(ok.traces[-1] - sys_.n_occ)
    assert ok.converged and ok.status == "ok" and miss > 0.0
    bad = oracle.gsp2(sys_.H, P, tau, part, n_parts, sys_.n_occ, trace_tol=0.5 * miss).sp2
    assert not bad.converged and bad.status == "wrong_trace" and bad.n_products == ok.n_products
    assert bad.alphas == ok.alphas
    again = oracle.gsp2(sys_.H, P, tau, part, n_parts, sys_.n_occ, trace_tol=2.0 * miss).sp2
    assert again.status == "ok"


def check_gsp2_truncation(sys_, n_parts=8):
    P, _ = oracle.dense_sp2(sys_.H, sys_.n_occ)
    Ps = oracle.eig_projector(sys_.H, sys_.n_occ)
    part = uneven_spatial_partition(sys_, n_parts, seed=0)
    out = {}
    for tau in (1e-5, 1e-2):
        g = oracle.gsp2(sys_.H, P, tau, part, n_parts, sys_.n_occ)
        assert g.sp2.converged
        err = rel(g.dense(), Ps)
        assert err <= 10 * tau, (tau, err)
        out[tau] = (err, g)
    # a real truncation at 1e-2: smaller blocks, non-zero error
    g2 = out[1e-2][1]
    assert max(g2.sizes) < sys_.n and out[1e-2][0] > 1e-4
    return out


def check_gsp2_blocks_share_sequence(sys_, tau=1e-2, n_parts=8):
    """With truncated halos, each part's final block is still the common
    branch polynomial of its own X0 (one global sequence for every part)."""
    P, _ = oracle.dense_sp2(sys_.H, sys_.n_occ)
    part = uneven_spatial_partition(sys_, n_parts, seed=0)
    g = oracle.gsp2(sys_.H, P, tau, part, n_parts, sys_.n_occ)
    lo, hi = g.eps
    kept = g.sp2.alphas
    for k in (0, n_parts - 1):
        idx = g.index[k]
        X0 = oracle.initial_guess(sys_.H[idx][:, idx].toarray(), lo, hi)
        w, V = np.linalg.eigh(X0)
        x = w.copy()
        for a in kept:
            x = (2 * x - x * x) if a > 0 else (x * x)
        Xk = (V * x) @ V.T
        c = len(g.cores[k])
        assert np.allclose(Xk[:, :c], g.core_columns[k], atol=1e-9)


def check_core_column_layout(sys_, tau=1e-2, n_parts=8):
    """Part k writes P's core columns: column j of part k is non-zero only in
    part k's rows (core + halo)."""
    P, _ = oracle.dense_sp2(sys_.H, sys_.n_occ)
    part = uneven_spatial_partition(sys_, n_parts, seed=0)
    g = oracle.gsp2(sys_.H, P, tau, part, n_parts, sys_.n_occ)
    D = g.dense()
    for k in range(n_parts):
        outside = np.setdiff1d(np.arange(sys_.n), g.index[k])
        assert np.abs(D[np.ix_(outside, g.cores[k])]).max(initial=0.0) == 0.0
        assert np.array_equal(D[np.ix_(g.index[k], g.cores[k])], g.core_columns[k])


def check_thresholded_sp2(sys_):
    """Thresholded-algebra SP2 of the whole matrix: with a threshold below any
    rounding-level entry it is the eigen projector; every entry it keeps
    exceeds the threshold in magnitude; and its distance from the projector
    grows with the threshold but stays within the sum of what can be dropped
    (at most n^2 entries of size eps per product over the run)."""
    Pstar = oracle.eig_projector(sys_.H, sys_.n_occ)
    P0, r0 = oracle.thresholded_sp2(sys_.H, sys_.n_occ, 1e-14)
    assert r0.status == "ok" and rel(P0, Pstar) <= 1e-12
    prev = 0.0
    for eps in (1e-8, 1e-6, 1e-4):
        P, r = oracle.thresholded_sp2(sys_.H, sys_.n_occ, eps)
        kept = P[P != 0]
        assert r.status == "ok" and np.all(np.abs(kept) > eps), eps
        err = rel(P, Pstar)
        bound = r.n_products * sys_.n * eps / np.linalg.norm(Pstar)
        assert prev <= err <= bound, (eps, err, bound)
        prev = err


def battery():
    """Every pin, on small systems; raises on the first failure."""
    check_gershgorin_textbook()
    for seed in (0, 1):
        check_gershgorin_contains(water(64, seed).H)
    check_initial_guess(water(16, 0).H)
    check_dense_projector(water(64, 0))
    check_iterates_are_polynomials(water(16, 1))
    check_branch_direction(water(64, 0))
    check_diagonal_step()
    check_monomer()
    check_fig2()
    check_threshold_rule()
    for seed in range(4):
        check_halo_brute_force(seed)
    check_gsp2_one_part_is_dense(water(32, 0))
    check_gsp2_full_halo_is_dense(water(24, 2))
    check_gsp2_truncation(water(64, 0))
    check_gsp2_blocks_share_sequence(water(64, 0))
    check_core_column_layout(water(64, 0))
    check_symmetrize(water(32, 0))
    check_occupation_status(water(32, 0))
    check_thresholded_sp2(water(64, 1))
    check_adjoint_finite_differences()
    check_adjoint_closed_form()


if __name__ == "__main__":
    battery()


# -- adjoint of the recursion (oracle/adjoint.py) -----------------------------

def _grad_case():
    from synth.water import hopping_derivatives
    s = water(16, 0)
    P0 = cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    part = uneven_spatial_partition(s, 3, seed=0)
    tau = 1e-2
    fw = oracle.gsp2(s.H, P0, tau, part, 3, s.n_occ)
    rng = np.random.default_rng(2)
    W = rng.normal(size=(s.n, s.n))
    W = W + W.T
    adj = oracle.threshold_graph(P0, tau)

    def L_of(H):
        g = oracle.gsp2(H, P0, tau, part, 3, s.n_occ, alpha_seq=fw.sp2.alphas, trace_tol=1e9, adjacency=adj)
        return float(np.sum(W * g.dense()))
    gr = oracle.gsp2_grad(s.H, P0, tau, part, 3, fw.sp2.alphas, W)
    Hc = s.H.tocsr()
    E = sp.csr_matrix((rng.normal(size=Hc.nnz), Hc.indices, Hc.indptr), shape=Hc.shape)
    E = 0.5 * (E + E.T)
    return s, gr, L_of, E, hopping_derivatives(s), fw


def check_adjoint_finite_differences():
    """Central differences (replayed branches) along a random symmetric
    direction and along dH/dA, dH/dlam of the hopping model."""
    s, gr, L_of, E, (DA, DL), fw = _grad_case()
    assert np.array_equal(gr.P, fw.dense())
    # the gradient under symmetric perturbations is split evenly between H_uv and H_vu
    assert np.allclose(gr.dH, gr.dH.T, rtol=0, atol=1e-12 * np.abs(gr.dH).max())
    for D, h, tol in ((E, 1e-4, 1e-6), (DA, 1e-4, 1e-6), (DL, 1e-5, 1e-5)):
        fd = (L_of(s.H + h * D) - L_of(s.H - h * D)) / (2 * h)
        an = float(np.sum(gr.dH * D.toarray()))
        assert abs(fd - an) <= tol * abs(fd), (fd, an)


def check_adjoint_closed_form():
    """Converged dense SP2: the adjoint of the recursion is the derivative of
    the spectral projector, sum_{o,u} [v_o (v_o^T W v_u) v_u^T + transpose] / (e_o - e_u),
    and for L = Tr(P H) the part through P vanishes (Hellmann-Feynman)."""
    s = water(8, 1)
    Pd, rd = oracle.dense_sp2(s.H, s.n_occ)
    rng = np.random.default_rng(5)
    W = rng.normal(size=(s.n, s.n))
    W = W + W.T
    one = np.zeros(s.n, dtype=np.int32)
    g1 = oracle.gsp2_grad(s.H, Pd, 0.0, one, 1, rd.alphas, W)
    w, V = np.linalg.eigh(s.H.toarray())
    no = s.n_occ
    Vo, Vu = V[:, :no], V[:, no:]
    C = Vo @ ((Vo.T @ W @ Vu) / (w[:no, None] - w[None, no:])) @ Vu.T
    cf = C + C.T
    pat = s.H.toarray() != 0
    cf = np.where(pat, cf, 0.0)
    assert np.linalg.norm(cf - g1.dH) <= 1e-10 * np.linalg.norm(cf)
    g2 = oracle.gsp2_grad(s.H, Pd, 0.0, one, 1, rd.alphas, s.H.toarray())
    assert np.linalg.norm(g2.dH) <= 1e-10 * np.linalg.norm(Pd)

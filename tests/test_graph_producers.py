"""Producers of the graph and partition (host, no GPU).

gsp2_partition_anneal: simulated-annealing refinement of a
partition for the cost of eq. (4), C = sum_k (c_k + h_k)^3.

Pins: the cost the library reports for the partition it was given and for
the one it returns equals the oracle's eq. (4) cost of the same partitions
(exact integers); on graphs small enough to enumerate every partition, the
annealer reaches the brute-force optimum; it never returns a worse
partition, never empties a part, and is deterministic for a seed.

gsp2_locality_graph: the graph of the locality construction, against its
definition evaluated by brute force over all atom pairs, and against the
threshold of the distance-based stand-in for a previous P (equal by
construction of the stand-in's radius)."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_1801_10016_amd as g
from paper_1801_10016_amd import gsp2 as binding
from synth.partition import uneven_spatial_partition
from tests import _pins as pins


def _csr(A):
    A = sp.csr_matrix(A)
    return A.indptr.astype(np.int64), A.indices.astype(np.int32)


def _cost(A, part, n_parts):
    cores, halos = oracle.core_halo(oracle.threshold_graph(A, 0.5), part, n_parts)
    return oracle.ch_cost([len(c) + len(h) for c, h in zip(cores, halos)])


def _brute_force(A, n, n_parts):
    best = None
    for labels in itertools.product(range(n_parts), repeat=n):
        if len(set(labels)) < n_parts:
            continue
        c = _cost(A, np.array(labels), n_parts)
        best = c if best is None else min(best, c)
    return best


def _fig2():
    import json
    import os
    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fig2_corehalo.json")))
    names = spec["vertices"]
    ix = {v: i for i, v in enumerate(names)}
    A = np.zeros((6, 6))
    for a, b in spec["edges"]:
        A[ix[a], ix[b]] = A[ix[b], ix[a]] = 1.0
    part_b = np.zeros(6, dtype=np.int32)
    for k, members in enumerate(spec["partitions"]["b"]["parts"]):
        for v in members:
            part_b[ix[v]] = k
    return A, part_b


def test_fig2_reaches_the_optimum_from_the_worse_partition():
    # the paper's Fig. 2: partition (b) costs 243; the better (a) costs 189
    A, part_b = _fig2()
    ptr, col = _csr(A)
    out, before, after = g.gsp2_partition_anneal(ptr, col, part_b, 2, sweeps=50, seed=1)
    assert before == 243 == _cost(A, part_b, 2)
    assert after == _cost(A, out, 2) == _brute_force(A, 6, 2)
    assert after <= 189


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_small_graphs_reach_the_brute_force_optimum(seed):
    rng = np.random.default_rng(seed)
    n, k = 8, 3
    A = np.triu((rng.random((n, n)) < 0.35).astype(float), 1)
    A = A + A.T
    start = np.arange(n, dtype=np.int32) % k
    ptr, col = _csr(A)
    best = min(g.gsp2_partition_anneal(ptr, col, start, k, sweeps=200, seed=s)[2] for s in range(3))
    assert best == _brute_force(A, n, k)


def test_water_graph_costs_match_the_oracle():
    s = pins.water(64, 0)
    P = pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    adj = oracle.threshold_graph(P, 1e-3)
    n_parts = 8
    part = uneven_spatial_partition(s, n_parts, seed=0)
    ptr, col = _csr(adj)
    out, before, after = g.gsp2_partition_anneal(ptr, col, part, n_parts, seed=5)
    assert before == _cost(adj, part, n_parts)
    assert after == _cost(adj, out, n_parts)
    assert after <= before
    assert np.bincount(out, minlength=n_parts).min() >= 1
    again = g.gsp2_partition_anneal(ptr, col, part, n_parts, seed=5)
    assert np.array_equal(again[0], out) and again[2] == after
    print(f"water 64, 8 parts, tau 1e-3: C {before} -> {after} ({after / before:.3f})")


def test_greedy_refinement_never_worsens():
    s = pins.water(32, 1)
    P = pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    adj = oracle.threshold_graph(P, 1e-3)
    part = uneven_spatial_partition(s, 4, seed=0)
    ptr, col = _csr(adj)
    out, before, after = g.gsp2_partition_anneal(ptr, col, part, 4, t0=-1.0, seed=2)
    assert after <= before and after == _cost(adj, out, 4)


def test_bad_arguments_are_refused():
    A, part_b = _fig2()
    ptr, col = _csr(A)
    with pytest.raises(g.Gsp2Error) as e:
        g.gsp2_partition_anneal(ptr, col, np.zeros(6, dtype=np.int32), 2)        # part 1 empty
    assert e.value.status == binding.GSP2_E_INVALID and "empty" in str(e.value)
    with pytest.raises(g.Gsp2Error):
        g.gsp2_partition_anneal(ptr, col, part_b, 2, cooling=1.5)
    with pytest.raises(g.Gsp2Error):
        g.gsp2_partition_anneal(ptr, col, part_b, 2, sweeps=-1)


# -- locality construction of the graph -----------------------------------------

def _brute_locality(system, radius):
    """Adjacency by definition: orbitals on atoms closer than radius (minimum image)."""
    oa = system.orbital_atom()
    X = system.atoms
    d = X[:, None, :] - X[None, :, :]
    d -= system.box * np.round(d / system.box)
    close = np.sqrt((d ** 2).sum(-1)) < radius            # includes each atom with itself
    A = close[np.ix_(oa, oa)]
    np.fill_diagonal(A, False)
    return A


@pytest.mark.parametrize("n_mol,radius", [(8, 3.0), (32, 4.5), (64, 7.0)])
def test_locality_graph_matches_brute_force(n_mol, radius):
    s = pins.water(n_mol, 0)
    ptr, col = g.gsp2_locality_graph(s.orbital_atom(), s.atoms, radius, s.box)
    A = sp.csr_matrix((np.ones(col.size), col, ptr), shape=(s.n, s.n)).toarray() != 0
    want = _brute_locality(s, radius)
    assert np.array_equal(A, want)
    assert np.array_equal(A, A.T)
    for u in range(s.n):                                   # rows ascending, no self loops
        row = col[ptr[u]:ptr[u + 1]]
        assert np.all(np.diff(row) > 0) and u not in row


def test_locality_graph_is_the_thresholded_distance_stand_in():
    # the stand-in for a previous P is 1e-3 exp(-(r - R3) / XI) for atoms at
    # distance r: above tau exactly inside the radius R3 + XI ln(1e-3 / tau)
    from synth.locality import surrogate_prev_density, surrogate_radius
    s = pins.water(200, 2)
    tau = 1e-4
    Q = surrogate_prev_density(s, q_floor=tau / 2)
    ref = oracle.threshold_graph(Q, tau)
    ptr, col = g.gsp2_locality_graph(s.orbital_atom(), s.atoms, surrogate_radius(tau), s.box)
    A = sp.csr_matrix((np.ones(col.size), col, ptr), shape=(s.n, s.n))
    assert ((A != 0) != (ref != 0)).nnz == 0


def test_locality_graph_open_boundaries_and_errors():
    xyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    oa = np.array([0, 0, 1, 2], dtype=np.int32)             # two orbitals on atom 0
    ptr, col = g.gsp2_locality_graph(oa, xyz, 1.5)
    rows = [col[ptr[u]:ptr[u + 1]].tolist() for u in range(4)]
    assert rows == [[1, 2], [0, 2], [0, 1], []]
    with pytest.raises(g.Gsp2Error):
        g.gsp2_locality_graph(oa, xyz, 0.0)
    with pytest.raises(g.Gsp2Error):
        g.gsp2_locality_graph(np.array([0, 3], dtype=np.int32), xyz, 1.0)


# -- gsp2_sparse_sp2_host: the first P by thresholded sparse SP2 ------------

def _sparse_vs_oracle(s, eps, **kw):
    P, info = g.gsp2_sparse_sp2_host(s.H, s.n_occ, eps, **kw)
    Po, r = oracle.thresholded_sp2(s.H, s.n_occ, eps, **kw)
    return P, info, Po, r


@pytest.mark.parametrize("n_mol,seed,eps", [(64, 0, 1e-10), (64, 0, 1e-6), (64, 0, 1e-4), (100, 2, 1e-6),
                                            (100, 2, 1e-3)])
def test_sparse_sp2_matches_the_oracle(n_mol, seed, eps):
    # the same steps in FP64 on both sides: the branch sequences agree (a
    # stop may fall one product apart where e_t sits at rounding level), P
    # agrees to rounding, and both keep exactly the entries above eps
    s = pins.water(n_mol, seed)
    P, info, Po, r = _sparse_vs_oracle(s, eps)
    a, b = info["alpha"], r.alphas
    m = min(len(a), len(b))
    assert info["status"] == 0 and r.status == "ok" and a[:m] == b[:m] and abs(len(a) - len(b)) <= 1
    err = np.linalg.norm(P.toarray() - Po) / np.linalg.norm(Po)
    print(f"{n_mol} molecules, eps {eps:g}: {info['n_products']} products, nnz {P.nnz}, rel_err {err:.2e}", flush=True)
    assert err <= (1e-12 if a == b else 1e-9)
    assert np.all(np.abs(P.data) > eps)
    if a == b:
        assert P.nnz == np.count_nonzero(Po)
    assert abs(info["trace"] - np.trace(P.toarray())) <= 1e-9 * s.n
    emin, emax = oracle.gershgorin_bounds(s.H)
    assert (info["eps_min"], info["eps_max"]) == pytest.approx((emin, emax), rel=1e-14, abs=1e-12)


def test_sparse_sp2_without_threshold_is_the_projector():
    s = pins.water(32, 1)
    P, info = g.gsp2_sparse_sp2_host(s.H, s.n_occ, 0.0)
    Pstar = oracle.eig_projector(s.H, s.n_occ)
    assert info["status"] == 0
    assert np.linalg.norm(P.toarray() - Pstar) <= 1e-12 * np.linalg.norm(Pstar)


def test_sparse_sp2_graph_feeds_a_plan_graph():
    # thresholding the sparse P at tau gives the oracle's graph of its own
    # thresholded P (an input the plan takes as it is)
    s = pins.water(100, 0)
    P, _, Po, _ = _sparse_vs_oracle(s, 1e-7)
    A = oracle.threshold_graph(P, 1e-4)
    Ao = oracle.threshold_graph(Po, 1e-4)
    assert (A != Ao).nnz == 0 and A.nnz > 0


def test_sparse_sp2_statuses_and_arguments():
    s = pins.water(16, 0)
    P, info = g.gsp2_sparse_sp2_host(s.H, s.n_occ, 1e-6, max_iter=5, check=False)
    assert info["status"] == binding.GSP2_E_NOT_CONVERGED and np.isfinite(P.data).all()
    P1, _ = g.gsp2_sparse_sp2_host(s.H, s.n_occ, 1e-6)
    P2, _ = g.gsp2_sparse_sp2_host(s.H, s.n_occ, 1e-6)
    assert (P1 != P2).nnz == 0
    for kw in ({"n_occ": s.n + 1}, {"n_occ": -1}, {"eps": -1.0}, {"max_iter": 0}):
        args = dict(n_occ=s.n_occ, eps=1e-6, max_iter=60)
        args.update(kw)
        with pytest.raises(binding.Gsp2Error) as e:
            g.gsp2_sparse_sp2_host(s.H, args["n_occ"], args["eps"], max_iter=args["max_iter"])
        assert e.value.status == binding.GSP2_E_INVALID

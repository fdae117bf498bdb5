"""Batched plans: several independent systems in one plan, the tiles of all
of them in every product launch, each system with its own Gershgorin bounds,
occupation, trace, branch sequence, stop and status.

Bars:
* each system's P against the FP64 oracle run on that system alone,
  <= 1e-5 relative Frobenius with FP32 products (tie-aware, as in the
  single-system parity tests), index sets bit-exact;
* a batched run equals, bit for bit, runs of plans that hold one system each
  (FP32, and FP16 with FP32 refinement products);
* per-system statuses are independent; graphs that join two systems, and
  backward passes of batched plans, are refused."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth.partition import uneven_spatial_partition
from tests import _pins as pins

pytestmark = pytest.mark.gpu

TOL = 1e-5
MIXED_TOL_FP16 = 1e-3          # the stated bar of 16-bit products, against the FP64 oracle


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_10016_amd as g
    g.load()


def tie_band(n):
    return 1e-4 * max(1.0, n / 1000.0)


def _dense_prev(s):
    return pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])


class Batch:
    """Block-diagonal union of systems; parts numbered system by system."""

    def __init__(self, systems, n_parts, tau):
        self.systems = systems
        self.n_parts = list(n_parts)
        self.tau = tau
        self.H_s = [s.H.tocsr().sorted_indices() for s in systems]
        self.Pp_s = [sp.csr_matrix(_dense_prev(s)) for s in systems]
        self.part_s = [uneven_spatial_partition(s, k, seed=0) for s, k in zip(systems, n_parts)]
        self.offs = np.cumsum([0] + [s.n for s in systems])
        self.part_offs = np.cumsum([0] + self.n_parts)
        self.H = sp.block_diag(self.H_s, format="csr").sorted_indices()
        self.Pp = sp.block_diag(self.Pp_s, format="csr")
        self.part = np.concatenate([p + o for p, o in zip(self.part_s, self.part_offs)]).astype(np.int32)
        self.part_system = np.repeat(np.arange(len(systems)), self.n_parts).astype(np.int32)
        self.n_occ = [s.n_occ for s in systems]

    def run(self, **kw):
        import torch
        import paper_1801_10016_amd as g
        Hd = g.csr_to_device(self.H)
        Pd = g.csr_to_device(self.Pp)
        with g.gsp2_plan_create(Pd, self.tau, self.part, int(self.part_offs[-1]),
                                part_system=self.part_system) as plan:
            info, _, _ = g.gsp2_plan_query(plan)
            assert info["n_systems"] == len(self.systems)
            col_ptr, row_idx = g.gsp2_plan_pattern(plan)
            P_val = torch.full((info["nnz_P"],), float("nan"), dtype=torch.float32, device="cuda")
            runs = g.gsp2_density(plan, Hd, self.n_occ, P_val, **kw)
            torch.cuda.synchronize()
            vals = P_val.cpu().numpy()
            index = [g.gsp2_plan_part_index(plan, k) for k in range(int(self.part_offs[-1]))]
        n = self.H.shape[0]
        P = sp.csc_matrix((vals.astype(np.float64), row_idx, col_ptr), shape=(n, n))
        return P, runs, vals, col_ptr, index

    def block(self, P, i):
        a, b = self.offs[i], self.offs[i + 1]
        return P[a:b, a:b]

    def system_vals(self, vals, col_ptr, i):
        # a system's columns are contiguous, and each column lists its rows ascending
        return vals[col_ptr[self.offs[i]]:col_ptr[self.offs[i + 1]]]


def _small_batch():
    systems = [pins.water(16, 0), pins.water(40, 1), pins.water(64, 2), pins.water(24, 3),
               pins.water(100, 4), pins.water(48, 5)]
    return pins.cached(("batch", "small"), lambda: Batch(systems, [2, 4, 8, 3, 6, 5], 1e-3))


def _oracles(b):
    return [oracle.gsp2(b.H_s[i], b.Pp_s[i], b.tau, b.part_s[i], b.n_parts[i], s.n_occ)
            for i, s in enumerate(b.systems)]


def test_batch_matches_oracle_per_system():
    from tests._gpu import rel_fro
    b = _small_batch()
    refs = _oracles(b)
    P, runs, vals, col_ptr, index = b.run()
    assert len(runs) == len(b.systems)
    assert np.isfinite(vals).all()
    replay = False
    for i, (s, ref, run) in enumerate(zip(b.systems, refs, runs)):
        assert run["status"] == 0, (i, run)
        for k in range(b.n_parts[i]):
            got = index[b.part_offs[i] + k] - b.offs[i]
            assert np.array_equal(got, ref.index[k]), (i, k)
        lo, hi = oracle.gershgorin_bounds(b.H_s[i])
        assert abs(run["eps_min"] - lo) <= 1e-12 * abs(lo) and abs(run["eps_max"] - hi) <= 1e-12 * abs(hi)
        ga, oa = run["alpha"], ref.sp2.alphas
        diff = [t for t in range(min(len(ga), len(oa))) if ga[t] != oa[t]]
        if diff:
            gap = abs(ref.sp2.traces[diff[0]] - s.n_occ)
            print(f"  system {i}: branch sequences part at product {diff[0]}, |Tr - N_occ| = {gap:.2e}")
            assert gap <= tie_band(s.n)
            replay = True
    if replay:
        P, runs, vals, col_ptr, index = b.run(alpha_seq=[r.sp2.alphas for r in refs], trace_tol=1e9)
    for i, ref in enumerate(refs):
        err = rel_fro(b.block(P, i), ref.csc())
        print(f"system {i}: N={b.systems[i].n} parts={b.n_parts[i]} products gpu={runs[i]['n_products']} "
              f"oracle={ref.sp2.n_products} rel_err={err:.2e}", flush=True)
        assert err <= TOL, (i, err)


@pytest.mark.parametrize("precision,refine,refine_precision", [("fp32", 0, "fp32"), ("fp16", 2, "fp32"),
                                                                ("fp16", 2, "fp16x3")])
def test_batch_equals_one_system_plans(precision, refine, refine_precision):
    from tests._gpu import run_gsp2
    b = _small_batch()
    P, runs, vals, col_ptr, _ = b.run(precision=precision, refine=refine, refine_precision=refine_precision)
    for i, s in enumerate(b.systems):
        _, run1, _, _, vals1 = run_gsp2(b.H_s[i], b.Pp_s[i], b.tau, b.part_s[i], b.n_parts[i], s.n_occ,
                                        precision=precision, refine=refine, refine_precision=refine_precision)
        assert runs[i]["alpha"] == run1["alpha"] and runs[i]["n_products"] == run1["n_products"], i
        assert runs[i]["traces"] == run1["traces"], i
        assert np.array_equal(b.system_vals(vals, col_ptr, i), vals1), i


def test_batch_mixed_precision_against_oracle():
    from tests._gpu import rel_fro
    b = _small_batch()
    refs = _oracles(b)
    P, runs, vals, _, _ = b.run(precision="fp16", refine=2)
    for i, ref in enumerate(refs):
        assert runs[i]["status"] == 0 and runs[i]["n_refine"] == 2, (i, runs[i])
        err = rel_fro(b.block(P, i), ref.csc())
        print(f"fp16+2 system {i}: rel_err={err:.2e}", flush=True)
        assert err <= MIXED_TOL_FP16, (i, err)


def test_per_system_status_is_independent():
    # system 2 replays five 2X - X^2 branches, which push its trace towards n:
    # it alone misses its occupation
    b = _small_batch()
    refs = _oracles(b)
    seqs = [r.sp2.alphas for r in refs]
    seqs[2] = [1] * 5
    P, runs, vals, col_ptr, _ = b.run(alpha_seq=seqs, trace_tol=0.5, check=False)
    assert runs[2]["status"] == 5 and runs[2]["n_alpha"] == 5          # GSP2_E_WRONG_TRACE
    assert "system 2" in runs[0]["message"]
    for i in (0, 1, 3, 4, 5):
        assert runs[i]["status"] == 0, (i, runs[i])
        assert runs[i]["n_alpha"] == len(seqs[i])


def test_graph_joining_two_systems_is_refused():
    import paper_1801_10016_amd as g
    b = _small_batch()
    Pp = b.Pp.tolil()
    u, v = int(b.offs[1]) - 1, int(b.offs[1])          # last vertex of system 0, first of system 1
    Pp[u, v] = Pp[v, u] = 1.0
    with pytest.raises(g.Gsp2Error) as e:
        g.gsp2_plan_create(g.csr_to_device(Pp.tocsr()), b.tau, b.part, int(b.part_offs[-1]),
                           part_system=b.part_system)
    assert e.value.status == 1 and "joins systems 0 and 1" in str(e.value)


def test_backward_of_batched_plan_is_refused():
    import torch
    import paper_1801_10016_amd as g
    b = _small_batch()
    with g.gsp2_plan_create(g.csr_to_device(b.Pp), b.tau, b.part, int(b.part_offs[-1]),
                            part_system=b.part_system) as plan:
        dLdP = torch.zeros(plan.nnz_P, dtype=torch.float32, device="cuda")
        with pytest.raises(g.Gsp2Error) as e:
            g.gsp2_backward(plan, g.csr_to_device(b.H), [-1, 1], dLdP)
        assert e.value.status == 6                       # GSP2_E_UNSUPPORTED

"""Full-size G-SP2 on the GPU against the FP64 oracle, in the benchmark's
workload and launch configuration: 3,500 water molecules (21,000 orbitals),
128 uneven parts, tau = 1e-5, one HIP graph per density matrix.

The graph comes from a previous P computed by regular SP2 (Methods, "Graph
Theory"): here the library's FP64 dense SP2 of H, whose threshold must give
exactly the graph of the oracle's own FP64 dense SP2 P (stored digest; no
entry of the oracle's P lies within 1e-7 relative of tau, so rounding-level
differences cannot move an edge).  The stored expectations
(tests/golden/gsp2_water3500_densep_tau1e-5.*, oracle calls only) give, per
part, its index list digest and a Gaussian sketch of its core columns, so
every one of the 128 parts is compared element-sensitively; three parts are
also recomputed here by the oracle and compared element by element."""
import numpy as np
import pytest

from synth.partition import uneven_spatial_partition
from synth.water import make_water
from tests import _full

pytestmark = pytest.mark.gpu

STEM = "gsp2_water3500_densep_tau1e-5"
TOL = 1e-5                 # FP32 products
TOL64 = 1e-10              # FP64 products
MIXED_TOL = 1e-3           # 16-bit products, before refinement


@pytest.fixture(scope="module")
def case():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_10016_amd as g
    gold, arrays = _full.load_golden(STEM)
    sp_ = gold["spec"]
    s = make_water(sp_["n_mol"], sp_["seed"])
    part = uneven_spatial_partition(s, sp_["n_parts"], sp_["core_lo"], sp_["core_hi"], seed=sp_["seed"])
    stream = torch.cuda.Stream()
    Hd = g.csr_to_device(s.H)
    print(f"full size: N={s.n}; FP64 regular SP2 for the previous P", flush=True)
    Pprev, dense_run = _full.fp64_previous_p(g, torch, Hd, s.n, s.n_occ, stream)
    dsk = _full.dense_sketch(torch, Pprev.val, s.n)
    with torch.cuda.stream(stream):
        plan = g.gsp2_plan_create(Pprev, sp_["tau"], part, sp_["n_parts"], stream=stream)
    del Pprev
    torch.cuda.empty_cache()
    info, cs, ss = g.gsp2_plan_query(plan)
    col_ptr, _ = g.gsp2_plan_pattern(plan)
    adj_ptr, adj_col = g.gsp2_plan_graph(plan)
    digest, nnz_sym = _full.graph_digest(adj_ptr, adj_col, s.n)
    P_val = torch.empty(info["nnz_P"], dtype=torch.float32, device="cuda")
    print("oracle: replaying the stored sequence on the three sampled parts", flush=True)
    samples = _full.oracle_sampled_parts(gold, arrays, s, gold["alphas"])
    yield dict(g=g, torch=torch, gold=gold, arrays=arrays, s=s, part=part, plan=plan, info=info, cs=cs, ss=ss,
               col_ptr=col_ptr, P_val=P_val, Hd=Hd, stream=stream, dense_run=dense_run, dense_sketch=dsk,
               digest=digest, nnz_sym=nnz_sym, samples=samples)
    plan.close()


def _run(c, precision="fp32", **kw):
    torch = c["torch"]
    P = c["P_val"] if precision != "fp64" else torch.empty(c["info"]["nnz_P"], dtype=torch.float64, device="cuda")
    with torch.cuda.stream(c["stream"]):
        run = c["g"].gsp2_density(c["plan"], c["Hd"], c["s"].n_occ, P, precision=precision, **kw)
    torch.cuda.synchronize()
    return run, P.cpu().numpy()


def test_fp64_previous_p_is_the_oracles(case):
    """The GPU's FP64 dense SP2 of H against the oracle's: sequence, trace and
    a sketch of the whole 21,000 x 21,000 P."""
    gold, run = case["gold"]["dense_run"], case["dense_run"]
    m = min(len(run["alpha"]), len(gold["alphas"]))
    err = float(np.linalg.norm(case["dense_sketch"] - case["arrays"]["dense_sketch"]) /
                np.linalg.norm(case["arrays"]["dense_sketch"]))
    print(f"dense FP64: products {run['n_products']} / oracle {gold['n_products']}, "
          f"Tr P {run['trace']:.9f} / {gold['trace_P']:.9f}, sketch rel_err {err:.2e}", flush=True)
    assert run["status"] == 0 and run["alpha"][:m] == gold["alphas"][:m]
    assert abs(run["n_products"] - gold["n_products"]) <= 2
    assert abs(run["trace"] - gold["trace_P"]) <= 1e-9 * case["s"].n
    assert err <= TOL64


def test_graph_and_plan_are_the_oracles(case):
    gold = case["gold"]
    print(f"graph: {case['nnz_sym']} entries (oracle {gold['graph']['nnz_sym']}); "
          f"s in [{case['info']['min_s']}, {case['info']['max_s']}]", flush=True)
    assert case["nnz_sym"] == gold["graph"]["nnz_sym"] and case["digest"] == gold["graph"]["sha256"]
    assert case["cs"].tolist() == [p["c"] for p in gold["parts"]]
    assert case["ss"].tolist() == [p["s"] for p in gold["parts"]]
    g, plan = case["g"], case["plan"]
    for k, p in enumerate(gold["parts"]):
        assert _full.index_digest(g.gsp2_plan_part_index(plan, k)) == p["idx_sha256"], k


def test_replayed_sequence_matches_oracle(case):
    """FP32 products replaying the oracle's branch sequence: every part's core
    columns against the oracle's (sketch), three parts element by element."""
    gold = case["gold"]
    run, vals = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9)
    assert np.isfinite(vals).all()
    assert abs(run["eps_min"] - gold["eps"][0]) <= 1e-12 * abs(gold["eps"][0])
    assert abs(run["eps_max"] - gold["eps"][1]) <= 1e-12 * abs(gold["eps"][1])
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"all 128 parts: sketch rel_err max {errs.max():.2e}, median {np.median(errs):.2e}", flush=True)
    assert errs.max() <= TOL
    for k, e in _full.sampled_errors(case["samples"], vals, case["col_ptr"], case["part"]).items():
        print(f"part {k} (s={gold['parts'][k]['s']}): element-wise rel_err={e:.2e}", flush=True)
        assert e <= TOL
    assert abs(run["trace"] - gold["traces"][-1]) <= 1e-5 * case["s"].n


def test_trace_mode_run(case):
    """FP32 products taking their own branches.  Where the run parts from the
    oracle's sequence, the two traces must sit on either side of N_occ by no
    more than FP32 rounding moves the trace: at that product the GPU's trace
    differs from the oracle's by more than the oracle's distance to N_occ,
    and by no more than sqrt(N) ||dP||_F (Cauchy-Schwarz over the N diagonal
    entries), ||dP||_F measured on the replayed sequence.  Different branch
    sequences give different (equally valid) G-SP2 results, so P is compared
    with the oracle's only when the sequences agree."""
    gold = case["gold"]
    _, rvals = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9)
    rerr = _full.part_errors(gold, case["arrays"], rvals, case["col_ptr"], case["part"]).max()
    run, vals = _run(case)
    assert run["status"] == 0, run
    n_occ = case["s"].n_occ
    ga, oa = run["alpha"], gold["alphas"]
    m = min(len(ga), len(oa))
    diff = [i for i in range(m) if ga[i] != oa[i]]
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"gpu products {run['n_products']}, oracle {gold['n_products']}; first branch difference "
          f"{diff[0] if diff else None}; Tr P - N_occ = {run['trace'] - n_occ:.3e}; "
          f"parts sketch rel_err max {errs.max():.2e}", flush=True)
    if diff:
        d = diff[0]
        gap = abs(gold["traces"][d] - n_occ)
        dtr = abs(run["traces"][d] - gold["traces"][d])
        bound = np.sqrt(case["s"].n) * rerr * gold["fro_total"]
        print(f"product {d}: oracle |Tr - N_occ| = {gap:.3e}, |Tr_gpu - Tr_oracle| = {dtr:.3e}, "
              f"sqrt(N) ||dP||_F = {bound:.3e}", flush=True)
        assert (run["traces"][d] - n_occ) * (gold["traces"][d] - n_occ) <= 0.0
        assert gap <= dtr <= bound
    else:
        assert errs.max() <= TOL
    assert abs(run["trace"] - gold["traces"][-1]) <= 1e-1


def test_fp64_products_full_size(case):
    gold = case["gold"]
    run, vals = _run(case, precision="fp64", alpha_seq=gold["alphas"], trace_tol=1e9)
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"fp64 replay: parts sketch rel_err max {errs.max():.2e}", flush=True)
    assert run["status"] == 0 and errs.max() <= TOL64


@pytest.mark.parametrize("refine", [0, 2])
def test_fp16_error_vs_oracle(case, refine):
    """FP16 operands (diagonal exact) on the full workload, the oracle's
    sequence replayed: every part at the 16-bit bar, with and without two
    FP32 refinement products."""
    gold = case["gold"]
    run, vals = _run(case, precision="fp16", alpha_seq=gold["alphas"], trace_tol=1e9, refine=refine)
    assert np.isfinite(vals).all()
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    samp = _full.sampled_errors(case["samples"], vals, case["col_ptr"], case["part"])
    print(f"fp16 refine={refine}: parts sketch rel_err max {errs.max():.2e} median {np.median(errs):.2e}; "
          f"sampled " + ", ".join(f"{e:.2e}" for e in samp.values()) +
          f"; Tr P - N_occ = {run['trace'] - case['s'].n_occ:.3e}", flush=True)
    assert errs.max() <= MIXED_TOL and max(samp.values()) <= MIXED_TOL


def test_fp16_trace_mode_full_size(case):
    """FP16 products in trace mode with two FP32 refinement products: the run
    takes its own branches and stop, passes the occupation check, and its P
    meets the 16-bit bar against the oracle's P."""
    gold = case["gold"]
    run, vals = _run(case, precision="fp16", refine=2, check=False)
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"fp16 trace mode: status {run['status_name']}, {run['n_products']} products, "
          f"Tr P - N_occ = {run['trace'] - case['s'].n_occ:.3e}, parts sketch rel_err max {errs.max():.2e}",
          flush=True)
    assert run["status"] == 0 and abs(run["trace"] - case["s"].n_occ) <= 0.5
    assert errs.max() <= MIXED_TOL


@pytest.mark.xfail(strict=True, raises=AssertionError,
                   reason="BF16 products miss the 1e-3 bar at full size (2.4e-3 measured with the oracle's "
                          "sequence replayed; the subspace rotation left by 2^-8 rounding is not undone)")
def test_bf16_error_vs_oracle(case):
    gold = case["gold"]
    run, vals = _run(case, precision="bf16", alpha_seq=gold["alphas"], trace_tol=1e9)
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"bf16: parts sketch rel_err max {errs.max():.2e} median {np.median(errs):.2e}", flush=True)
    assert np.isfinite(vals).all() and errs.max() <= MIXED_TOL


@pytest.mark.parametrize("refine", [0, 2])
@pytest.mark.xfail(strict=True, raises=AssertionError,
                   reason="BF16 in trace mode misses the 1e-3 bar at full size (1.8e-3, and 1.3e-3 with two FP32 "
                          "refinement products, measured)")
def test_bf16_trace_mode_full_size(case, refine):
    """BF16 products in trace mode: the run stops at its own floor (before the
    late products, where BF16 rounding costs most), passes the occupation
    check, and is compared with the oracle's P on every part."""
    gold = case["gold"]
    run, vals = _run(case, precision="bf16", refine=refine, check=False)
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"bf16 trace mode refine={refine}: status {run['status_name']}, {run['n_products']} products, "
          f"Tr P - N_occ = {run['trace'] - case['s'].n_occ:.3e}, parts sketch rel_err max {errs.max():.2e}",
          flush=True)
    assert run["status"] == 0 and abs(run["trace"] - case["s"].n_occ) <= 0.5
    assert errs.max() <= MIXED_TOL


def test_split_fp16_full_size(case):
    """Split FP16 products meet the FP32 bar on every part, replayed and in
    trace mode."""
    gold = case["gold"]
    run, vals = _run(case, precision="fp16x3", alpha_seq=gold["alphas"], trace_tol=1e9)
    errs = _full.part_errors(gold, case["arrays"], vals, case["col_ptr"], case["part"])
    print(f"fp16x3: parts sketch rel_err max {errs.max():.2e}", flush=True)
    assert run["precision"] == 3 and errs.max() <= TOL
    run, vals = _run(case, precision="fp16x3")
    print(f"fp16x3 trace mode: {run['n_products']} products, Tr P - N_occ = {run['trace'] - case['s'].n_occ:.3e}",
          flush=True)
    assert run["status"] == 0 and abs(run["trace"] - gold["traces"][-1]) <= 1e-2


@pytest.mark.skip(reason="persistent product launch switched off: its first GPU run did not return "
                         "within 120 s and the cause has not been established (see the design notes)")
def test_persistent_launch_full_size(case):
    """The full workload with every product in one persistent launch gives the
    same bits as one launch per product."""
    gold = case["gold"]
    _, v1 = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9)
    run, v2 = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9, persistent=True)
    assert run["n_products"] == len(gold["alphas"])
    assert np.array_equal(v1, v2)

"""Full-size G-SP2 on the GPU against the FP64 oracle: 3,500 water molecules
(21,000 orbitals), 128 uneven parts, tau = 1e-5, in the bench's launch
configuration (one HIP graph, FP32 products).

The oracle cannot redo the whole run inside a test, so the stored
expectations (tests/golden/gsp2_water3500_tau1e-5.json, written by
tests/golden/make_full_size_golden.py from the oracle alone) give its branch
sequence and per-part norms and traces; a few parts are recomputed here by
the oracle, one by one, by replaying that sequence, and compared with the
GPU element by element.  The graph comes from the distance-based stand-in
for the previous P, which both sides threshold in FP64."""
import json
import os

import numpy as np
import pytest

import oracle
from synth.locality import surrogate_prev_density
from synth.partition import uneven_spatial_partition
from synth.water import make_water

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "gsp2_water3500_tau1e-5.json")
TOL = 1e-5


@pytest.fixture(scope="module")
def case():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_10016_amd as g
    with open(GOLDEN) as f:
        gold = json.load(f)
    sp = gold["spec"]
    s = make_water(sp["n_mol"], sp["seed"])
    part = uneven_spatial_partition(s, sp["n_parts"], sp["core_lo"], sp["core_hi"], seed=sp["seed"])
    Q = surrogate_prev_density(s, sp["q_floor"])
    print(f"full size: N={s.n} nnz(Q)={Q.nnz}", flush=True)
    stream = torch.cuda.Stream()
    Hd = g.csr_to_device(s.H)
    Qd = g.csr_to_device(Q)
    with torch.cuda.stream(stream):
        plan = g.gsp2_plan_create(Qd, sp["tau"], part, sp["n_parts"], stream=stream)
    info, cs, ss = g.gsp2_plan_query(plan)
    col_ptr, row_idx = g.gsp2_plan_pattern(plan)
    P_val = torch.empty(info["nnz_P"], dtype=torch.float32, device="cuda")
    # the oracle recomputes three parts (smallest, median, largest) by replaying its sequence
    sizes = np.array([p["s"] for p in gold["parts"]])
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    ref = oracle.gsp2(s.H, Q, sp["tau"], part, sp["n_parts"], s.n_occ, alpha_seq=gold["alphas"],
                      parts_subset=pick, trace_tol=1e9)
    yield dict(g=g, torch=torch, gold=gold, s=s, part=part, Q=Q, plan=plan, info=info, cs=cs, ss=ss,
               col_ptr=col_ptr, row_idx=row_idx, P_val=P_val, Hd=Hd, stream=stream, pick=pick, ref=ref,
               sizes=sizes)
    plan.close()


def _sampled_errors(c, vals):
    errs = {}
    for i, k in enumerate(c["pick"]):
        idx, blk = _core_block(c, vals, k)
        assert np.array_equal(idx, c["ref"].index[i])
        errs[k] = np.linalg.norm(blk - c["ref"].core_columns[i]) / np.linalg.norm(c["ref"].core_columns[i])
    return errs


def _run(c, **kw):
    with c["torch"].cuda.stream(c["stream"]):
        run = c["g"].gsp2_density(c["plan"], c["Hd"], c["s"].n_occ, c["P_val"], **kw)
    c["torch"].cuda.synchronize()
    return run, c["P_val"].cpu().numpy()


def _core_block(c, vals, k):
    """Part k's core columns from the GPU's P, rows in the part's local order."""
    g, plan = c["g"], c["plan"]
    idx = g.gsp2_plan_part_index(plan, k)
    core = np.flatnonzero(c["part"] == k)
    order = np.argsort(idx, kind="stable")          # pattern rows are ascending global ids
    blk = np.empty((len(idx), len(core)))
    for jl, j in enumerate(core):
        col = vals[c["col_ptr"][j]:c["col_ptr"][j + 1]]
        blk[order, jl] = col
    return idx, blk


def test_plan_sizes_match_oracle(case):
    gold = case["gold"]
    assert case["cs"].tolist() == [p["c"] for p in gold["parts"]]
    assert case["ss"].tolist() == [p["s"] for p in gold["parts"]]
    print(f"s in [{case['info']['min_s']}, {case['info']['max_s']}]", flush=True)


def test_replayed_sequence_matches_oracle(case):
    gold = case["gold"]
    run, vals = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9)
    assert np.isfinite(vals).all()
    assert abs(run["eps_min"] - gold["eps"][0]) <= 1e-12 * abs(gold["eps"][0])
    assert abs(run["eps_max"] - gold["eps"][1]) <= 1e-12 * abs(gold["eps"][1])
    # every part: Frobenius norm and core trace of its core columns
    fro_err = []
    for k, p in enumerate(gold["parts"]):
        _, blk = _core_block(case, vals, k)
        fro_err.append(abs(np.linalg.norm(blk) - p["fro"]) / p["fro"])
        assert abs(np.trace(blk[:p["c"], :p["c"]]) - p["core_trace"]) <= 1e-5 * p["c"]
    print(f"max per-part |fro - fro_oracle| / fro_oracle = {max(fro_err):.2e}", flush=True)
    assert max(fro_err) <= TOL
    # sampled parts, element by element, against the oracle replaying the sequence
    for k, err in _sampled_errors(case, vals).items():
        print(f"part {k} (s={case['sizes'][k]}): rel_err={err:.2e}", flush=True)
        assert err <= TOL


def test_trace_mode_run(case):
    gold = case["gold"]
    run, vals = _run(case)
    assert run["status"] == 0, run
    assert np.isfinite(vals).all()
    n_occ = case["s"].n_occ
    ga, oa = run["alpha"], gold["alphas"]
    m = min(len(ga), len(oa))
    diff = [i for i in range(m) if ga[i] != oa[i]]
    print(f"gpu products {run['n_products']}, oracle {gold['n_products']}; first branch difference "
          f"{diff[0] if diff else None}; Tr P - N_occ = {run['trace'] - n_occ:.3e}", flush=True)
    if diff:
        d = diff[0]
        assert abs(gold["traces"][d] - n_occ) <= 1e-4 * case["s"].n / 1000.0
    assert abs(run["trace"] - gold["traces"][-1]) <= 1e-2
    # same branches, same bits: a replay of the GPU's own sequence is identical
    if not diff and run["n_alpha"] == len(oa):
        _, vals2 = _run(case, alpha_seq=oa, trace_tol=1e9)
        assert np.array_equal(vals, vals2)


@pytest.mark.parametrize("precision,bar", [("fp16", 3e-3), ("bf16", 3e-2)])
def test_mixed_precision_error_vs_oracle(case, precision, bar):
    """FP16/BF16 product operands on the full workload: the error against the
    FP64 oracle, stated per mode (same replayed sequence), with and without
    two FP32 refinement products."""
    gold = case["gold"]
    for refine in (0, 2):
        run, vals = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9, precision=precision, refine=refine)
        assert np.isfinite(vals).all()
        errs = _sampled_errors(case, vals)
        print(f"{precision} refine={refine}: sampled-part rel_err " +
              ", ".join(f"{e:.2e}" for e in errs.values()) + f"; Tr P - N_occ = {run['trace'] - case['s'].n_occ:.3e}",
              flush=True)
        if refine == 0:
            assert max(errs.values()) <= bar


def test_split_fp16_full_size(case):
    """Split FP16 products (three FP16 products per product) on the full
    workload meet the FP32 bar against the FP64 oracle."""
    gold = case["gold"]
    run, vals = _run(case, alpha_seq=gold["alphas"], trace_tol=1e9, precision="fp16x3")
    assert np.isfinite(vals).all() and run["precision"] == 3
    errs = _sampled_errors(case, vals)
    print("fp16x3: sampled-part rel_err " + ", ".join(f"{e:.2e}" for e in errs.values()) +
          f"; Tr P - N_occ = {run['trace'] - case['s'].n_occ:.3e}", flush=True)
    assert max(errs.values()) <= TOL
    # trace mode: the stop rule fires, as with FP32 products
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

"""GPU (HIP, through the C ABI) against the FP64 oracle on the same inputs.

Bar: ||P_gpu - P_oracle||_F / ||P_oracle||_F <= 1e-5 (FP32 products), index
sets bit-exact, run-to-run bitwise determinism."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth.partition import molecule_partition, uneven_spatial_partition
from tests import _pins as pins

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_10016_amd as g
    g.load()


def _dense_prev(s):
    return pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])


def tie_band(n, s_max=1000):
    """|Tr X - N_occ| below which an FP32 and an FP64 run may take different
    branches: the FP32 trace carries a rounding error that grows with the n
    diagonal entries summed, with the length s of the FP32 sums that form
    each entry, and with the amplification of near-crossover eigenvalues by
    the recursion."""
    return 1e-4 * max(1.0, n / 1000.0) * max(1.0, s_max / 1000.0)


def _check_parity(s, tau, n_parts, part=None, **kw):
    """Trace-mode GPU run against the oracle.  Where the two branch
    sequences agree, P is unique and must match.  If they part, the first
    difference must be a near-tie of the trace rule (both branches valid);
    the GPU's arithmetic is then checked by replaying the oracle's sequence."""
    from tests._gpu import rel_fro, run_gsp2
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, n_parts, seed=0) if part is None else part
    ref = oracle.gsp2(s.H, Pp, tau, part, n_parts, s.n_occ)
    P, run, info, index, vals = run_gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, **kw)
    print(f"N={s.n} parts={n_parts} tau={tau} s=[{min(ref.sizes)},{max(ref.sizes)}] "
          f"gpu products={run['n_products']} oracle products={ref.sp2.n_products}", flush=True)
    assert run["status"] == 0, run
    assert np.isfinite(vals).all()
    for k in range(n_parts):
        assert np.array_equal(index[k], ref.index[k]), k
    ga, oa = run["alpha"], ref.sp2.alphas
    m = min(len(ga), len(oa))
    diff = [i for i in range(m) if ga[i] != oa[i]]
    if diff:
        d = diff[0]
        gap = abs(ref.sp2.traces[d] - s.n_occ)
        band = tie_band(s.n, max(ref.sizes))
        print(f"  branch sequences part at product {d}: |Tr - N_occ| = {gap:.2e} (band {band:.1e})", flush=True)
        assert gap <= band, (d, gap)
        P, run2, _, _, _ = run_gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, alpha_seq=oa, trace_tol=1e9, **kw)
    err = rel_fro(P, ref.csc())
    print(f"  rel_err={err:.3e}", flush=True)
    assert err <= TOL, err
    return P, run, ref


def test_tiny_config_dense_threshold():
    # 64 molecules, 384 orbitals, 8 uneven parts, tau = 1e-5 (halos cover nearly all)
    _check_parity(pins.water(64, 0), 1e-5, 8)


@pytest.mark.parametrize("tau", [1e-3, 1e-2])
def test_tiny_config_truncated_halos(tau):
    _check_parity(pins.water(64, 0), tau, 8)


def test_several_tiles_and_ragged_tail():
    # 200 molecules: sub-problems of several 128-tiles with a ragged last tile
    _check_parity(pins.water(200, 1), 1e-4, 6)


def test_single_part_is_dense_sp2():
    s = pins.water(48, 2)
    part = np.zeros(s.n, dtype=np.int32)
    P, run, ref = _check_parity(s, 1e-5, 1, part=part)
    Ps = oracle.eig_projector(s.H, s.n_occ)
    from tests._gpu import rel_fro
    assert rel_fro(P, Ps) <= TOL


def test_fp32_inputs():
    import torch
    _check_parity(pins.water(64, 1), 1e-3, 8, h_dtype=torch.float32, p_dtype=torch.float32)


def test_monomers_exact():
    s = pins.water(40, 3, hop_a=0.0)
    part = molecule_partition(s)
    from tests._gpu import rel_fro, run_gsp2
    P, run, info, index, vals = run_gsp2(s.H, s.H, 1e-5, part, s.n_mol, s.n_occ)
    assert run["status"] == 0 and info["max_s"] == 6
    assert rel_fro(P, oracle.eig_projector(s.H, s.n_occ)) <= TOL


def test_bitwise_deterministic():
    from tests._gpu import run_gsp2
    s = pins.water(64, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 8, seed=0)
    a = run_gsp2(s.H, Pp, 1e-3, part, 8, s.n_occ)[4]
    b = run_gsp2(s.H, Pp, 1e-3, part, 8, s.n_occ)[4]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("seq", [[], [-1], [1], [-1, 1, -1]])
def test_replayed_prefix_matches_oracle(seq):
    # replaying a fixed branch prefix isolates the stages: no product (gather
    # and scatter of eq. (1)), then one or a few products of eq. (2)
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(100, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 3, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=seq)
    P, run, info, index, vals = run_gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=seq, trace_tol=1e9)
    err = rel_fro(P, ref.csc())
    print(f"replay {seq}: rel_err={err:.3e} eps=({run['eps_min']:.6f},{run['eps_max']:.6f}) "
          f"oracle eps={ref.eps}", flush=True)
    assert abs(run["eps_min"] - ref.eps[0]) <= 1e-12 * abs(ref.eps[0])
    assert abs(run["eps_max"] - ref.eps[1]) <= 1e-12 * abs(ref.eps[1])
    assert err <= TOL, err


def test_small_system_near_tie_branch():
    # 32 molecules, 4 parts, tau = 1e-3: the trace lands within FP32 rounding
    # of N_occ late in the run, so the branch sequences may part there
    _check_parity(pins.water(32, 0), 1e-3, 4)


# Mixed precision: FP16/BF16 operands, FP32 accumulation and master iterate,
# the diagonal of X taken exactly in FP32.  The bar is the stated one for
# 16-bit products before refinement, 1e-3 against the FP64 oracle.  FP16
# meets it.  BF16 does not: one product alone costs 2.4e-3 (2^-8 relative
# rounding of the off-diagonal operand), and each rounded product leaves a
# rotation of the occupied subspace that purification does not undo.  CPU
# emulation puts most of it in the products after the occupation has
# settled: with the oracle's sequence replayed, BF16 for all but the last
# four products of 28 gives 6.8e-4, all of them 3.4e-3 (100 molecules).  A
# BF16 run in trace mode stops at its own floor before those products, and
# lands at 1.4e-3 (6.6e-4 with two FP32 refinement products) at 100
# molecules, but 1.8e-3 (1.3e-3 refined) on the 21,000-orbital workload.
# Its tests against the bar are expected failures, so a BF16 result that met
# it would be reported.
MIXED_TOL = 1e-3
BF16_MISSES = pytest.mark.xfail(strict=True, raises=AssertionError,
                                reason="BF16 products miss the 1e-3 bar (1.3e-3 to 2.4e-3 measured against the "
                                       "oracle on the full workload; the subspace rotation left by 2^-8 rounding "
                                       "is not undone by purification)")


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_mixed_precision_one_product(precision):
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(100, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 3, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=[-1])
    P, run, _, _, _ = run_gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=[-1], trace_tol=1e9,
                               precision=precision)
    err = rel_fro(P, ref.csc())
    print(f"{precision} one product: rel_err={err:.2e}", flush=True)
    unit = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}[precision]
    assert run["precision"] == {"fp16": 1, "bf16": 2}[precision]
    assert err <= 4 * unit


@pytest.mark.parametrize("precision", ["fp16", "bf16", "fp16x3"])
def test_16bit_one_update_product(precision):
    # one X' = 2X - X^2 product: the 16-bit epilogue reads X_old at the
    # mirrored position and applies the update; the parts' padded sizes are
    # 5, 5 and 4 times 128, so 256-wide tiles with a half-empty last row and
    # column are exercised next to full ones
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(100, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 3, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=[1])
    P, run, _, index, _ = run_gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=[1], trace_tol=1e9,
                                   precision=precision)
    pads = sorted(-(-len(ix) // 128) for ix in index)
    assert any(p % 2 for p in pads) and any(p % 2 == 0 for p in pads), pads
    err = rel_fro(P, ref.csc())
    print(f"{precision} one update product: rel_err={err:.2e}, s_pad/128 = {pads}", flush=True)
    unit = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "fp16x3": 2.0 ** -22}[precision]
    assert run["alpha"][:1] == [1]
    assert err <= 4 * unit


@pytest.mark.parametrize("precision", ["fp16", pytest.param("bf16", marks=BF16_MISSES)])
def test_mixed_precision_trace_mode(precision):
    # trace mode: the run's own branches, stop and occupation check
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(200, 1)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 6, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ)
    out = {}
    for refine in (0, 2):
        P, run, _, _, vals = run_gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ, precision=precision, refine=refine,
                                      check=False)
        assert np.isfinite(vals).all()
        out[refine] = rel_fro(P, ref.csc())
        print(f"{precision} refine={refine}: status {run['status_name']} products={run['n_products']} "
              f"rel_err={out[refine]:.2e} |Tr P - N_occ|={abs(run['trace'] - s.n_occ):.2e}", flush=True)
        assert run["status"] == 0 and run["n_refine"] == refine, run
    assert out[0] <= MIXED_TOL and out[2] <= MIXED_TOL
    assert out[2] <= 1.05 * out[0]           # a purification pair cannot undo the subspace error, nor add to it


@pytest.mark.parametrize("precision", ["fp16", pytest.param("bf16", marks=BF16_MISSES), "fp16x3"])
def test_16bit_products_on_128_tiles(precision):
    # the tile autotuner's other candidates: 16-bit products on 128 x 128
    # tiles (every block formed, or padding and mirror blocks skipped) meet
    # the same bars as on 256 x 256 tiles, against the oracle
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(200, 1)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 6, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ)
    bar = {"fp16": MIXED_TOL, "bf16": MIXED_TOL, "fp16x3": 1e-5}[precision]
    errs = {}
    for form in ("t128", "t128_skip", "t256"):
        P, run, _, _, vals = run_gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ, precision=precision, kernel=form)
        assert run["status"] == 0 and np.isfinite(vals).all(), run
        errs[form] = rel_fro(P, ref.csc())
    print(f"{precision}: rel_err " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) <= bar


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16", "fp16x3", "fp64"])
@pytest.mark.parametrize("n_mol,seed,n_parts,tau", [(64, 0, 8, 1e-3), (200, 1, 6, 1e-4), (8, 0, 8, 1e-2)])
def test_skip_form_gives_the_same_bits(precision, n_mol, seed, n_parts, tau):
    # the skipped 32 x 32 blocks lie wholly in the zero padding or below the
    # diagonal of a diagonal tile (transposes of formed ones), and a block
    # formed by another wave is formed alike, so the two 128-tile forms give
    # the same P, branch sequence and traces bit for bit (8 molecules in 8
    # parts: 6-orbital cores padded to 128, where all but one 32-row block is
    # padding).  The skip form's diagonal tiles also stage only their A panel
    # and read B fragments from it, while the plain form stages both, so the
    # bit equality covers that path too.  Split FP16 is the exception: a block above the diagonal sums
    # its two cross terms in the other order than the block below it, so the
    # two forms agree to FP32 rounding.
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(n_mol, seed)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, n_parts, seed=0)
    out = {}
    for form in ("t128", "t128_skip"):
        P, run, _, _, vals = run_gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, precision=precision, kernel=form)
        assert run["status"] == 0 and np.isfinite(vals).all(), run
        out[form] = (vals, run)
    v0, r0 = out["t128"]
    v1, r1 = out["t128_skip"]
    if precision == "fp16x3":
        assert r0["alpha"] == r1["alpha"]
        assert np.allclose(r0["traces"], r1["traces"], rtol=0.0, atol=1e-6 * s.n)
        assert np.linalg.norm(v0 - v1) <= 1e-6 * np.linalg.norm(v0)
    else:
        assert r0["alpha"] == r1["alpha"] and r0["traces"] == r1["traces"]
        assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32))
    if precision in ("fp32", "fp16x3", "fp64"):
        ref = oracle.gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, alpha_seq=r1["alpha"])
        err = rel_fro(P, ref.csc())
        print(f"{precision} {n_mol} mol: skip form vs oracle {err:.2e}", flush=True)
        assert err <= (1e-10 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision,published", [("fp32", 157.3), ("fp16", 2500.0), ("bf16", 2500.0)])
def test_mfma_probe_rate_is_plausible(precision, published):
    # back-to-back MFMAs reach most of the published dense peak, and not more
    # than the peak at the top clock allows
    import paper_1801_10016_amd as g
    rate = g.gsp2_probe_mfma(precision)
    print(f"{precision}: measured {rate:.1f} TFLOP/s of {published}", flush=True)
    assert 0.6 * published < rate < 1.05 * published


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp64"])
def test_tile_autotuner_choice_is_used(precision):
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(200, 1)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 6, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ)
    P, run, _, _, _ = run_gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ, precision=precision, tune=precision)
    rec = run["tune"]
    print(f"tuner: {rec}", flush=True)
    want = {"fp32": {"t128", "t128_skip"}, "fp64": {"t128", "t128_skip"},
            "fp16": {"t128", "t128_skip", "t256"}}[precision]
    assert set(rec["ms_per_product"]) == want and rec["n_products"] == 4
    assert all(v > 0 for v in rec["ms_per_product"].values())
    # the fastest form, unless it is within 1% of the default (which then stays)
    ms = rec["ms_per_product"]
    default = {"fp32": "t128_skip", "fp64": "t128_skip", "fp16": "t256"}[precision]
    fastest = min(ms, key=ms.get)
    assert rec["chosen"] == (fastest if ms[fastest] < 0.99 * ms[default] else default)
    bar = {"fp32": 1e-5, "fp64": 1e-10}.get(precision, MIXED_TOL)
    assert run["status"] == 0 and rel_fro(P, ref.csc()) <= bar


def test_kernel_form_is_checked():
    # forms a precision does not have are refused before any work
    import torch
    import paper_1801_10016_amd as g
    from paper_1801_10016_amd.gsp2 import GSP2_E_INVALID
    s = pins.water(16, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 2, seed=0)
    Hd = g.csr_to_device(s.H)
    with g.gsp2_plan_create(g.csr_to_device(sp.csr_matrix(Pp)), 1e-3, part, 2) as plan:
        P32 = torch.empty(plan.nnz_P, dtype=torch.float32, device="cuda")
        P64 = torch.empty(plan.nnz_P, dtype=torch.float64, device="cuda")
        for prec, form, out in (("fp32", "t256", P32), ("fp64", "t256", P64), ("fp32", 7, P32)):
            with pytest.raises(g.Gsp2Error) as e:
                g.gsp2_density(plan, Hd, s.n_occ, out, precision=prec, kernel=form)
            assert e.value.status == GSP2_E_INVALID
        with pytest.raises(g.Gsp2Error) as e:
            g.gsp2_plan_tune(plan, Hd, s.n_occ, "fp32", n_products=1)
        assert e.value.status == GSP2_E_INVALID


@pytest.mark.parametrize("n_mol,seed,n_parts,tau", [(64, 0, 8, 1e-5), (200, 1, 6, 1e-4)])
def test_split_fp16_products_meet_the_fp32_bar(n_mol, seed, n_parts, tau):
    # three FP16 products with the operand split X = A + 2^-11 B: the FP32 bar applies
    P, run, ref = _check_parity(pins.water(n_mol, seed), tau, n_parts, precision="fp16x3")
    assert run["precision"] == 3


def test_split_fp16_one_product():
    # one product isolates the operand split: its error is that of FP32 products
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(100, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 3, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=[-1])
    errs = {}
    for prec in ("fp32", "fp16x3"):
        P, run, _, _, _ = run_gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, alpha_seq=[-1], trace_tol=1e9, precision=prec)
        errs[prec] = rel_fro(P, ref.csc())
    print(f"one product: fp32 {errs['fp32']:.2e}, split fp16 {errs['fp16x3']:.2e}", flush=True)
    assert errs["fp16x3"] <= 4 * 2.0 ** -22


def test_refinement_products_do_not_drift():
    # 24 molecules, 3 parts: after the FP16 stop the trace sits above n_occ, so
    # branches taken by the trace rule would square towards one side only;
    # alternating pairs keep every eigenvalue at the nearer of 0 and 1
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(24, 3)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 3, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ)
    err = {}
    for refine in (0, 2, 8):
        P, run, _, _, _ = run_gsp2(s.H, Pp, 1e-3, part, 3, s.n_occ, precision="fp16", refine=refine)
        assert run["status"] == 0 and run["n_refine"] == refine
        err[refine] = rel_fro(P, ref.csc())
        n = run["n_alpha"]
        print(f"fp16 refine={refine}: rel_err={err[refine]:.2e} branches after the stop "
              f"{run['alpha'][n - refine:]} |Tr P - N_occ|={abs(run['trace'] - s.n_occ):.2e}", flush=True)
        assert run["alpha"][n - refine:] == [-1, 1] * (refine // 2)
    assert err[8] <= 1.05 * err[2] and err[2] <= MIXED_TOL


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_split_fp16_refinement_products(precision):
    # refinement products with split-FP16 operands after 16-bit products:
    # FP32-grade products, so the result agrees with FP32 refinement products
    # to FP32 rounding and meets the same bar against the oracle; in trace
    # mode and with the oracle's sequence replayed, on 128 and 256 tiles
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(200, 1)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 6, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ)
    for kw in ({}, {"alpha_seq": ref.sp2.alphas, "trace_tol": 1e9}, {"kernel": "t128"}):
        out = {}
        for rp in ("fp32", "fp16x3"):
            P, run, _, _, vals = run_gsp2(s.H, Pp, 1e-4, part, 6, s.n_occ, precision=precision, refine=2,
                                          refine_precision=rp, check=False, **kw)
            assert run["status"] == 0 and run["n_refine"] == 2 and np.isfinite(vals).all(), run
            out[rp] = (P, run)
        gap = rel_fro(out["fp16x3"][0], out["fp32"][0])
        errs = {rp: rel_fro(P, ref.csc()) for rp, (P, _) in out.items()}
        print(f"{precision} {kw.get('kernel', 'auto')} {'replay' if kw.get('alpha_seq') else 'trace'}: split vs FP32 "
              f"refinement {gap:.2e}; vs oracle {errs['fp32']:.2e} / {errs['fp16x3']:.2e}", flush=True)
        assert out["fp16x3"][1]["alpha"] == out["fp32"][1]["alpha"]
        assert gap <= 1e-5
        assert abs(errs["fp16x3"] - errs["fp32"]) <= 1e-5
        if precision == "fp16":
            assert errs["fp16x3"] <= MIXED_TOL


def test_split_refinement_needs_16bit_products():
    import torch
    import paper_1801_10016_amd as g
    from paper_1801_10016_amd.gsp2 import GSP2_E_INVALID
    s = pins.water(16, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 2, seed=0)
    Hd = g.csr_to_device(s.H)
    with g.gsp2_plan_create(g.csr_to_device(sp.csr_matrix(Pp)), 1e-3, part, 2) as plan:
        P32 = torch.empty(plan.nnz_P, dtype=torch.float32, device="cuda")
        for prec, rp in (("fp32", "fp16x3"), ("fp16x3", "fp16x3"), ("fp16", "bf16")):
            with pytest.raises(g.Gsp2Error) as e:
                g.gsp2_density(plan, Hd, s.n_occ, P32, precision=prec, refine=2, refine_precision=rp)
            assert e.value.status == GSP2_E_INVALID


def test_fp32_refinement_products():
    # refine FP32 products after the FP32 stop: the iterate stays at the oracle's result
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(64, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 8, seed=0)
    ref = oracle.gsp2(s.H, Pp, 1e-5, part, 8, s.n_occ)
    P, run, _, _, _ = run_gsp2(s.H, Pp, 1e-5, part, 8, s.n_occ, refine=2)
    print(f"fp32 refine=2: products={run['n_products']} rel_err={rel_fro(P, ref.csc()):.2e}", flush=True)
    assert run["status"] == 0 and run["n_refine"] == 2
    assert rel_fro(P, ref.csc()) <= TOL



def test_persistent_request_is_refused():
    # the persistent product launch is switched off; asking for it is an error, not a launch
    import paper_1801_10016_amd as g
    from tests._gpu import run_gsp2
    s = pins.water(16, 0)
    part = np.zeros(s.n, dtype=np.int32)
    with pytest.raises(g.Gsp2Error) as e:
        run_gsp2(s.H, s.H, 1e-5, part, 1, s.n_occ, persistent=True)
    assert e.value.status == 6          # GSP2_E_UNSUPPORTED


def test_plan_graph_is_the_threshold_graph():
    # the graph the GPU built, exported from the plan, is the oracle's G_tau
    import paper_1801_10016_amd as g
    s = pins.water(64, 0)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 8, seed=0)
    with g.gsp2_plan_create(g.csr_to_device(sp.csr_matrix(Pp)), 1e-3, part, 8) as plan:
        adj_ptr, adj_col = g.gsp2_plan_graph(plan)
        info, _, _ = g.gsp2_plan_query(plan)
    A = sp.csr_matrix((np.ones(adj_col.size), adj_col, adj_ptr), shape=(s.n, s.n))
    ref = oracle.threshold_graph(Pp, 1e-3)
    assert info["nnz_graph"] == adj_col.size
    assert ((A + A.T) != 0).toarray().tolist() == (ref != 0).toarray().tolist()


def test_annealed_partition_runs_and_matches_its_cost():
    # f4: the plan's graph, refined by simulated annealing for eq. (4), feeds a
    # new plan: its sum of s^3 is the annealer's cost, and P matches the oracle
    import paper_1801_10016_amd as g
    s = pins.water(200, 1)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 6, seed=0)
    Pd = g.csr_to_device(sp.csr_matrix(Pp))
    with g.gsp2_plan_create(Pd, 1e-4, part, 6) as plan:
        adj_ptr, adj_col = g.gsp2_plan_graph(plan)
        before = g.gsp2_plan_query(plan)[0]["sum_s3"]
    new, c0, c1 = g.gsp2_partition_anneal(adj_ptr, adj_col, part, 6, seed=3)
    print(f"annealed: C {c0} -> {c1} ({c1 / c0:.3f})", flush=True)
    assert c0 == before and c1 <= c0
    with g.gsp2_plan_create(Pd, 1e-4, new, 6) as plan:
        assert g.gsp2_plan_query(plan)[0]["sum_s3"] == c1
    _check_parity(s, 1e-4, 6, part=new)


@pytest.mark.parametrize("which", ["empty", "full"])
def test_degenerate_occupations(which):
    # N_occ = 0 gives P = 0, N_occ = N gives P = I on P's pattern (one branch
    # repeated until the trace reaches N_occ, where a tie takes 2X - X^2,
    # which leaves 0 and I in place); the oracle agrees
    from tests._gpu import run_gsp2
    s = pins.water(32, 1)
    Pp = _dense_prev(s)
    part = uneven_spatial_partition(s, 4, seed=0)
    n_occ = 0.0 if which == "empty" else float(s.n)
    ref = oracle.gsp2(s.H, Pp, 1e-3, part, 4, n_occ)
    P, run, _, _, vals = run_gsp2(s.H, Pp, 1e-3, part, 4, n_occ)
    print(f"{which}: {run['n_products']} products, branches {run['alpha']}, Tr P = {run['trace']:.3e}", flush=True)
    assert run["status"] == 0
    if which == "full":
        assert set(run["alpha"]) == {1}
    want = ref.csc().toarray()
    assert np.abs(P.toarray() - want).max() <= 1e-5
    assert abs(run["trace"] - n_occ) <= 1e-4 * max(1.0, n_occ)


def test_one_core_vertex_per_part():
    # every part is a single core orbital with its halo: many tiny blocks,
    # each padded to one 128 tile
    s = pins.water(12, 4)
    part = np.arange(s.n, dtype=np.int32)
    _check_parity(s, 1e-3, s.n, part=part)


def test_largest_checked_single_block():
    # one part of 3,000 orbitals: a 24 x 24 grid of 128-tiles in one block,
    # against the oracle's dense SP2
    s = pins.water(500, 0)
    part = np.zeros(s.n, dtype=np.int32)
    P, run, ref = _check_parity(s, 1e-5, 1, part=part)


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_one_large_part_beside_small_ones(precision):
    # a part holding more than half an XCD's share of the product work (a
    # sixteenth of it) is dealt to the XCDs block by block while the other
    # parts go whole: tile lists of both kinds in one plan, for 128- and
    # 256-wide tiles.  200 molecules in 48 uneven parts, the first 16 joined:
    # 33 parts, of which only the joined one (s = 1,043) is split.
    from oracle.graph import core_halo, threshold_graph
    s = pins.water(200, 1)
    part = uneven_spatial_partition(s, 48, seed=0)
    part = np.where(part < 16, 0, part - 15).astype(np.int32)
    cores, halos = core_halo(threshold_graph(_dense_prev(s), 1e-3), part, 33)
    nt = -(-np.array([len(c) + len(h) for c, h in zip(cores, halos)]) // 128)
    work = nt * (nt + 1) / 2 * nt
    assert np.flatnonzero(work > work.sum() / 16).tolist() == [0], work
    _check_parity(s, 1e-3, 33, part=part, precision=precision)


def test_plan_from_the_sparse_first_p():
    # the first P by thresholded sparse SP2 on the host, thresholded into the
    # plan's graph, then G-SP2 on the GPU: against the oracle's G-SP2 on the
    # oracle's own thresholded first P
    from tests._gpu import rel_fro, run_gsp2
    import paper_1801_10016_amd as g
    s = pins.water(100, 0)
    P_first, info = g.gsp2_sparse_sp2_host(s.H, s.n_occ, 1e-7)
    Po_first, _ = oracle.thresholded_sp2(s.H, s.n_occ, 1e-7)
    part = uneven_spatial_partition(s, 6, seed=0)
    ref = oracle.gsp2(s.H, Po_first, 1e-4, part, 6, s.n_occ)
    P, run, _, index, _ = run_gsp2(s.H, P_first.toarray(), 1e-4, part, 6, s.n_occ, alpha_seq=ref.sp2.alphas,
                                   trace_tol=1e9)
    for k in range(6):
        assert np.array_equal(index[k], ref.index[k]), k
    err = rel_fro(P, ref.csc())
    print(f"first P: {info['n_products']} host products, nnz {P_first.nnz}; G-SP2 rel_err {err:.2e}", flush=True)
    assert run["status"] == 0 and err <= TOL


def test_dense_block_beyond_the_lds_index_list():
    # a single part of 9,000 orbitals: the gather's vertex list no longer fits
    # LDS (8,192 entries) and is read from global memory.  No oracle runs at
    # this size: the result is checked by properties of the projector,
    # computed in FP64 on the GPU: trace, idempotency, commutation with H
    import torch
    import paper_1801_10016_amd as g
    s = pins.water(1500, 0)
    n = s.n
    part = np.zeros(n, dtype=np.int32)
    Hd = g.csr_to_device(s.H)
    with g.gsp2_plan_create(Hd, 0.0, part, 1) as plan:
        assert g.gsp2_plan_query(plan)[0]["max_s"] == n > 8192
        P_val = torch.empty(n * n, dtype=torch.float32, device="cuda")
        run = g.gsp2_density(plan, Hd, s.n_occ, P_val)
        torch.cuda.synchronize()
    P = P_val.double().view(n, n).t()          # CSC of one part: column j holds all rows in order
    H = torch.as_tensor(s.H.toarray(), device="cuda")
    tr = float(torch.trace(P))
    idem = float(torch.linalg.matrix_norm(P @ P - P) / torch.linalg.matrix_norm(P))
    comm = float(torch.linalg.matrix_norm(H @ P - P @ H) / (torch.linalg.matrix_norm(H) * torch.linalg.matrix_norm(P)))
    print(f"N={n}: {run['n_products']} products, Tr P - N_occ = {tr - s.n_occ:.2e}, "
          f"|P^2 - P|/|P| = {idem:.2e}, |[H,P]|/(|H||P|) = {comm:.2e}", flush=True)
    assert run["status"] == 0
    assert abs(tr - s.n_occ) <= 1e-2
    assert idem <= 1e-4 and comm <= 1e-5


def test_non_finite_or_flat_h_is_rejected():
    import paper_1801_10016_amd as g
    from tests._gpu import run_gsp2
    s = pins.water(16, 0)
    part = np.zeros(s.n, dtype=np.int32)
    bad = s.H.tocsr().copy()
    bad.data[3] = np.nan
    with pytest.raises(g.Gsp2Error) as e:
        run_gsp2(bad, s.H, 1e-5, part, 1, s.n_occ)
    assert e.value.status == 1 and "Gershgorin" in str(e.value)
    flat = sp.identity(s.n, format="csr") * 2.0          # eps_max == eps_min
    with pytest.raises(g.Gsp2Error) as e:
        run_gsp2(flat, s.H, 1e-5, part, 1, s.n_occ)
    assert e.value.status == 1

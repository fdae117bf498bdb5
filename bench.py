#!/usr/bin/env python3
"""Time per G-SP2 density matrix on one MI355X.

Workload (defaults): 3,500 synthetic water molecules (21,000 orbitals,
14,000 occupied states), 128 spatial parts of uneven size (cores drawn
U[60, 300] orbitals), graph of the previous P thresholded at tau = 1e-5.
The previous P is the regular (dense, single-part) SP2 density matrix of
the same H, computed by the library beforehand; it is thresholded on the
GPU when the plan is built.  Plan construction is timed separately: the
paper reuses a partition over several MD steps.

A step is one density matrix: Gershgorin bounds, gather of every core+halo
block with eq. (1), every SP2 product with its trace/branch/stop control,
and the scatter of core columns into P, replayed from one HIP graph with H
and P resident in HBM.  Prints one JSON line on stdout; progress goes to
stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "fp16": 2500.0, "bf16": 2500.0, "fp16x3": 2500.0,
                    "fp64": 78.6}                                  # dense, per operand format
MFMA_PRODUCTS = {"fp32": 1, "fp16": 1, "bf16": 1, "fp16x3": 3, "fp64": 1}   # matrix-core products per SP2 product
DTYPE = {"fp32": "f32", "fp16": "f16", "bf16": "bf16", "fp16x3": "f16x3", "fp64": "f64"}
PEAK_HBM_GBS = 8000.0
METRIC = "ms per density matrix P + batched-GEMM TFLOP/s (frac. of MFMA peak) at 10k atoms"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-mol", type=int, default=3500)
    ap.add_argument("--n-parts", type=int, default=128)
    ap.add_argument("--core-lo", type=float, default=60.0)
    ap.add_argument("--core-hi", type=float, default=300.0)
    ap.add_argument("--tau", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=60)
    ap.add_argument("--graph", choices=["dense-sp2", "surrogate"], default="dense-sp2",
                    help="previous P: regular SP2 on the GPU, or the distance-based stand-in")
    ap.add_argument("--cpu-sample-parts", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--save-state", help="write the thresholded graph and product count to this .npz")
    ap.add_argument("--load-state", help="reuse a graph and product count saved by --save-state "
                    "(skips the previous-P computation and the first, stop-finding run)")
    ap.add_argument("--precision", choices=["fp32", "fp16", "bf16", "fp16x3", "fp64"], default=None,
                    help="operand precision of the timed products (default: fp32, or fp16 for batch16)")
    ap.add_argument("--variant-tau", type=float, default=1e-3,
                    help="also time the same P thresholded at this tau (sub-problems in the 400-1,600 range); 0: skip")
    ap.add_argument("--variant-steps", type=int, default=5)
    ap.add_argument("--compare-precisions", default="fp16,bf16,fp16x3,fp64",
                    help="after the FP32 timing, also time these operand precisions (empty: none)")
    ap.add_argument("--compare-steps", type=int, default=3)
    ap.add_argument("--no-library-compare", action="store_true",
                    help="skip timing the same sub-matrix products with torch.matmul (rocBLAS / hipBLASLt)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the kernel autotuner (gsp2_plan_tune) and use the default forms: 128 x 128 "
                         "tiles for FP32 products, 256 x 256 for 16-bit ones")
    ap.add_argument("--kernel", choices=["auto", "t128", "t128_skip", "t256"], default="auto",
                    help="product-kernel form of the headline precision when the autotuner is skipped "
                         "(--no-tune); auto = the library's default form")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (HBM counter calibration)")
    ap.add_argument("--workload", choices=["water3500", "batch16", "backward1000"], default="water3500",
                    help="water3500: one system (the default line); batch16: 16 independent systems of "
                    "500-8,000 molecules, each one MD step on, in one batched plan; backward1000: forward "
                    "and reverse mode on 1,000 molecules, 32 parts, tau = 1e-3")
    ap.add_argument("--refine", type=int, default=None,
                    help="refinement products after the stop (default: 0, or 2 for batch16)")
    ap.add_argument("--refine-precision", choices=["fp32", "fp16x3"], default="fp32",
                    help="operands of the refinement products (fp16x3: split FP16, after 16-bit products only)")
    ap.add_argument("--no-alone", action="store_true", help="batch16: skip timing each system in a plan of its own")
    return ap.parse_args()


def dense_bootstrap(g, torch, Hd, n, n_occ, stream):
    """Regular SP2 on the whole H (one part, no halo) with FP64 products, the
    arithmetic of the paper's runs -> previous P as a device CSR (FP64)."""
    part = np.zeros(n, dtype=np.int32)
    with torch.cuda.stream(stream):
        with g.gsp2_plan_create(Hd, 0.0, part, 1, stream=stream) as plan:
            info, _, _ = g.gsp2_plan_query(plan)
            assert info["nnz_P"] == n * n
            P = torch.empty(n * n, dtype=torch.float64, device="cuda")
            run = g.gsp2_density(plan, Hd, n_occ, P, precision="fp64")
            torch.cuda.synchronize()
    # with a single part every column holds all n rows in ascending order
    col_ptr = torch.arange(0, n * n + 1, n, dtype=torch.int64, device="cuda")
    row_idx = torch.arange(n, dtype=torch.int32, device="cuda").repeat(n)
    return g.DeviceCSR(n, col_ptr, row_idx, P), run


def kernel_name(precision, form):
    """Name of the product kernel that runs `precision` in the tuner's `form`."""
    if precision == "fp64":
        return "k_sp2_step64"
    if form == "t256" or (form == "auto" and precision != "fp32"):
        return "k_sp2_wide"
    # the library's untuned FP32 form is the skip form
    return "k_sp2_step_skip" if form in ("t128_skip", "auto") else "k_sp2_step"


def counter_traffic(precision, workload, kernel):
    """HBM bytes per launch of the product kernel `kernel` at `precision` from
    the committed rocprofv3 counter record, or None when the record holds no
    such kernel, was taken on another workload (molecules, parts, tau, sum of
    s^3), or the kernel or planner sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_sp2_step_counters.json")
    try:
        rec = json.load(open(path))[f"{precision}/{kernel}"]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("match") != workload:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def library_products(torch, stream, sizes, gemm_flops, ours_ms, reps=3):
    """The products of one SP2 product step done by the vendor GEMM instead:
    torch.matmul (rocBLAS / hipBLASLt) of every sub-matrix with itself, the
    full s_k x s_k result, without the fused update, trace partials or
    symmetry.  Random operands of the same sizes; median of `reps` timed
    passes over all parts, after one untimed pass.  A comparison only: no
    result of it is used."""
    dtypes = {"fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}
    out = {"what": "torch.matmul of each s_k x s_k sub-matrix with itself (full product, no update), "
                   "all parts of one product step, event-timed on the bench stream"}
    for prec, dt in dtypes.items():
        gen = torch.Generator(device="cuda").manual_seed(0)
        with torch.cuda.stream(stream):
            A = [torch.randn(s, s, device="cuda", dtype=dt, generator=gen) / s for s in sizes]
            Y = [torch.empty(s, s, device="cuda", dtype=dt) for s in sizes]
            for a, y in zip(A, Y):
                torch.matmul(a, a, out=y)
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for a, y in zip(A, Y):
                    torch.matmul(a, a, out=y)
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
        ms = statistics.median(times)
        rec = {"ms_per_product": round(ms, 3), "full_gemm_tflops": round(gemm_flops / (ms * 1e-3) / 1e12, 1)}
        if prec in ours_ms:
            rec["product_kernel_ms"] = round(ours_ms[prec], 4)
            rec["library_over_kernel"] = round(ms / ours_ms[prec], 3)
        out[prec] = rec
        del A, Y
        torch.cuda.empty_cache()
    return out


def copy_probe(torch, gib):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    n = int(gib * 2**30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "copies": 3}))
    return 0


def host_cores():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info() if p.get("internal_api") == "openblas"]
                   or [os.cpu_count() or 1])
    except Exception:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((line.split(":", 1)[1].strip() for line in f if line.startswith("model name")), "unknown")
    except OSError:
        return "unknown"


def cpu_baseline(system, index, cores, alphas, budget_flop=6e12, whole=False):
    """Time the FP64 oracle's SP2 products (numpy/OpenBLAS) on parts of the
    benched plan: sub-problems built by the oracle from H with the plan's own
    index lists, the run's branch sequence replayed.  `whole`: every part;
    otherwise parts spread over the size range, within about budget_flop of
    work, and the time scaled by sum_k s_k^3 of the whole plan."""
    import oracle
    sizes = np.array([len(ix) for ix in index])
    order = np.argsort(sizes, kind="stable")
    if whole:
        pick = [int(k) for k in order]
    else:
        pick, spent = [], 0.0
        for q in np.linspace(0.0, 1.0, 9):
            k = int(order[int(q * (len(order) - 1))])
            cost = 2.0 * float(sizes[k]) ** 3 * len(alphas)
            if k not in pick and (not pick or spent + cost <= budget_flop):
                pick.append(k)
                spent += cost
    emin, emax = oracle.gershgorin_bounds(system.H)
    X0 = [oracle.initial_guess(system.H[index[k]][:, index[k]].toarray(), emin, emax) for k in pick]
    t0 = time.perf_counter()
    oracle.sp2_blocks(X0, [int(cores[k]) for k in pick], system.n_occ, alpha_seq=list(alphas), trace_tol=1e30)
    dt = time.perf_counter() - t0
    s3_sample = float(sum(float(sizes[k]) ** 3 for k in pick))
    s3_all = float(np.sum(sizes.astype(np.float64) ** 3))
    ms = dt * 1e3 * s3_all / s3_sample
    what = ("all" if whole else f"{len(pick)}") + f" of {len(index)} parts of the benched plan"
    return {"value": round(ms, 1), "unit": "ms/P", "cores": int(host_cores()), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"FP64 numpy/OpenBLAS SP2 products of {what} (s = "
                       f"{', '.join(str(int(sizes[k])) for k in pick[:9])}{', ...' if len(pick) > 9 else ''}), "
                       f"{len(alphas)} products each, {dt:.1f} s" +
                       ("" if whole else ", scaled by sum_k s_k^3 of the whole plan"))}


def syrk_flops(sizes) -> float:
    """Flops of one symmetric product over parts of sizes s_k: s(s+1)/2 distinct
    entries, 2 s flops each."""
    s = np.asarray(sizes, dtype=np.float64)
    return float(np.sum(s * s * (s + 1.0)))


def bench_backward(args, g, torch):
    """Forward density matrix and reverse-mode pass (dL/dH for L = Tr(P W),
    W random on P's pattern) on 1,000 molecules, 32 parts, tau = 1e-3."""
    from synth.partition import uneven_spatial_partition
    from synth.water import make_water
    n_mol, n_parts, tau = 1000, 32, 1e-3
    system = make_water(n_mol, seed=0)
    n, n_occ = system.n, system.n_occ
    stream = torch.cuda.Stream()
    Hd = g.csr_to_device(system.H)
    Pprev, boot = dense_bootstrap(g, torch, Hd, n, n_occ, stream)
    part = uneven_spatial_partition(system, n_parts, seed=0)
    with torch.cuda.stream(stream):
        plan = g.gsp2_plan_create(Pprev, tau, part, n_parts, stream=stream)
    del Pprev
    info, _, sub_sizes = g.gsp2_plan_query(plan)
    P_val = torch.empty(info["nnz_P"], dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(11)
    W = torch.randn(info["nnz_P"], dtype=torch.float32, device="cuda", generator=gen)
    with torch.cuda.stream(stream):
        run = g.gsp2_density(plan, Hd, n_occ, P_val)
        alphas = run["alpha"]
        n_prod = run["n_products"]
        dH = None
        for _ in range(args.warmup):
            g.gsp2_density(plan, Hd, n_occ, P_val, max_iter=n_prod, want_info=False)
            dH, binfo = g.gsp2_backward(plan, Hd, alphas, W, dH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.gsp2_density(plan, Hd, n_occ, P_val, max_iter=n_prod, want_info=False)
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dH, binfo = g.gsp2_backward(plan, Hd, alphas, W, dH)
        torch.cuda.synchronize()
        bwd_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # matrix-core work of the pass: the forward replay to the checkpoints, the
    # recomputation inside each segment, and two products per reverse step
    m = len(alphas)
    k = binfo["checkpoint_every"]
    nseg = max(1, -(-m // k))
    replay = (nseg - 1) * k + sum(max(0, min(k, m - j * k) - 1) for j in range(nseg))
    unit = syrk_flops(sub_sizes)
    flops = (replay + 2 * m) * unit
    out = {
        "metric": "ms per reverse-mode pass dL/dH (and per forward P) at 1,000 molecules",
        "value": round(bwd_ms, 3), "unit": "ms/backward", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(bwd_ms, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n_mol} water molecules ({n} orbitals), {n_parts} uneven parts, tau={tau:g}, "
                               "L = Tr(P W) with W random on P's pattern",
                   "n_products": m, "checkpoint_every": k, "s_min": info["min_s"], "s_max": info["max_s"]},
        "forward_ms": round(fwd_ms, 3), "backward_over_forward": round(bwd_ms / fwd_ms, 3),
        "backward_tflops": round(flops / (bwd_ms * 1e-3) / 1e12, 2),
        "backward_tflops_convention": ("(forward replay + segment recomputation + 2 per reverse step) products "
                                       "x sum_k s_k^2 (s_k + 1), over the pass's wall time"),
        "backward_workspace_gib": round(binfo["workspace_bytes"] / 2**30, 3),
        "previous_P": f"regular SP2 of H on the GPU ({boot['n_products']} products)",
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


def bench_batch(args, g, torch):
    """The uneven batch: every system's density matrix from one batched plan,
    one launch per product carrying the tiles of all systems still iterating."""
    from synth.batch import make_batch
    precision, refine = args.precision, args.refine
    t = time.perf_counter()
    b = make_batch()
    log(f"batch: {len(b.steps)} systems, N={b.H.shape[0]}, {b.n_parts} parts, inputs {time.perf_counter() - t:.1f} s")
    stream = torch.cuda.Stream()
    Hd = g.csr_to_device(b.H)
    t = time.perf_counter()
    with torch.cuda.stream(stream):
        plan = g.gsp2_plan_create(g.csr_to_device(b.P_prev), b.tau, b.part, b.n_parts, stream=stream,
                                  part_system=b.part_system)
    plan_s = time.perf_counter() - t
    torch.cuda.empty_cache()
    info, _, sub_sizes = g.gsp2_plan_query(plan)
    log(f"plan: s in [{info['min_s']}, {info['max_s']}], {info['n_tiles']} tiles per product, "
        f"workspace {info['workspace_bytes'] / 2**30:.1f} GiB, {plan_s:.1f} s")
    P_val = torch.empty(info["nnz_P"], dtype=torch.float32, device="cuda")
    sys_flops = [syrk_flops(sub_sizes[b.part_offs[i]:b.part_offs[i + 1]]) for i in range(len(b.steps))]
    tuning = None
    if not args.no_tune:
        with torch.cuda.stream(stream):
            tuning = g.gsp2_plan_tune(plan, Hd, 0.0, precision, n_products=6)
        log(f"kernel autotuner: {tuning}")
    form = tuning["chosen"] if tuning else "auto"
    with torch.cuda.stream(stream):
        first = g.gsp2_density(plan, Hd, b.n_occ, P_val, max_iter=args.max_iter, precision=precision, refine=refine,
                               refine_precision=args.refine_precision)
    n_main = [r["n_products"] - r["n_refine"] for r in first]
    max_main = max(n_main)
    log(f"first run: main products per system {n_main}")
    kw = dict(max_iter=max_main, precision=precision, refine=refine, kernel=form,
              refine_precision=args.refine_precision)
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            runs = g.gsp2_density(plan, Hd, b.n_occ, P_val, timing=True, **kw)
            assert all(r["status"] == 0 for r in runs), runs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        product_ms, totals = [], []
        for i in range(args.steps):
            g.gsp2_density(plan, Hd, b.n_occ, P_val, timing=True, want_info=False, **kw)
            tm = g.gsp2_run_timing(plan)
            product_ms.append(tm["product_ms"]); totals.append(tm["total_ms"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs = g.gsp2_run_status(plan)
    assert all(r["status"] == 0 for r in runs), runs
    ms_per_batch = wall * 1e3 / args.steps
    # launch t of the main phase carries every system whose main phase formed more than t products
    per_launch = np.median(np.asarray(product_ms), axis=0)
    main_ms, main_flops = 0.0, 0.0
    for t_ in range(max_main):
        main_ms += float(per_launch[t_])
        main_flops += sum(f for f, m in zip(sys_flops, n_main) if m > t_)
    ref_ms = float(np.sum(per_launch[max_main:]))
    ref_flops = refine * sum(sys_flops)
    total_flops = main_flops + ref_flops
    per_system = []
    for i, (st, r) in enumerate(zip(b.steps, runs)):
        # device time until the system's last product: setup excluded, launches it took part in
        done = float(np.sum(per_launch[:n_main[i]])) + ref_ms
        per_system.append({"n_mol": st.system.n_mol, "n_orbitals": st.system.n, "n_parts": st.n_parts,
                           "n_products": r["n_products"], "n_refine": r["n_refine"],
                           "product_kernels_ms_until_done": round(done, 3),
                           "trace_minus_nocc": r["trace"] - st.system.n_occ,
                           "idempotency_e": r["errors"]})
    alone_ms = None
    if not args.no_alone:
        alone_ms = []
        for i, st in enumerate(b.steps):
            Hs = g.csr_to_device(st.system.H)
            with torch.cuda.stream(stream):
                with g.gsp2_plan_create(g.csr_to_device(st.P_prev), b.tau, st.part, st.n_parts,
                                        stream=stream) as p1:
                    Pv = torch.empty(p1.nnz_P, dtype=torch.float32, device="cuda")
                    k1 = dict(kw, max_iter=n_main[i])
                    g.gsp2_density(p1, Hs, st.system.n_occ, Pv, **k1)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    for _ in range(args.compare_steps):
                        g.gsp2_density(p1, Hs, st.system.n_occ, Pv, want_info=False, **k1)
                    torch.cuda.synchronize()
                    alone_ms.append((time.perf_counter() - t1) * 1e3 / args.compare_steps)
            per_system[i]["alone_ms_per_P"] = round(alone_ms[-1], 3)
            del Pv, Hs
            torch.cuda.empty_cache()
        log(f"each system in a plan of its own: {sum(alone_ms):.1f} ms in total, batch {ms_per_batch:.1f} ms")
    peak_main = PEAK_MFMA_TFLOPS[precision]
    main_tf = main_flops / (main_ms * 1e-3) / 1e12
    out = {
        "metric": "ms per batch of 16 density matrices (uneven systems, one plan) + aggregate TFLOP/s",
        "value": round(ms_per_batch, 3), "unit": "ms/batch", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_batch, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[precision], "data": "synthetic",
        "config": {
            "workload": (f"{len(b.steps)} independent water systems of {min(s_.system.n_mol for s_ in b.steps)}-"
                         f"{max(s_.system.n_mol for s_ in b.steps)} molecules ({b.H.shape[0]} orbitals, "
                         f"{b.n_parts} parts), 0.05 A displacements, repartitioned, tau={b.tau:g}, "
                         f"{precision.upper()} products + {refine} "
                         f"{'split-FP16' if args.refine_precision == 'fp16x3' else 'FP32'} refinement products"),
            "n_systems": len(b.steps), "n_orbitals": b.H.shape[0], "n_parts": b.n_parts, "tau": b.tau,
            "s_min": info["min_s"], "s_max": info["max_s"], "tiles_per_product": info["n_tiles"],
            "precision": precision, "refine": refine, "refine_precision": args.refine_precision,
        },
        "aggregate_tflops": round(total_flops / (float(np.sum(per_launch)) * 1e-3) / 1e12, 2),
        "aggregate_tflops_convention": "symmetric-product flops of every system in every launch it took part in "
                                       "/ summed product-kernel time",
        "roofline": {"bound": "mfma",
                     "kernel": f"{kernel_name(precision, form)}<{precision}>", "achieved": round(main_tf, 2),
                     "peak": peak_main, "unit": "TFLOP/s", "frac": round(main_tf / peak_main, 4), "traffic": None,
                     "refine_kernel_tflops": round(ref_flops / (ref_ms * 1e-3) / 1e12, 2) if ref_ms > 0 else None},
        "event_total_ms_median": round(statistics.median(totals), 3),
        "main_launches": max_main, "main_launch_ms": round(main_ms, 3), "refine_launch_ms": round(ref_ms, 3),
        "alone_total_ms": round(sum(alone_ms), 3) if alone_ms else None,
        "kernel_tuning": tuning,
        "per_system": per_system,
        "plan_ms": round(plan_s * 1e3, 1),
        "workspace_gib": round(info["workspace_bytes"] / 2**30, 2),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


def graph_digest(g, plan, n):
    """SHA-256 of the plan's graph (union of both orientations, canonical CSR),
    hashed as the stored oracle expectations hash the oracle's graph."""
    import hashlib

    import scipy.sparse as sp
    adj_ptr, adj_col = g.gsp2_plan_graph(plan)
    A = sp.csr_matrix((np.ones(len(adj_col), dtype=np.int8), adj_col, adj_ptr), shape=(n, n))
    A = ((A + A.T) > 0).astype(np.int8).tocsr()
    A.sort_indices()
    h = hashlib.sha256()
    h.update(np.asarray(A.indptr, dtype="<i8").tobytes())
    h.update(np.asarray(A.indices, dtype="<i4").tobytes())
    return h.hexdigest(), int(A.nnz)


GOLDEN_STEM = os.path.join(ROOT, "tests", "golden", "gsp2_water3500_densep_tau1e-5")


def stored_oracle(args, digest):
    """The FP64 oracle's stored per-part sketches of this workload (written by
    tests/golden/make_full_size_golden.py), when the benched graph is the one
    they were taken on; else None."""
    try:
        gold = json.load(open(GOLDEN_STEM + ".json"))
        arrays = dict(np.load(GOLDEN_STEM + ".npz"))
    except (OSError, ValueError):
        return None
    sp_ = gold["spec"]
    same = (sp_["n_mol"], sp_["seed"], sp_["n_parts"], sp_["core_lo"], sp_["core_hi"], sp_["tau"]) == \
        (args.n_mol, args.seed, args.n_parts, args.core_lo, args.core_hi, args.tau)
    return (gold, arrays) if same and gold["graph"]["sha256"] == digest else None


def oracle_sketch_errors(stored, vals, col_ptr, part):
    """Relative error of every part's core columns against the oracle's,
    through the stored Gaussian sketches (synth.sketch): max and median."""
    from synth import sketch
    gold, arrays = stored
    errs = []
    for k, p in enumerate(gold["parts"]):
        core = np.flatnonzero(part == k)
        B = vals[col_ptr[core][None, :] + np.arange(p["s"])[:, None]].astype(np.float64)
        S, R = sketch.probes(k, p["s"], p["c"])
        want = arrays["part_sketch"][k]
        errs.append(float(np.linalg.norm(S @ B @ R - want) / np.linalg.norm(want)))
    return {"max": float(np.max(errs)), "median": float(np.median(errs)), "parts": len(errs),
            "against": "FP64 oracle, per-part Gaussian sketches of the core columns, oracle's branch sequence"}


def timed_runs(g, torch, plan, Hd, n_occ, P, steps, warmup, stream, **kw):
    """`warmup` untimed and `steps` timed density matrices; each timed step is
    bracketed by device synchronisations.  Returns per-step wall ms, per-step
    event timings and the last run's status."""
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            g.gsp2_density(plan, Hd, n_occ, P, want_info=False, check=False, **kw)
        torch.cuda.synchronize()
        wall, timings = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            g.gsp2_density(plan, Hd, n_occ, P, want_info=False, check=False, **kw)
            if kw.get("timing"):
                timings.append(g.gsp2_run_timing(plan))
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t0) * 1e3)
        last = g.gsp2_run_status(plan)
    return wall, timings, last


def bench_water(args, g, torch):
    """The headline workload: 3,500 water molecules, 128 uneven parts, graph
    of the regular-SP2 previous P at tau, FP32 products; then the same P
    with the other operand precisions, and the shape-matched tau variant."""
    from synth.locality import surrogate_prev_density
    from synth.partition import uneven_spatial_partition
    from synth.water import make_water
    stream = torch.cuda.Stream()
    t = time.perf_counter()
    system = make_water(args.n_mol, seed=args.seed)
    n, n_occ = system.n, system.n_occ
    part = uneven_spatial_partition(system, args.n_parts, args.core_lo, args.core_hi, seed=args.seed)
    log(f"system: {args.n_mol} molecules, N={n}, nnz(H)={system.H.nnz}, {time.perf_counter() - t:.1f} s")
    Hd = g.csr_to_device(system.H)

    t = time.perf_counter()
    saved = None
    if args.load_state:
        saved = np.load(args.load_state)
        # the saved graph as a 0/1 matrix: thresholding it at 0.5 gives the same graph
        adj_ptr, adj_col = saved["adj_ptr"], saved["adj_col"]
        Pprev = g.DeviceCSR(n, torch.as_tensor(adj_ptr).cuda(), torch.as_tensor(adj_col).cuda(),
                            torch.ones(len(adj_col), dtype=torch.float32, device="cuda"))
        tau = 0.5
        boot_desc = str(saved["previous_P"])
    elif args.graph == "dense-sp2":
        Pprev, boot = dense_bootstrap(g, torch, Hd, n, n_occ, stream)
        boot_desc = f"regular SP2 of H on the GPU, FP64 products ({boot['n_products']} products)"
        tau = args.tau
    else:
        Pprev = g.csr_to_device(surrogate_prev_density(system))
        boot_desc = "distance-based stand-in for the previous P"
        tau = args.tau
    boot_s = time.perf_counter() - t
    log(f"previous P: {boot_desc}, {boot_s:.1f} s")

    t = time.perf_counter()
    with torch.cuda.stream(stream):
        plan = g.gsp2_plan_create(Pprev, tau, part, args.n_parts, stream=stream)
    plan_s = time.perf_counter() - t
    digest, nnz_sym = graph_digest(g, plan, n)
    if args.save_state:
        adj_ptr, adj_col = g.gsp2_plan_graph(plan)
        np.savez(args.save_state, adj_ptr=adj_ptr, adj_col=adj_col, previous_P=boot_desc)
    info, core_sizes, sub_sizes = g.gsp2_plan_query(plan)
    log(f"plan: s in [{info['min_s']}, {info['max_s']}], sum s^3 = {info['sum_s3']:.3e}, "
        f"tiles/product = {info['n_tiles']}, workspace = {info['workspace_bytes'] / 2**30:.2f} GiB, {plan_s:.1f} s, "
        f"graph {nnz_sym} entries sha256 {digest[:16]}")
    stored = stored_oracle(args, digest) if saved is None else None
    log("stored oracle sketches: " + ("used (the benched graph is the oracle's)" if stored else "not applicable"))
    P_val = torch.empty(info["nnz_P"], dtype=torch.float64 if args.precision == "fp64" else torch.float32,
                        device="cuda")
    col_ptr, _ = g.gsp2_plan_pattern(plan)

    # the kernel autotuner's form for the headline precision, timed on this plan
    head_tune = None
    if not args.no_tune and args.precision != "fp64":
        with torch.cuda.stream(stream):
            head_tune = g.gsp2_plan_tune(plan, Hd, n_occ, args.precision, n_products=6)
        log(f"kernel autotuner: {head_tune}")
    head_form = head_tune["chosen"] if head_tune else args.kernel
    # the first run, in the form the timed runs take, finds where the stop
    # rule fires; later runs form exactly that many products (the same stop
    # fires at the same product), so no empty launches follow the stop
    if saved is not None:
        n_prod = int(saved["n_products"])
        alphas = None
    else:
        with torch.cuda.stream(stream):
            first = g.gsp2_density(plan, Hd, n_occ, P_val, max_iter=args.max_iter, precision=args.precision,
                                   kernel=head_form)
        n_prod = first["n_products"]
        alphas = first["alpha"]
        log(f"first run: status {first['status_name']}, {n_prod} products, Tr P = {first['trace']:.6f}")
    if args.save_state:
        with np.load(args.save_state) as z:
            d = dict(z)
        np.savez(args.save_state, n_products=n_prod, **d)
        log(f"state saved to {args.save_state}")
    timed = not args.no_kernel_timing
    kw = dict(max_iter=n_prod, precision=args.precision, timing=timed, kernel=head_form)
    wall, timings, last = timed_runs(g, torch, plan, Hd, n_occ, P_val, args.steps, args.warmup, stream, **kw)
    assert last["status"] == 0 and last["n_products"] == n_prod, last
    ms_median = statistics.median(wall)
    log(f"timed {args.steps} steps: median {ms_median:.1f} ms per P (mean {statistics.fmean(wall):.1f})")
    if timed:
        product_ms = [x for tm in timings for x in tm["product_ms"]]
        setup = [tm["setup_ms"] for tm in timings]
        sp2 = [tm["sp2_ms"] for tm in timings]
        scatter = [tm["scatter_ms"] for tm in timings]
        totals = [tm["total_ms"] for tm in timings]
    else:
        product_ms, setup, scatter, totals = [float("nan")], [float("nan")], [float("nan")], [float("nan")]
        sp2 = wall
    head_err = None
    if stored is not None and args.precision != "fp64":
        with torch.cuda.stream(stream):
            g.gsp2_density(plan, Hd, n_occ, P_val, alpha_seq=stored[0]["alphas"], trace_tol=1e9, kernel=head_form,
                           precision=args.precision)
        head_err = oracle_sketch_errors(stored, P_val.cpu().numpy(), col_ptr, part)
        log(f"{args.precision} vs oracle: max {head_err['max']:.2e}")

    s = np.asarray(sub_sizes, dtype=np.float64)
    sym_flops = float(np.sum(s * s * (s + 1.0)))          # distinct entries s(s+1)/2, 2s flops each
    product_kernel = kernel_name(args.precision, head_form)
    with torch.cuda.stream(stream):
        probe = {p: g.gsp2_probe_mfma(p, stream=stream)
                 for p in {"fp32", args.precision, *[q for q in args.compare_precisions.split(",") if q]}
                 if p != "fp64"}
    log("measured MFMA rate: " + ", ".join(f"{p} {v:.1f} TFLOP/s" for p, v in sorted(probe.items())))
    avg_prod_ms = statistics.fmean(product_ms)
    achieved = MFMA_PRODUCTS[args.precision] * sym_flops / (avg_prod_ms * 1e-3) / 1e12
    peak = PEAK_MFMA_TFLOPS[args.precision]
    sp2_med = statistics.median(sp2)

    # the same density matrix with other product precisions, on the same GPU
    compare = {}
    for prec in [p for p in args.compare_precisions.split(",") if p]:
        dt = torch.float64 if prec == "fp64" else torch.float32
        P_mp = torch.empty(info["nnz_P"], dtype=dt, device="cuda")
        tune_rec = None
        with torch.cuda.stream(stream):
            if not args.no_tune and prec in ("fp32", "fp16", "bf16", "fp16x3", "fp64"):
                tune_rec = g.gsp2_plan_tune(plan, Hd, n_occ, prec, n_products=6)
            r0 = g.gsp2_density(plan, Hd, n_occ, P_mp, max_iter=args.max_iter, precision=prec, check=False)
        n_mp = r0["n_products"]
        w, tms, last_mp = timed_runs(g, torch, plan, Hd, n_occ, P_mp, args.compare_steps, 1, stream,
                                     max_iter=n_mp, precision=prec, timing=True)
        avg = statistics.fmean([x for tm in tms for x in tm["product_ms"]])
        hw = MFMA_PRODUCTS[prec] * sym_flops
        rec = {"ms_per_P": round(statistics.median(w), 3), "n_products": n_mp, "status": r0["status_name"],
               "trace_minus_nocc": r0["trace"] - n_occ, "product_kernel_ms": round(avg, 4),
               "tflops": round(sym_flops / (avg * 1e-3) / 1e12, 2), "mfma_products_per_product": MFMA_PRODUCTS[prec],
               "frac_of_peak": round(hw / (avg * 1e-3) / 1e12 / PEAK_MFMA_TFLOPS[prec], 4),
               "kernel": kernel_name(prec, tune_rec["chosen"] if tune_rec else "auto"), "kernel_tuning": tune_rec}
        if prec in probe:
            rec["frac_of_measured_peak"] = round(hw / (avg * 1e-3) / 1e12 / probe[prec], 4)
        if stored is not None:
            with torch.cuda.stream(stream):
                for refine in ((0, 2) if prec in ("fp16", "bf16") else (0,)):
                    # the oracle's branch sequence replayed (every product of the oracle's run formed
                    # with this precision's operands) ...
                    g.gsp2_density(plan, Hd, n_occ, P_mp, alpha_seq=stored[0]["alphas"], trace_tol=1e9,
                                   precision=prec, refine=refine)
                    rec[f"error_vs_oracle_refine{refine}"] = oracle_sketch_errors(
                        stored, P_mp.cpu().numpy(), col_ptr, part)["max"]
                    # ... and the run's own branches and stop (at this precision's floor), against the
                    # oracle's P
                    r_t = g.gsp2_density(plan, Hd, n_occ, P_mp, precision=prec, refine=refine, check=False)
                    rec[f"trace_mode_refine{refine}"] = {
                        "error_vs_oracle": oracle_sketch_errors(stored, P_mp.cpu().numpy(), col_ptr, part)["max"],
                        "n_products": r_t["n_products"], "status": r_t["status_name"],
                        "trace_minus_nocc": r_t["trace"] - n_occ}
        if prec in ("fp16", "bf16"):
            # the whole P with two refinement products, FP32 or split FP16, timed like the main line
            rec["with_refinement"] = {}
            for rp in ("fp32", "fp16x3"):
                kw_r = dict(max_iter=n_mp, precision=prec, refine=2, refine_precision=rp)
                w_r, _, last_r = timed_runs(g, torch, plan, Hd, n_occ, P_mp, args.compare_steps, 1, stream, **kw_r)
                e_r = (oracle_sketch_errors(stored, P_mp.cpu().numpy(), col_ptr, part)["max"]
                       if stored is not None else None)
                rec["with_refinement"][rp] = {"ms_per_P": round(statistics.median(w_r), 3),
                                              "n_products": last_r["n_products"], "status": last_r["status_name"],
                                              "error_vs_oracle": e_r, "trace_minus_nocc": last_r["trace"] - n_occ}
                log(f"{prec} + 2 {rp} refinement products: {statistics.median(w_r):.1f} ms/P" +
                    (f", error vs oracle {e_r:.2e}" if e_r is not None else ""))
        compare[prec] = rec
        log(f"{prec}: {rec['ms_per_P']:.1f} ms/P, {n_mp} products, status {r0['status_name']}, "
            f"Tr P - N_occ = {rec['trace_minus_nocc']:.3e}" +
            (f", error vs oracle {rec['error_vs_oracle_refine0']:.2e}" if stored is not None else ""))
        del P_mp
        torch.cuda.empty_cache()

    library = None
    if not args.no_library_compare:
        ours = {args.precision: avg_prod_ms, **{p: c["product_kernel_ms"] for p, c in compare.items()}}
        library = library_products(torch, stream, [int(v) for v in sub_sizes], float(np.sum(2.0 * s ** 3)), ours)
        log("library products: " + ", ".join(f"{p} {v['ms_per_product']:.2f} ms" for p, v in library.items()
                                             if isinstance(v, dict)))

    cpu = None
    if not args.no_cpu_baseline and alphas is not None:
        log("cpu baseline: timing the FP64 oracle on parts of the benched plan")
        index = [g.gsp2_plan_part_index(plan, k) for k in range(args.n_parts)]
        cpu = cpu_baseline(system, index, core_sizes, alphas)
        log(f"cpu baseline: {cpu['value']:.0f} ms/P on {cpu['cores']} threads ({cpu['sample']})")
    plan.close()
    del P_val
    torch.cuda.empty_cache()

    variant = None
    if args.variant_tau > 0 and saved is None:
        variant = shape_matched(args, g, torch, system, part, Hd, Pprev, stream, probe)
    del Pprev
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": round(ms_median, 3),
        "unit": "ms/P",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_median, 3),
        "ms_per_step_mean": round(statistics.fmean(wall), 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"G-SP2 density matrix of {args.n_mol} synthetic water molecules ({n} orbitals), "
                         f"{args.n_parts} uneven spatial parts, graph of the previous P at tau={args.tau:g}"),
            "n_mol": args.n_mol, "n_orbitals": n, "n_occ": n_occ, "n_parts": args.n_parts,
            "tau": args.tau, "previous_P": boot_desc, "graph_entries": nnz_sym, "graph_sha256": digest,
            "s_min": info["min_s"], "s_max": info["max_s"], "s_mean": round(float(s.mean()), 1),
            "sum_s3": info["sum_s3"], "n_products": n_prod, "tiles_per_product": info["n_tiles"],
            "precision": f"{args.precision.upper()} MFMA operands, FP32 accumulation and iterate, FP64 traces",
        },
        "error_vs_oracle": head_err,
        "gemm_convention_rate": {
            "value": round(n_prod * float(np.sum(2.0 * s ** 3)) / (sp2_med * 1e-3) / 1e12, 2),
            "convention": ("n_products * sum_k 2 s_k^3 / SP2-phase time, in 1e12 per second: the flop count of "
                           "full dense GEMMs, twice what the symmetric product performs; not a rate of executed "
                           "flops (roofline.achieved is)")},
        "roofline": {
            "bound": "mfma", "kernel": product_kernel,
            "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "measured_peak": round(probe[args.precision], 1) if args.precision in probe else None,
            "frac_of_measured_peak": round(achieved / probe[args.precision], 4) if args.precision in probe else None,
            "traffic": counter_traffic(
                args.precision, {"n_mol": args.n_mol, "n_parts": args.n_parts, "tau": args.tau,
                                 "sum_s3": info["sum_s3"]}, product_kernel),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "flops_per_launch": MFMA_PRODUCTS[args.precision] * sym_flops, "avg_launch_ms": round(avg_prod_ms, 4),
            "flops_convention": "symmetric product: sum_k s_k^2 (s_k + 1) per launch (one launch = one product)",
        },
        "phase_ms": {"setup": round(statistics.median(setup), 3), "sp2": round(sp2_med, 3),
                     "scatter": round(statistics.median(scatter), 3),
                     "event_total_median": round(statistics.median(totals), 3)},
        # the analogue of the paper's linear-algebra-only time against the whole step
        "time_split": {"products_ms": round(sum(product_ms) / args.steps, 3),
                       "other_ms": round(statistics.median(totals) - sum(product_ms) / args.steps, 3),
                       "products_share": round(sum(product_ms) / args.steps / statistics.median(totals), 4),
                       "convention": "event time of the product launches (matrix products with their fused "
                                     "update and trace partials) against the rest of one P: Gershgorin, gather, "
                                     "branch decisions, scatter and launch gaps"},
        "kernel_tuning": head_tune,
        "precision_compare": compare,
        "shape_matched": variant,
        "plan_ms": round(plan_s * 1e3, 1),
        "plan_info": {k: info[k] for k in ("nnz_graph", "nnz_P", "sum_s", "workspace_bytes")},
        "previous_P_s": round(boot_s, 2),
        "library_products": library,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def shape_matched(args, g, torch, system, part, Hd, Pprev, stream, probe):
    """The same system and previous P thresholded at the variant tau, whose
    sub-problems fall in the 400-1,600 range the workload names: FP32 and
    FP16 timings, and the whole FP64 oracle on the host as its CPU baseline."""
    n_occ = system.n_occ
    tau = args.variant_tau
    with torch.cuda.stream(stream):
        plan = g.gsp2_plan_create(Pprev, tau, part, args.n_parts, stream=stream)
    info, core_sizes, sub_sizes = g.gsp2_plan_query(plan)
    s = np.asarray(sub_sizes, dtype=np.float64)
    sym_flops = float(np.sum(s * s * (s + 1.0)))
    P = torch.empty(info["nnz_P"], dtype=torch.float32, device="cuda")
    out = {"tau": tau, "s_min": info["min_s"], "s_max": info["max_s"], "s_mean": round(float(s.mean()), 1),
           "sum_s3": info["sum_s3"], "tiles_per_product": info["n_tiles"]}
    alphas = None
    for prec in ("fp32", "fp16"):
        tune = None
        with torch.cuda.stream(stream):
            if not args.no_tune:
                tune = g.gsp2_plan_tune(plan, Hd, n_occ, prec, n_products=6)
            first = g.gsp2_density(plan, Hd, n_occ, P, max_iter=args.max_iter, precision=prec, check=False)
        if prec == "fp32":
            alphas = first["alpha"]
        n_prod = first["n_products"]
        w, tms, _ = timed_runs(g, torch, plan, Hd, n_occ, P, args.variant_steps, 2, stream,
                               max_iter=n_prod, precision=prec, timing=True)
        avg = statistics.fmean([x for tm in tms for x in tm["product_ms"]])
        ach = MFMA_PRODUCTS[prec] * sym_flops / (avg * 1e-3) / 1e12
        out[prec] = {"ms_per_P": round(statistics.median(w), 3), "n_products": n_prod, "status": first["status_name"],
                     "trace_minus_nocc": first["trace"] - n_occ, "product_kernel_ms": round(avg, 4),
                     "achieved_tflops": round(ach, 2), "frac": round(ach / PEAK_MFMA_TFLOPS[prec], 4),
                     "frac_of_measured_peak": round(ach / probe[prec], 4) if prec in probe else None,
                     "kernel": kernel_name(prec, tune["chosen"] if tune else "auto"), "kernel_tuning": tune}
        log(f"tau={tau:g}: {prec} {out[prec]['ms_per_P']:.2f} ms/P, kernel {avg:.3f} ms, {ach:.1f} TFLOP/s")
    if not args.no_cpu_baseline:
        index = [g.gsp2_plan_part_index(plan, k) for k in range(args.n_parts)]
        out["cpu_baseline"] = cpu_baseline(system, index, core_sizes, alphas, whole=True)
        log(f"tau={tau:g}: cpu baseline {out['cpu_baseline']['value']:.0f} ms/P")
    plan.close()
    return out


def main():
    args = parse()
    batch = args.workload == "batch16"
    args.precision = args.precision or ("fp16" if batch else "fp32")
    args.refine = (2 if batch else 0) if args.refine is None else args.refine
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        return 2
    import torch

    import paper_1801_10016_amd as g

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    g.load()
    torch.cuda.set_device(0)
    if args.copy_probe_gib > 0:
        return copy_probe(torch, args.copy_probe_gib)
    if args.workload == "batch16":
        return bench_batch(args, g, torch)
    if args.workload == "backward1000":
        return bench_backward(args, g, torch)
    return bench_water(args, g, torch)


if __name__ == "__main__":
    sys.exit(main())

"""ctypes binding of libgsp2.so (the C ABI declared in include/gsp2.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and the HIP stream.  Importing
this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsp2.so")

GSP2_OK, GSP2_E_INVALID, GSP2_E_HIP, GSP2_E_OOM, GSP2_E_NOT_CONVERGED, GSP2_E_WRONG_TRACE, GSP2_E_UNSUPPORTED = range(7)
GSP2_F32, GSP2_F64 = 0, 1
GSP2_ALPHA_TRACE, GSP2_ALPHA_REPLAY = 0, 1
GSP2_PREC_FP32, GSP2_PREC_FP16, GSP2_PREC_BF16, GSP2_PREC_FP16X3, GSP2_PREC_FP64 = 0, 1, 2, 3, 4
PRECISIONS = {"fp32": GSP2_PREC_FP32, "fp16": GSP2_PREC_FP16, "bf16": GSP2_PREC_BF16,
              "fp16x3": GSP2_PREC_FP16X3, "fp64": GSP2_PREC_FP64}
GSP2_MAX_ITER = 100
GSP2_KERNEL_AUTO, GSP2_KERNEL_T128, GSP2_KERNEL_T128_SKIP, GSP2_KERNEL_T256 = 0, 1, 2, 3
KERNELS = {"auto": GSP2_KERNEL_AUTO, "t128": GSP2_KERNEL_T128, "t128_skip": GSP2_KERNEL_T128_SKIP,
           "t256": GSP2_KERNEL_T256}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}
GSP2_TUNE_MAX = 4

STATUS_NAMES = {0: "GSP2_OK", 1: "GSP2_E_INVALID", 2: "GSP2_E_HIP", 3: "GSP2_E_OOM",
                4: "GSP2_E_NOT_CONVERGED", 5: "GSP2_E_WRONG_TRACE", 6: "GSP2_E_UNSUPPORTED"}


class gsp2_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("dtype", C.c_int32)]


class gsp2_plan_options(C.Structure):
    _fields_ = [("tile", C.c_int32), ("n_systems", C.c_int32), ("part_system", C.POINTER(C.c_int32)),
                ("tile16", C.c_int32), ("reserved", C.c_int32 * 3)]


class gsp2_tune_info(C.Structure):
    _fields_ = [("precision", C.c_int32), ("chosen", C.c_int32), ("n_candidates", C.c_int32),
                ("n_products", C.c_int32), ("candidate", C.c_int32 * GSP2_TUNE_MAX),
                ("ms", C.c_double * GSP2_TUNE_MAX)]


class gsp2_plan_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_parts", C.c_int32), ("max_s", C.c_int32), ("min_s", C.c_int32),
                ("nnz_graph", C.c_int64), ("nnz_P", C.c_int64), ("sum_s", C.c_int64), ("sum_s3", C.c_double),
                ("tile", C.c_int32), ("n_tiles", C.c_int32), ("workspace_bytes", C.c_int64),
                ("plan_ms", C.c_double), ("n_systems", C.c_int32), ("pad_", C.c_int32)]


class gsp2_run_options(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("alpha_mode", C.c_int32), ("alpha_seq", C.POINTER(C.c_int8)),
                ("n_alpha", C.c_int32), ("stop_rule", C.c_int32), ("trace_tol", C.c_double),
                ("timing", C.c_int32), ("precision", C.c_int32), ("refine", C.c_int32),
                ("persistent", C.c_int32), ("n_occ_system", C.POINTER(C.c_double)),
                ("alpha_seq_system", C.POINTER(C.c_int8)), ("n_alpha_system", C.POINTER(C.c_int32)),
                ("symmetrize", C.c_int32), ("kernel", C.c_int32), ("refine_precision", C.c_int32),
                ("pad2_", C.c_int32)]


class gsp2_run_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_products", C.c_int32), ("n_alpha", C.c_int32),
                ("result_iterate", C.c_int32), ("n_refine", C.c_int32), ("precision", C.c_int32),
                ("eps_min", C.c_double), ("eps_max", C.c_double),
                ("trace", C.c_double), ("idempotency", C.c_double),
                ("alpha", C.c_int8 * GSP2_MAX_ITER), ("traces", C.c_double * (GSP2_MAX_ITER + 1)),
                ("errors", C.c_double * GSP2_MAX_ITER)]


class gsp2_timing(C.Structure):
    _fields_ = [("n_products", C.c_int32), ("setup_ms", C.c_float), ("sp2_ms", C.c_float),
                ("scatter_ms", C.c_float), ("total_ms", C.c_float), ("persistent_ms", C.c_float),
                ("product_ms", C.c_float * GSP2_MAX_ITER)]


class gsp2_anneal_options(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("pad_", C.c_int32), ("t0", C.c_double), ("cooling", C.c_double),
                ("seed", C.c_uint64), ("reserved", C.c_int32 * 4)]


class gsp2_backward_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_alpha", C.c_int32), ("checkpoint_every", C.c_int32),
                ("row_min", C.c_int32), ("row_max", C.c_int32), ("eps_min", C.c_double),
                ("eps_max", C.c_double), ("d_eps_min", C.c_double), ("d_eps_max", C.c_double),
                ("workspace_bytes", C.c_int64)]


class gsp2_sparse_sp2_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_products", C.c_int32), ("n_alpha", C.c_int32), ("pad_", C.c_int32),
                ("eps_min", C.c_double), ("eps_max", C.c_double), ("trace", C.c_double),
                ("idempotency", C.c_double), ("nnz", C.c_int64), ("alpha", C.c_int8 * GSP2_MAX_ITER)]


_PLAN = C.c_void_p

# name -> (restype, argtypes), exactly the functions declared in gsp2.h
SIGNATURES = {
    "gsp2_status_string": (C.c_char_p, [C.c_int]),
    "gsp2_last_error": (C.c_char_p, []),
    "gsp2_run_options_default": (C.c_int, [C.POINTER(gsp2_run_options)]),
    "gsp2_plan_create": (C.c_int, [C.POINTER(gsp2_csr), C.c_double, C.POINTER(C.c_int32), C.c_int32,
                                   C.POINTER(gsp2_plan_options), C.c_void_p, C.POINTER(_PLAN)]),
    "gsp2_plan_query": (C.c_int, [_PLAN, C.POINTER(gsp2_plan_info), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gsp2_plan_pattern": (C.c_int, [_PLAN, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "gsp2_plan_part_index": (C.c_int, [_PLAN, C.c_int32, C.POINTER(C.c_int32)]),
    "gsp2_plan_set_stream": (C.c_int, [_PLAN, C.c_void_p]),
    "gsp2_density": (C.c_int, [_PLAN, C.POINTER(gsp2_csr), C.c_double, C.POINTER(gsp2_run_options),
                               C.c_void_p, C.POINTER(gsp2_run_info)]),
    "gsp2_density_noalloc": (C.c_int, [_PLAN, C.POINTER(gsp2_csr), C.c_double, C.POINTER(gsp2_run_options),
                                       C.c_void_p, C.POINTER(gsp2_run_info)]),
    "gsp2_run_status": (C.c_int, [_PLAN, C.POINTER(gsp2_run_info)]),
    "gsp2_run_timing": (C.c_int, [_PLAN, C.POINTER(gsp2_timing)]),
    "gsp2_plan_destroy": (None, [_PLAN]),
    "gsp2_backward": (C.c_int, [_PLAN, C.POINTER(gsp2_csr), C.POINTER(C.c_int8), C.c_int32, C.c_void_p,
                                C.c_void_p, C.POINTER(gsp2_backward_info)]),
    "gsp2_plan_graph": (C.c_int, [_PLAN, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "gsp2_plan_tune": (C.c_int, [_PLAN, C.POINTER(gsp2_csr), C.c_double, C.c_int32, C.c_int32,
                                 C.POINTER(gsp2_tune_info)]),
    "gsp2_probe_mfma": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
    "gsp2_locality_graph": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_double),
                                      C.c_double, C.c_double, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "gsp2_partition_anneal": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(gsp2_anneal_options),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gsp2_sparse_sp2_host": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int32,
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                       C.POINTER(gsp2_sparse_sp2_info)]),
    "gsp2_core_halo_host": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
}

_lib = None


def load() -> C.CDLL:
    """Load libgsp2.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -m paper_1801_10016_amd.build)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class Gsp2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int):
    if status != GSP2_OK:
        raise Gsp2Error(status, load().gsp2_last_error().decode())


def _i32(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _i64(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


@dataclass
class DeviceCSR:
    """A CSR matrix whose arrays are torch tensors on the GPU."""
    n: int
    row_ptr: "object"     # torch.int64, n+1
    col: "object"         # torch.int32, nnz
    val: "object"         # torch.float32 or torch.float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def as_c(self) -> gsp2_csr:
        import torch
        dt = GSP2_F64 if self.val.dtype == torch.float64 else GSP2_F32
        return gsp2_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                        self.val.data_ptr(), dt)


def csr_to_device(M, dtype=None, device="cuda") -> DeviceCSR:
    """scipy.sparse matrix -> DeviceCSR (values float64 unless dtype given)."""
    import scipy.sparse as sp
    import torch
    M = sp.csr_matrix(M)
    dtype = dtype or torch.float64
    return DeviceCSR(M.shape[0],
                     torch.as_tensor(M.indptr.astype(np.int64)).to(device),
                     torch.as_tensor(M.indices.astype(np.int32)).to(device),
                     torch.as_tensor(M.data).to(device=device, dtype=dtype))


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def gsp2_run_options_default() -> gsp2_run_options:
    o = gsp2_run_options()
    _check(load().gsp2_run_options_default(C.byref(o)))
    return o


class Plan:
    """Owns a gsp2_plan handle."""

    def __init__(self, handle: int):
        self.handle = C.c_void_p(handle)
        self.nnz_P = None
        self.n_systems = 1

    def close(self):
        if self.handle and self.handle.value:
            load().gsp2_plan_destroy(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def gsp2_plan_create(P_prev: DeviceCSR, tau: float, part, n_parts: int, tile: int = 0, stream=None,
                     part_system=None, tile16: int = 0) -> Plan:
    """part_system (n_parts ids) batches independent systems in one plan;
    tile16 fixes the 16-bit product tile edge (0: the tuned form, else 256
    x 256 tiles)."""
    part = np.ascontiguousarray(part, dtype=np.int32)
    if part.shape != (P_prev.n,):
        raise ValueError("part must have one entry per vertex")
    c = P_prev.as_c()
    opt = gsp2_plan_options(tile)
    opt.tile16 = int(tile16)
    keep = None
    if part_system is not None:
        keep = np.ascontiguousarray(part_system, dtype=np.int32)
        if keep.shape != (n_parts,):
            raise ValueError("part_system must have one entry per part")
        opt.n_systems = int(keep.max()) + 1 if keep.size else 0
        opt.part_system = _i32(keep)
    out = _PLAN()
    _check(load().gsp2_plan_create(C.byref(c), float(tau), _i32(part), int(n_parts), C.byref(opt),
                                   C.c_void_p(_stream_handle(stream)), C.byref(out)))
    del keep
    plan = Plan(out.value)
    info = gsp2_plan_query(plan)[0]
    plan.nnz_P = info["nnz_P"]
    plan.n_systems = info["n_systems"]
    return plan


def gsp2_plan_query(plan: Plan):
    lib = load()
    info = gsp2_plan_info()
    _check(lib.gsp2_plan_query(plan.handle, C.byref(info), None, None))
    cs = np.empty(info.n_parts, dtype=np.int32)
    ss = np.empty(info.n_parts, dtype=np.int32)
    _check(lib.gsp2_plan_query(plan.handle, None, _i32(cs), _i32(ss)))
    d = {f: getattr(info, f) for f, _ in gsp2_plan_info._fields_}
    return d, cs, ss


def gsp2_plan_pattern(plan: Plan):
    info, _, _ = gsp2_plan_query(plan)
    col_ptr = np.empty(info["n"] + 1, dtype=np.int64)
    row_idx = np.empty(info["nnz_P"], dtype=np.int32)
    _check(load().gsp2_plan_pattern(plan.handle, _i64(col_ptr), _i32(row_idx)))
    return col_ptr, row_idx


def gsp2_plan_part_index(plan: Plan, k: int) -> np.ndarray:
    _, _, ss = gsp2_plan_query(plan)
    idx = np.empty(int(ss[k]), dtype=np.int32)
    _check(load().gsp2_plan_part_index(plan.handle, int(k), _i32(idx)))
    return idx


def gsp2_probe_mfma(precision: str, stream=None) -> float:
    """Matrix-core rate (TFLOP/s) of back-to-back MFMAs of the product
    kernels' shape for `precision`, measured on this GPU (gsp2_probe_mfma)."""
    out = C.c_double()
    _check(load().gsp2_probe_mfma(PRECISIONS[precision], C.c_void_p(_stream_handle(stream)), C.byref(out)))
    return out.value


def gsp2_plan_tune(plan: Plan, H: DeviceCSR, n_occ, precision: str, n_products: int = 8) -> dict:
    """Time every product-kernel form of `precision` on the plan's
    sub-problems and keep the fastest (gsp2_plan_tune in gsp2.h).  Returns
    the timings and the choice; json.dump of it is the tuning record."""
    info = gsp2_tune_info()
    c = H.as_c()
    _check(load().gsp2_plan_tune(plan.handle, C.byref(c), float(n_occ), PRECISIONS[precision], int(n_products),
                                 C.byref(info)))
    return {"precision": precision, "chosen": KERNEL_NAMES[info.chosen], "n_products": info.n_products,
            "ms_per_product": {KERNEL_NAMES[info.candidate[i]]: info.ms[i] for i in range(info.n_candidates)}}


def gsp2_plan_graph(plan: Plan):
    """The plan's thresholded graph as host CSR arrays (adj_ptr int64, adj_col int32)."""
    info, _, _ = gsp2_plan_query(plan)
    adj_ptr = np.empty(info["n"] + 1, dtype=np.int64)
    _check(load().gsp2_plan_graph(plan.handle, _i64(adj_ptr), None))
    adj_col = np.empty(int(adj_ptr[-1]), dtype=np.int32)
    _check(load().gsp2_plan_graph(plan.handle, _i64(adj_ptr), _i32(adj_col)))
    return adj_ptr, adj_col


def gsp2_locality_graph(orbital_atom, xyz, radius: float, box: float = 0.0):
    """Host CSR arrays (adj_ptr int64, adj_col int32) of the locality graph:
    orbitals adjacent when their atoms are closer than radius."""
    oa = np.ascontiguousarray(orbital_atom, dtype=np.int32)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    lib = load()
    adj_ptr = np.empty(oa.size + 1, dtype=np.int64)
    args = (oa.size, _i32(oa), xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)), float(radius), float(box))
    _check(lib.gsp2_locality_graph(*args, _i64(adj_ptr), None))
    adj_col = np.empty(int(adj_ptr[-1]), dtype=np.int32)
    _check(lib.gsp2_locality_graph(*args, _i64(adj_ptr), _i32(adj_col)))
    return adj_ptr, adj_col


def gsp2_partition_anneal(adj_ptr, adj_col, part, n_parts: int, sweeps: int = 0, t0: float = 0.0,
                          cooling: float = 0.0, seed: int = 0):
    """Simulated-annealing refinement of a partition for eq. (4) (host only).
    Returns (refined part, cost before, cost after); zero options mean defaults."""
    adj_ptr = np.ascontiguousarray(adj_ptr, dtype=np.int64)
    adj_col = np.ascontiguousarray(adj_col, dtype=np.int32)
    out = np.array(part, dtype=np.int32, copy=True)
    if adj_ptr.size != out.size + 1:
        raise ValueError("adj_ptr must have n+1 entries")
    opt = gsp2_anneal_options(int(sweeps), 0, float(t0), float(cooling), int(seed))
    before, after = C.c_int64(), C.c_int64()
    _check(load().gsp2_partition_anneal(out.size, _i64(adj_ptr), _i32(adj_col), int(n_parts), _i32(out),
                                        C.byref(opt), C.byref(before), C.byref(after)))
    return out, before.value, after.value


def gsp2_plan_set_stream(plan: Plan, stream=None):
    _check(load().gsp2_plan_set_stream(plan.handle, C.c_void_p(_stream_handle(stream))))


def make_run_options(max_iter=60, alpha_seq=None, stop_rule=True, trace_tol=0.5, timing=False,
                     precision="fp32", refine=0, persistent=False, n_occ_system=None, symmetrize=False,
                     kernel="auto", refine_precision="fp32"):
    """Options struct and the arrays it points to (keep them alive for the
    call).  alpha_seq: one sequence, or (batched plans) a list of sequences,
    one per system; n_occ_system: occupations of a batched plan's systems;
    kernel: the product kernel's form ("auto", "t128", "t128_skip", "t256");
    refine_precision: operands of the refinement products ("fp32" or "fp16x3")."""
    o = gsp2_run_options_default()
    o.refine_precision = (PRECISIONS[refine_precision] if isinstance(refine_precision, str)
                          else int(refine_precision))
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.persistent = 1 if persistent else 0
    o.max_iter = int(max_iter)
    o.timing = 1 if timing else 0
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.refine = int(refine)
    o.stop_rule = 1 if stop_rule else 0
    o.trace_tol = float(trace_tol)
    o.symmetrize = 1 if symmetrize else 0
    keep = []
    if alpha_seq is not None:
        o.alpha_mode = GSP2_ALPHA_REPLAY
        if len(alpha_seq) and np.ndim(alpha_seq[0]) == 1:       # one sequence per system
            rows = np.zeros((len(alpha_seq), GSP2_MAX_ITER), dtype=np.int8)
            lens = np.zeros(len(alpha_seq), dtype=np.int32)
            for y, a in enumerate(alpha_seq):
                a = np.asarray(a, dtype=np.int8)
                if a.size > GSP2_MAX_ITER:
                    raise ValueError("alpha sequence longer than GSP2_MAX_ITER")
                rows[y, :a.size] = a
                lens[y] = a.size
            keep += [rows, lens]
            o.alpha_seq_system = rows.ctypes.data_as(C.POINTER(C.c_int8))
            o.n_alpha_system = _i32(lens)
        else:
            seq = np.ascontiguousarray(alpha_seq, dtype=np.int8)
            keep.append(seq)
            o.n_alpha = int(seq.size)
            o.alpha_seq = seq.ctypes.data_as(C.POINTER(C.c_int8))
    if n_occ_system is not None:
        occ = np.ascontiguousarray(n_occ_system, dtype=np.float64)
        keep.append(occ)
        o.n_occ_system = occ.ctypes.data_as(C.POINTER(C.c_double))
    return o, keep


def run_info_dict(info: gsp2_run_info) -> dict:
    n = info.n_alpha
    return {
        "status": info.status, "status_name": STATUS_NAMES.get(info.status, str(info.status)),
        "n_products": info.n_products, "n_alpha": n, "result_iterate": info.result_iterate,
        "n_refine": info.n_refine, "precision": info.precision,
        "eps_min": info.eps_min, "eps_max": info.eps_max, "trace": info.trace,
        "idempotency": info.idempotency, "alpha": [int(a) for a in info.alpha[:n]],
        "traces": [float(t) for t in info.traces[:n + 1]],
        "errors": [float(e) for e in info.errors[:info.n_products]],
    }


def _density(entry: str, plan: Plan, H: DeviceCSR, n_occ, P_val, max_iter=60, alpha_seq=None,
             stop_rule=True, trace_tol=0.5, want_info=True, check=True, timing=False,
             precision="fp32", refine=0, persistent=False, symmetrize=False, kernel="auto",
             refine_precision="fp32"):
    """Enqueue one density matrix into P_val (torch on the GPU, nnz_P entries:
    float64 for precision "fp64", float32 otherwise).  With want_info the
    call waits and returns the run's info dict (a list of them, one per
    system, for a batched plan); with check a failing status raises
    Gsp2Error.  For a batched plan n_occ lists every system's occupation,
    and alpha_seq, if given, one sequence per system."""
    import torch
    want = torch.float64 if precision in ("fp64", GSP2_PREC_FP64) else torch.float32
    if P_val.dtype != want or not P_val.is_cuda or not P_val.is_contiguous():
        raise ValueError(f"P_val must be a contiguous {want} GPU tensor")
    if P_val.numel() < plan.nnz_P:
        raise ValueError(f"P_val holds {P_val.numel()} values, the plan needs {plan.nnz_P}")
    batched = plan.n_systems > 1
    if batched and np.ndim(n_occ) != 1:
        raise ValueError("a batched plan takes one n_occ per system")
    c = H.as_c()
    o, keep = make_run_options(max_iter, alpha_seq, stop_rule, trace_tol, timing, precision, refine, persistent,
                               n_occ_system=n_occ if batched else None, symmetrize=symmetrize, kernel=kernel,
                               refine_precision=refine_precision)
    info = (gsp2_run_info * plan.n_systems)() if want_info else None
    st = getattr(load(), entry)(plan.handle, C.byref(c), 0.0 if batched else float(n_occ), C.byref(o),
                                C.c_void_p(P_val.data_ptr()), info)
    del keep
    msg = load().gsp2_last_error().decode()
    if check and st != GSP2_OK:
        raise Gsp2Error(st, msg)
    if info is None:
        return {"status": st}
    ds = [run_info_dict(x) for x in info]
    for d in ds:
        d["call_status"] = st
        d["message"] = msg
    return ds if batched else ds[0]


def gsp2_density(plan: Plan, H: DeviceCSR, n_occ, P_val, **kw):
    """gsp2_density: one density matrix into P_val (see _density)."""
    return _density("gsp2_density", plan, H, n_occ, P_val, **kw)


def gsp2_density_noalloc(plan: Plan, H: DeviceCSR, n_occ, P_val, **kw):
    """gsp2_density_noalloc: the same run with its buffers in the library's
    static device scratch and no allocation (no timing option)."""
    return _density("gsp2_density_noalloc", plan, H, n_occ, P_val, **kw)


def gsp2_run_status(plan: Plan):
    info = (gsp2_run_info * plan.n_systems)()
    st = load().gsp2_run_status(plan.handle, info)
    ds = [run_info_dict(x) for x in info]
    for d in ds:
        d["call_status"] = st
    return ds if plan.n_systems > 1 else ds[0]


def gsp2_run_timing(plan: Plan) -> dict:
    t = gsp2_timing()
    _check(load().gsp2_run_timing(plan.handle, C.byref(t)))
    return {"n_products": t.n_products, "setup_ms": t.setup_ms, "sp2_ms": t.sp2_ms,
            "scatter_ms": t.scatter_ms, "total_ms": t.total_ms, "persistent_ms": t.persistent_ms,
            "product_ms": [float(x) for x in t.product_ms[:t.n_products]]}


def gsp2_backward(plan: Plan, H: DeviceCSR, alpha_seq, dLdP_val, dLdH_val=None) -> tuple:
    """dL/dH (torch float64 on the GPU, one value per stored entry of H) for a
    forward run with branch sequence alpha_seq, given dL/dP_val.  Returns
    (dLdH_val, info dict)."""
    import torch
    if dLdP_val.dtype != torch.float32 or not dLdP_val.is_cuda or not dLdP_val.is_contiguous():
        raise ValueError("dLdP_val must be a contiguous float32 GPU tensor")
    if dLdP_val.numel() < plan.nnz_P:
        raise ValueError("dLdP_val is shorter than the plan's P")
    if dLdH_val is None:
        dLdH_val = torch.empty(H.nnz, dtype=torch.float64, device=dLdP_val.device)
    if dLdH_val.dtype != torch.float64 or dLdH_val.numel() < H.nnz:
        raise ValueError("dLdH_val must hold H.nnz float64 values")
    seq = np.ascontiguousarray(alpha_seq, dtype=np.int8)
    c = H.as_c()
    info = gsp2_backward_info()
    _check(load().gsp2_backward(plan.handle, C.byref(c), seq.ctypes.data_as(C.POINTER(C.c_int8)), int(seq.size),
                                C.c_void_p(dLdP_val.data_ptr()), C.c_void_p(dLdH_val.data_ptr()), C.byref(info)))
    return dLdH_val, {f: getattr(info, f) for f, _ in gsp2_backward_info._fields_}


def gsp2_plan_destroy(plan: Plan):
    plan.close()


def gsp2_core_halo_host(adj_ptr, adj_col, part, n_parts: int):
    """Host planning step: (sub_ptr, sub_idx, core_count) for a directed adjacency."""
    adj_ptr = np.ascontiguousarray(adj_ptr, dtype=np.int64)
    adj_col = np.ascontiguousarray(adj_col, dtype=np.int32)
    part = np.ascontiguousarray(part, dtype=np.int32)
    n = part.size
    if adj_ptr.size != n + 1:
        raise ValueError("adj_ptr must have n+1 entries")
    lib = load()
    sub_ptr = np.empty(n_parts + 1, dtype=np.int64)
    _check(lib.gsp2_core_halo_host(n, _i64(adj_ptr), _i32(adj_col), _i32(part), int(n_parts),
                                   _i64(sub_ptr), None, None))
    sub_idx = np.empty(int(sub_ptr[-1]), dtype=np.int32)
    core = np.empty(n_parts, dtype=np.int32)
    _check(lib.gsp2_core_halo_host(n, _i64(adj_ptr), _i32(adj_col), _i32(part), int(n_parts),
                                   _i64(sub_ptr), _i32(sub_idx), _i32(core)))
    return sub_ptr, sub_idx, core


def gsp2_sparse_sp2_host(H, n_occ, eps: float, max_iter: int = 60, check: bool = True):
    """Host: the first density matrix of H (scipy sparse, FP64) by SP2 in
    thresholded sparse algebra (gsp2_sparse_sp2_host in gsp2.h).  Returns
    (P as scipy.sparse.csr_matrix, info dict); with check a failing run
    status raises Gsp2Error."""
    import scipy.sparse as sp
    H = sp.csr_matrix(H, dtype=np.float64)
    n = H.shape[0]
    rp = np.ascontiguousarray(H.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(H.indices, dtype=np.int32)
    hv = np.ascontiguousarray(H.data, dtype=np.float64)
    lib = load()
    ptr = np.empty(n + 1, dtype=np.int64)
    info = gsp2_sparse_sp2_info()
    args = (n, _i64(rp), _i32(ci), hv.ctypes.data_as(C.POINTER(C.c_double)), float(n_occ), float(eps), int(max_iter))
    st = lib.gsp2_sparse_sp2_host(*args, _i64(ptr), None, None, C.byref(info))
    if st not in (GSP2_OK, GSP2_E_NOT_CONVERGED, GSP2_E_WRONG_TRACE):
        _check(st)
    col = np.empty(int(ptr[-1]), dtype=np.int32)
    val = np.empty(int(ptr[-1]), dtype=np.float64)
    st = lib.gsp2_sparse_sp2_host(*args, _i64(ptr), _i32(col), val.ctypes.data_as(C.POINTER(C.c_double)),
                                  C.byref(info))
    if check:
        _check(st)
    d = {f: getattr(info, f) for f, _ in gsp2_sparse_sp2_info._fields_ if f not in ("alpha", "pad_")}
    d["alpha"] = [int(a) for a in info.alpha[:info.n_alpha]]
    d["status_name"] = STATUS_NAMES.get(info.status, str(info.status))
    return sp.csr_matrix((val, col, ptr), shape=(n, n)), d

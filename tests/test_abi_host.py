"""The C-ABI library without a GPU: it loads, exports every declared symbol,
and its host planning step matches the oracle's core/halo sets."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_1801_10016_amd as g
from paper_1801_10016_amd import gsp2 as binding
from synth.partition import uneven_spatial_partition
from tests import _pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gsp2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsp2_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = g.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.SIGNATURES) == names


def test_status_strings_and_defaults():
    lib = g.load()
    for code, name in g.STATUS_NAMES.items():
        assert lib.gsp2_status_string(code).decode() == name
    o = g.gsp2_run_options_default()
    assert (o.max_iter, o.alpha_mode, o.n_alpha, o.stop_rule, o.trace_tol) == (60, 0, 0, 1, 0.5)


def _as_csr(adj):
    adj = sp.csr_matrix(adj)
    return adj.indptr.astype(np.int64), adj.indices.astype(np.int32)


def _compare(adj, part, n_parts):
    ptr, col = _as_csr(adj)
    sub_ptr, sub_idx, core = g.gsp2_core_halo_host(ptr, col, part, n_parts)
    cores, halos = oracle.core_halo(oracle.threshold_graph(adj, 0.5), part, n_parts)
    for k in range(n_parts):
        got = sub_idx[sub_ptr[k]:sub_ptr[k + 1]]
        want = np.concatenate([cores[k], halos[k]])
        assert np.array_equal(got, want), k
        assert core[k] == len(cores[k])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_core_halo_host_matches_oracle_random(seed):
    rng = np.random.default_rng(seed)
    n, k = 200, 7
    A = (rng.random((n, n)) < 0.03).astype(float)   # directed: the union must be taken
    part = rng.integers(0, k, n).astype(np.int32)
    part[:k] = np.arange(k)
    _compare(sp.csr_matrix(A), part, k)


def test_core_halo_host_matches_oracle_water():
    s = pins.water(64, 0)
    P, _ = oracle.dense_sp2(s.H, s.n_occ)
    part = uneven_spatial_partition(s, 8, seed=0)
    for tau in (1e-5, 1e-3, 1e-2):
        A = oracle.threshold_graph(P, tau)
        _compare(A, part, 8)


def test_core_halo_host_fig2():
    # the worked example of Fig. 2 through the library's planner
    import json
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "fig2_corehalo.json")))
    ix = {v: i for i, v in enumerate(fx["vertices"])}
    A = np.zeros((6, 6))
    for a, b in fx["edges"]:
        A[ix[a], ix[b]] = 1.0          # one orientation only
    for key in ("a", "b"):
        case = fx["partitions"][key]
        part = np.empty(6, dtype=np.int32)
        for k, members in enumerate(case["parts"]):
            part[[ix[v] for v in members]] = k
        ptr, col = _as_csr(A)
        sub_ptr, _, _ = g.gsp2_core_halo_host(ptr, col, part, 2)
        sizes = np.diff(sub_ptr)
        assert sizes.tolist() == case["sizes"]
        assert int((sizes.astype(np.int64) ** 3).sum()) == case["cost"]


def test_core_halo_host_rejects_bad_partitions():
    ptr = np.array([0, 1, 2, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    with pytest.raises(g.Gsp2Error) as e:
        g.gsp2_core_halo_host(ptr, col, np.array([0, 0, 2], dtype=np.int32), 3)    # part 1 empty
    assert e.value.status == binding.GSP2_E_INVALID
    with pytest.raises(g.Gsp2Error):
        g.gsp2_core_halo_host(ptr, col, np.array([0, 1, 5], dtype=np.int32), 3)    # id out of range
    with pytest.raises(g.Gsp2Error):
        g.gsp2_core_halo_host(ptr, np.array([1, 7], dtype=np.int32), np.array([0, 1, 2], dtype=np.int32), 3)


def test_core_halo_host_isolated_vertices_and_self_loops():
    # self loops and isolated vertices: halos stay empty
    A = sp.identity(5, format="csr")
    part = np.array([0, 0, 1, 1, 2], dtype=np.int32)
    ptr, col = _as_csr(A)
    sub_ptr, sub_idx, core = g.gsp2_core_halo_host(ptr, col, part, 3)
    assert np.diff(sub_ptr).tolist() == [2, 2, 1]
    assert sub_idx.tolist() == [0, 1, 2, 3, 4]


def test_binding_structs_match_the_header(tmp_path):
    """sizeof and offsetof of every ABI struct, compiled from the header by the
    host C compiler, equal the ctypes layouts of the binding."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [binding.gsp2_csr, binding.gsp2_plan_options, binding.gsp2_plan_info, binding.gsp2_run_options,
               binding.gsp2_run_info, binding.gsp2_timing, binding.gsp2_backward_info, binding.gsp2_tune_info,
               binding.gsp2_sparse_sp2_info, binding.gsp2_anneal_options]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gsp2.h"', "int main(void) {"]
    for cls in structs:
        name = cls.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for cls in structs:
        name = cls.__name__
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def _plan_create_host(part, n_parts, n_systems, part_system, tile16=0):
    """gsp2_plan_create with host arrays: only its argument checks, which run
    before any HIP call, are reached when the arguments are invalid."""
    import ctypes as C
    n = part.size
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    c = binding.gsp2_csr(n, 0, row_ptr.ctypes.data, None, None, binding.GSP2_F64)
    opt = binding.gsp2_plan_options(0)
    keep = None
    if part_system is not None:
        keep = np.ascontiguousarray(part_system, dtype=np.int32)
        opt.part_system = keep.ctypes.data_as(C.POINTER(C.c_int32))
    opt.n_systems = n_systems
    opt.tile16 = tile16
    out = C.c_void_p()
    part = np.ascontiguousarray(part, dtype=np.int32)
    st = g.load().gsp2_plan_create(C.byref(c), 1e-3, part.ctypes.data_as(C.POINTER(C.c_int32)), n_parts,
                                   C.byref(opt), None, C.byref(out))
    return st, g.load().gsp2_last_error().decode(), out.value


@pytest.mark.parametrize("n_systems,part_system,message", [
    (3, [0, 1], "more systems than parts"),
    (2, None, "null part_system"),
    (2, [0, 2], "part_system out of range"),
    (2, [1, 1], "system 0 has no part"),
    (-1, [0, 0], "n_systems must be >= 0"),
])
def test_batched_plan_arguments_are_checked(n_systems, part_system, message):
    part = np.array([0, 0, 1, 1], dtype=np.int32)
    st, msg, handle = _plan_create_host(part, 2, n_systems, part_system)
    assert st == binding.GSP2_E_INVALID and message in msg and handle is None


@pytest.mark.parametrize("tile16", [64, 512, -1])
def test_tile16_option_is_checked(tile16):
    part = np.array([0, 0, 1, 1], dtype=np.int32)
    st, msg, handle = _plan_create_host(part, 2, 0, None, tile16)
    assert st == binding.GSP2_E_INVALID and "tile16" in msg and handle is None


def test_tune_rejects_bad_arguments_before_any_gpu_call():
    import ctypes as C
    c = binding.gsp2_csr(4, 0, None, None, None, binding.GSP2_F64)
    lib = g.load()
    assert lib.gsp2_plan_tune(None, C.byref(c), 1.0, binding.GSP2_PREC_FP16, 8, None) == binding.GSP2_E_INVALID
    assert "null" in lib.gsp2_last_error().decode()


def test_probe_rejects_bad_arguments_before_any_gpu_call():
    import ctypes as C
    lib = g.load()
    out = C.c_double()
    assert lib.gsp2_probe_mfma(99, None, C.byref(out)) == binding.GSP2_E_INVALID
    assert "precision" in lib.gsp2_last_error().decode()
    assert lib.gsp2_probe_mfma(binding.GSP2_PREC_FP32, None, None) == binding.GSP2_E_INVALID


def test_run_option_defaults_leave_batch_fields_empty():
    o = g.gsp2_run_options_default()
    assert not o.n_occ_system and not o.alpha_seq_system and not o.n_alpha_system

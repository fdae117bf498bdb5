"""The stored expectations of the full-size tests, without a GPU: they are
complete and self-consistent, and what the oracle's graph side recomputes
cheaply (the stand-in graph's threshold, cores and halos) matches them."""
import os

import numpy as np
import pytest

import oracle
from synth import sketch
from synth.locality import surrogate_prev_density
from synth.partition import uneven_spatial_partition
from synth.water import make_water
from tests import _full

STEMS = ["gsp2_water3500_densep_tau1e-5", "gsp2_water3500_tau1e-5"]


def _have(stem):
    return all(os.path.exists(os.path.join(_full.GOLDEN, stem + ext)) for ext in (".json", ".npz"))


@pytest.mark.parametrize("stem", STEMS)
def test_golden_is_complete(stem):
    if not _have(stem):
        pytest.skip(f"{stem} not written yet")
    gold, arrays = _full.load_golden(stem)
    sp_ = gold["spec"]
    assert (sp_["n_mol"], sp_["n_parts"], sp_["tau"]) == (3500, 128, 1e-5)
    assert gold["status"] == "ok" and gold["converged"]
    assert len(gold["parts"]) == sp_["n_parts"] and sum(p["c"] for p in gold["parts"]) == gold["n"]
    assert arrays["part_sketch"].shape == (sp_["n_parts"], sketch.SKETCH_M, sketch.SKETCH_R)
    assert np.isfinite(arrays["part_sketch"]).all()
    assert len(gold["alphas"]) == len(gold["traces"]) - 1 and len(gold["errors"]) == gold["n_products"]
    assert abs(gold["traces"][-1] - gold["n_occ"]) <= 0.5
    for k in gold["sample_parts"]:
        idx = arrays[f"index_{k}"]
        p = gold["parts"][k]
        assert len(idx) == p["s"] and _full.index_digest(idx) == p["idx_sha256"]
        assert np.all(np.diff(idx[:p["c"]]) > 0) and np.all(np.diff(idx[p["c"]:]) > 0)
    if "dense_run" in gold:
        d = gold["dense_run"]
        assert d["status"] == "ok" and abs(d["trace_P"] - gold["n_occ"]) <= 1e-6
        assert d["idempotency_rel"] <= 1e-12
        assert arrays["dense_sketch"].shape == (sketch.SKETCH_M, sketch.SKETCH_R)
        assert gold["near_tau"] == []          # no entry near enough tau for rounding to move an edge


def test_standin_graph_and_parts_recomputed():
    stem = "gsp2_water3500_tau1e-5"
    if not _have(stem):
        pytest.skip(f"{stem} not written yet")
    gold, _ = _full.load_golden(stem)
    sp_ = gold["spec"]
    s = make_water(sp_["n_mol"], sp_["seed"])
    part = uneven_spatial_partition(s, sp_["n_parts"], sp_["core_lo"], sp_["core_hi"], seed=sp_["seed"])
    adj = oracle.threshold_graph(surrogate_prev_density(s, sp_["q_floor"]), sp_["tau"])
    digest, nnz = _full.graph_digest(adj.indptr.astype(np.int64), adj.indices.astype(np.int32), s.n)
    assert nnz == gold["graph"]["nnz_sym"] and digest == gold["graph"]["sha256"]
    cores, halos = oracle.core_halo(adj, part, sp_["n_parts"])
    for k, p in enumerate(gold["parts"]):
        idx = oracle.subproblem_index(cores[k], halos[k])
        assert (len(idx), len(cores[k])) == (p["s"], p["c"])
        assert _full.index_digest(idx) == p["idx_sha256"], k

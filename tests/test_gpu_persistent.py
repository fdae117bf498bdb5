"""All products of a run in one persistent launch (grid barrier per
product) against one launch per product: the same tiles, the same
fixed-order reductions and the same decisions, so P must be bitwise equal."""
import numpy as np
import pytest

import oracle
from synth.partition import uneven_spatial_partition
from tests import _pins as pins

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="persistent product launch switched off: its first GPU run did not return "
                            "within 120 s and the cause has not been established (see the design notes)"),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n_mol,n_parts,tau,kw", [
    (64, 8, 1e-5, {}),
    (200, 6, 1e-4, {}),
    (200, 6, 1e-4, {"precision": "fp16"}),
    (100, 3, 1e-3, {"precision": "bf16", "refine": 2}),
    (64, 8, 1e-3, {"alpha_seq": [1, -1, 1, -1, -1], "trace_tol": 1e9}),
])
def test_persistent_matches_per_product_launches(n_mol, n_parts, tau, kw):
    from tests._gpu import rel_fro, run_gsp2
    s = pins.water(n_mol, 0)
    Pp = pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    part = uneven_spatial_partition(s, n_parts, seed=0)
    print(f"persistent: N={s.n} parts={n_parts} tau={tau} {kw}", flush=True)
    P1, r1, _, _, v1 = run_gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, **kw)
    P2, r2, _, _, v2 = run_gsp2(s.H, Pp, tau, part, n_parts, s.n_occ, persistent=True, **kw)
    print(f"  products {r1['n_products']} / {r2['n_products']}, status {r1['status']} / {r2['status']}", flush=True)
    assert r2["status"] == r1["status"] and r2["n_products"] == r1["n_products"]
    assert r2["alpha"] == r1["alpha"] and r2["result_iterate"] == r1["result_iterate"]
    assert np.array_equal(v1, v2)
    if not kw:
        ref = oracle.gsp2(s.H, Pp, tau, part, n_parts, s.n_occ)
        assert rel_fro(P2, ref.csc()) <= 1e-5 or r2["alpha"] != ref.sp2.alphas


def test_persistent_single_part_and_stop_budget():
    from tests._gpu import run_gsp2
    s = pins.water(32, 1)
    part = np.zeros(s.n, dtype=np.int32)
    Pp = pins.cached(("dense", s.n_mol, s.seed, s.hop_a), lambda: oracle.dense_sp2(s.H, s.n_occ)[0])
    for max_iter in (3, 60):
        _, r1, _, _, v1 = run_gsp2(s.H, Pp, 1e-5, part, 1, s.n_occ, max_iter=max_iter, check=False)
        _, r2, _, _, v2 = run_gsp2(s.H, Pp, 1e-5, part, 1, s.n_occ, max_iter=max_iter, check=False,
                                   persistent=True)
        assert r1["status"] == r2["status"] and np.array_equal(v1, v2)


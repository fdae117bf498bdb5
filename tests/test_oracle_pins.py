"""The FP64 oracle against what the paper and mathematics fix."""
import numpy as np
import pytest

import oracle
from synth.partition import block_partition
from tests import _pins as pins


def test_gershgorin_textbook_cases():
    pins.check_gershgorin_textbook()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gershgorin_contains_spectrum(seed):
    pins.check_gershgorin_contains(pins.water(64, seed).H)
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(30, 30))
    pins.check_gershgorin_contains(A + A.T)


def test_initial_guess_reverses_spectrum_into_unit_interval():
    pins.check_initial_guess(pins.water(16, 0).H)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_sp2_is_the_eigen_projector(seed):
    s = pins.water(64, seed)
    assert oracle.spectral_gap(s.H, s.n_occ) >= 1.0   # seed rejection rule of the system recipe
    pins.check_dense_projector(s)


def test_every_iterate_is_the_branch_polynomial():
    pins.check_iterates_are_polynomials(pins.water(16, 1))


def test_branch_rule_direction():
    pins.check_branch_direction(pins.water(64, 0))


def test_diagonal_hamiltonian_gives_step_function():
    pins.check_diagonal_step()


def test_monomer_closed_form_and_exact_gsp2():
    pins.check_monomer()


def test_fig2_core_halo_costs():
    pins.check_fig2()


def test_threshold_is_strict_and_undirected():
    pins.check_threshold_rule()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_halo_matches_brute_force(seed):
    pins.check_halo_brute_force(seed)


def test_block_partition_polyalanine_counts():
    # 41,185 vertices in 1,200 block parts have 34 or 35 cores each
    part = block_partition(41185, 1200)
    sizes = np.bincount(part)
    assert sizes.sum() == 41185 and len(sizes) == 1200
    assert set(sizes.tolist()) == {34, 35}
    assert (sizes == 35).sum() == 385 and (sizes == 34).sum() == 815
    assert np.all(np.diff(part) >= 0)


def test_gsp2_one_part_is_dense_sp2():
    pins.check_gsp2_one_part_is_dense(pins.water(32, 0))


def test_gsp2_complete_halo_is_dense_sp2():
    pins.check_gsp2_full_halo_is_dense(pins.water(24, 2))


def test_symmetrize_on_the_pattern():
    pins.check_symmetrize(pins.water(32, 0))


def test_occupation_check_of_a_stopped_run():
    pins.check_occupation_status(pins.water(32, 0))


def test_gsp2_truncation_error_is_order_tau():
    pins.check_gsp2_truncation(pins.water(64, 0))


def test_gsp2_blocks_share_one_branch_sequence():
    pins.check_gsp2_blocks_share_sequence(pins.water(64, 0))


def test_stop_rule_failures():
    s = pins.water(32, 0)
    _, res = oracle.dense_sp2(s.H, s.n_occ, max_iter=5)
    assert not res.converged and res.status == "not_converged" and res.n_products == 5
    with pytest.raises(oracle.NotConverged):
        oracle.dense_sp2(s.H, s.n_occ, max_iter=5, raise_on_failure=True)
    P, ok = oracle.dense_sp2(s.H, s.n_occ)
    # replaying the recorded sequence reproduces the result and passes the trace check
    Pr, rep = oracle.dense_sp2(s.H, s.n_occ, alpha_seq=ok.alphas)
    assert rep.converged and np.array_equal(Pr, P)
    # a corrupted sequence must be caught by the final trace check
    bad = list(ok.alphas)
    bad[3] = -bad[3]
    _, wr = oracle.dense_sp2(s.H, s.n_occ, alpha_seq=bad)
    assert wr.status == "wrong_trace"
    with pytest.raises(oracle.WrongTrace):
        oracle.dense_sp2(s.H, s.n_occ, alpha_seq=bad, raise_on_failure=True)


def test_empty_and_full_occupation():
    s = pins.water(8, 0)
    P0, r0 = oracle.dense_sp2(s.H, 0)
    assert r0.converged and np.abs(P0).max() < 1e-12
    P1, r1 = oracle.dense_sp2(s.H, s.n)
    assert r1.converged and np.allclose(P1, np.eye(s.n), atol=1e-12)


def test_adjoint_matches_central_differences():
    pins.check_adjoint_finite_differences()


def test_adjoint_closed_form_and_hellmann_feynman():
    pins.check_adjoint_closed_form()


@pytest.mark.parametrize("n_mol,seed", [(64, 1), (100, 0)])
def test_thresholded_sp2_bounds(n_mol, seed):
    pins.check_thresholded_sp2(pins.water(n_mol, seed))

"""A distance-based stand-in for a previously computed density matrix.

The graph of G-SP2 comes from thresholding the P of an earlier step.  Where
that earlier P is too costly for the FP64 CPU oracle to recompute (tens of
thousands of orbitals), both the oracle and the GPU library instead
threshold this cheap, deterministic surrogate, built from atom distances
alone, as the paper's locality-based construction of sub-problems does.

Surrogate entry for orbitals u != v on atoms at minimum-image distance r:

    Q_uv = 1e-3 * exp(-(r - R3) / XI)

with R3 = 4.42 Angstrom and XI = 1.12 Angstrom.  These two constants were
fitted to the FP64 dense-SP2 P of the 500-molecule system (seed 0): a
sharp sphere of radius R3 + XI ln(1e-3 / tau) then holds as many
neighbours per orbital as the real P thresholded at tau, for
tau in {1e-3, 1e-4, 1e-5} (mean degrees 71, 263, 729).  Entries with
Q_uv <= q_floor are not stored.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .water import WaterSystem, _min_image

R3 = 4.42
XI = 1.12


def surrogate_radius(q: float) -> float:
    return R3 + XI * np.log(1e-3 / q)


def surrogate_prev_density(system: WaterSystem, q_floor: float = 5e-6) -> sp.csr_matrix:
    """FP64 CSR, symmetric, unit diagonal, entries Q_uv > q_floor."""
    L = system.box
    rmax = surrogate_radius(q_floor)
    if rmax >= 0.5 * L:
        raise ValueError("surrogate radius exceeds half the box; use the real P instead")
    atoms = system.atoms
    oa = system.orbital_atom()
    tree = cKDTree(atoms, boxsize=L)
    pairs = tree.query_pairs(rmax, output_type="ndarray")
    d = _min_image(atoms[pairs[:, 1]] - atoms[pairs[:, 0]], L)
    r = np.linalg.norm(d, axis=1)
    q = 1e-3 * np.exp(-(r - R3) / XI)
    keep = q > q_floor
    pairs, q = pairs[keep], q[keep]
    # atom pair -> all orbital pairs; orbitals of one atom are contiguous
    n_atoms = atoms.shape[0]
    first = np.searchsorted(oa, np.arange(n_atoms))
    count = np.bincount(oa, minlength=n_atoms)
    rows, cols, vals = [], [], []
    same = 1e-3 * np.exp(R3 / XI)
    for a_cnt in np.unique(count):
        for b_cnt in np.unique(count):
            sel = (count[pairs[:, 0]] == a_cnt) & (count[pairs[:, 1]] == b_cnt)
            if not sel.any():
                continue
            pa, pb, qv = pairs[sel, 0], pairs[sel, 1], q[sel]
            ua = first[pa][:, None] + np.arange(a_cnt)[None, :]
            vb = first[pb][:, None] + np.arange(b_cnt)[None, :]
            ru = np.repeat(ua, b_cnt, axis=1).ravel()
            cv = np.tile(vb, (1, a_cnt)).ravel()
            v = np.repeat(qv, a_cnt * b_cnt)
            rows += [ru, cv]; cols += [cv, ru]; vals += [v, v]
    # orbitals on the same atom (r = 0), and the unit diagonal
    for a_cnt in np.unique(count):
        if a_cnt < 2:
            continue
        at = np.flatnonzero(count == a_cnt)
        u = first[at][:, None] + np.arange(a_cnt)[None, :]
        ru = np.repeat(u, a_cnt, axis=1).ravel()
        cv = np.tile(u, (1, a_cnt)).ravel()
        off = ru != cv
        rows.append(ru[off]); cols.append(cv[off]); vals.append(np.full(off.sum(), same))
    n = system.n
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(np.ones(n))
    Q = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    Q.sum_duplicates()
    Q.sort_indices()
    return Q

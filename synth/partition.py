"""Partitions of the orbital set, used as inputs (the partition is an argument
of the G-SP2 plan, never computed inside it).

* ``block_partition``: a fixed number of consecutive orbitals per part, in
  index order (the block scheme of the paper).
* ``uneven_spatial_partition``: whole molecules grouped into compact
  spatial parts of deliberately uneven target sizes, by recursive
  coordinate bisection with weighted cuts.  It stands in for an
  off-the-shelf graph partitioner, which is not available here, and for the
  paper's locality-based construction of cores.
"""
from __future__ import annotations

import numpy as np

from .water import ORB_PER_MOL, WaterSystem


def block_partition(n: int, n_parts: int) -> np.ndarray:
    """Part id of each of n vertices: parts of floor(n/k) or ceil(n/k)
    consecutive vertices, the larger ones first."""
    if n_parts < 1 or n_parts > n:
        raise ValueError("need 1 <= n_parts <= n")
    base, extra = divmod(n, n_parts)
    sizes = np.full(n_parts, base, dtype=np.int64)
    sizes[:extra] += 1
    return np.repeat(np.arange(n_parts, dtype=np.int32), sizes)


def uneven_targets(n_units: int, n_parts: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Integer part sizes (in units) drawn U[lo, hi], rescaled to sum to n_units,
    each at least one unit."""
    if n_parts > n_units:
        raise ValueError("more parts than units")
    rng = np.random.default_rng(seed)
    w = rng.uniform(lo, hi, size=n_parts)
    t = w / w.sum() * n_units
    sizes = np.maximum(1, np.floor(t).astype(np.int64))
    # distribute the remainder by largest fractional part, deterministic
    diff = n_units - sizes.sum()
    order = np.argsort(-(t - np.floor(t)), kind="stable")
    i = 0
    while diff != 0:
        j = order[i % n_parts]
        if diff > 0:
            sizes[j] += 1; diff -= 1
        elif sizes[j] > 1:
            sizes[j] -= 1; diff += 1
        i += 1
    return sizes


def _rcb(points: np.ndarray, ids: np.ndarray, targets: np.ndarray, first_part: int,
         out: np.ndarray) -> None:
    if len(targets) == 1:
        out[ids] = first_part
        return
    half = len(targets) // 2
    n_left = int(targets[:half].sum())
    ext = points[ids].max(axis=0) - points[ids].min(axis=0)
    axis = int(np.argmax(ext))
    order = np.argsort(points[ids, axis], kind="stable")
    left, right = ids[order[:n_left]], ids[order[n_left:]]
    _rcb(points, left, targets[:half], first_part, out)
    _rcb(points, right, targets[half:], first_part + half, out)


def uneven_spatial_partition(system: WaterSystem, n_parts: int, core_lo: float = 60.0,
                             core_hi: float = 300.0, seed: int = 0) -> np.ndarray:
    """Part id per orbital.  Core sizes (orbitals) are drawn U[core_lo, core_hi]
    and rescaled so they sum to N; molecules are never split."""
    lo = core_lo / ORB_PER_MOL
    hi = core_hi / ORB_PER_MOL
    sizes = uneven_targets(system.n_mol, n_parts, lo, hi, seed)
    mol_part = np.empty(system.n_mol, dtype=np.int32)
    _rcb(system.centres, np.arange(system.n_mol), sizes, 0, mol_part)
    return np.repeat(mol_part, ORB_PER_MOL).astype(np.int32)


def molecule_partition(system: WaterSystem) -> np.ndarray:
    """One part per molecule."""
    return np.repeat(np.arange(system.n_mol, dtype=np.int32), ORB_PER_MOL)

"""Input recipe of the uneven batch: independent water systems, each taken
one molecular-dynamics step forward, whose density matrices are computed
together in one batched plan.

For system i of the batch:

* molecule count drawn log-uniform in [lo, hi] molecules (one generator
  seeded by ``seed`` draws all counts), system built by ``make_water`` with
  seed ``seed + 1 + i``;
* previous density matrix: the distance-based surrogate of the system as
  built (entries above tau / 2 stored, so the library's threshold, not the
  generator, decides the graph);
* the step: every atom coordinate displaced by N(0, sigma^2), sigma = 0.05
  Angstrom, and H rebuilt from the displaced atoms;
* the graph repartitioned for the displaced atoms: whole molecules in
  compact spatial parts, core sizes drawn U[core_lo, core_hi] orbitals and
  rescaled to the system, round(n / mean_core) parts.

The batch is the block-diagonal union of the systems, with parts numbered
system by system.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .locality import surrogate_prev_density
from .partition import uneven_spatial_partition
from .water import WaterSystem, make_water, perturb


def batch_sizes(n_systems: int = 16, lo: int = 500, hi: int = 8000, seed: int = 2018) -> np.ndarray:
    """Molecule counts, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n_systems)).astype(np.int64)


@dataclass
class SystemStep:
    system: WaterSystem          # the displaced system (its H is the step's H)
    P_prev: sp.csr_matrix        # previous density matrix (surrogate of the undisplaced system)
    part: np.ndarray             # part of every orbital, 0 .. n_parts-1
    n_parts: int


@dataclass
class BatchInputs:
    steps: list
    tau: float
    H: sp.csr_matrix = field(repr=False)
    P_prev: sp.csr_matrix = field(repr=False)
    part: np.ndarray = field(repr=False)
    part_system: np.ndarray = field(repr=False)
    offs: np.ndarray = field(repr=False)         # first orbital of every system, and n
    part_offs: np.ndarray = field(repr=False)    # first part of every system, and n_parts

    @property
    def n_occ(self) -> list:
        return [st.system.n_occ for st in self.steps]

    @property
    def n_parts(self) -> int:
        return int(self.part_offs[-1])


def system_step(n_mol: int, seed: int, tau: float, sigma: float = 0.05, core_lo: float = 60.0,
                core_hi: float = 300.0, mean_core: float = 150.0) -> SystemStep:
    s0 = make_water(int(n_mol), seed)
    P_prev = surrogate_prev_density(s0, q_floor=0.5 * tau)
    s1 = perturb(s0, sigma, seed + 7919)
    n_parts = max(1, int(round(s1.n / mean_core)))
    part = uneven_spatial_partition(s1, n_parts, core_lo, core_hi, seed=seed)
    return SystemStep(s1, P_prev, part, n_parts)


def join(steps: list, tau: float) -> BatchInputs:
    """Block-diagonal union of independent steps."""
    offs = np.cumsum([0] + [st.system.n for st in steps])
    part_offs = np.cumsum([0] + [st.n_parts for st in steps])
    H = sp.block_diag([st.system.H for st in steps], format="csr")
    H.sort_indices()
    P_prev = sp.block_diag([st.P_prev for st in steps], format="csr")
    part = np.concatenate([st.part + po for st, po in zip(steps, part_offs)]).astype(np.int32)
    part_system = np.repeat(np.arange(len(steps)), [st.n_parts for st in steps]).astype(np.int32)
    return BatchInputs(steps, tau, H, P_prev, part, part_system, offs, part_offs)


def make_batch(n_systems: int = 16, lo: int = 500, hi: int = 8000, seed: int = 2018, tau: float = 1e-4,
               sigma: float = 0.05) -> BatchInputs:
    sizes = batch_sizes(n_systems, lo, hi, seed)
    steps = [system_step(m, seed + 1 + i, tau, sigma) for i, m in enumerate(sizes)]
    return join(steps, tau)

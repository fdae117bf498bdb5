"""Seeded synthetic water-like tight-binding systems.

This module only builds inputs: atom positions, orbital layout and the
Hamiltonian H.  It holds none of the density-matrix arithmetic; both the
FP64 oracle and the GPU library consume what it returns.

System recipe (the paper's own water, protein and urea inputs are not
available, so this stands in for them):

* M molecules, O atom uniform in a cubic, 3D-periodic box at
  0.033 molecules per cubic Angstrom, then pushed apart until every pair of
  O atoms is at least 3.1 Angstrom apart (minimum image).  Random
  sequential addition cannot reach this packing fraction (0.515), so
  positions are relaxed by gradient descent on the overlap penalty
  sum((1.02 d - r)_+^2) instead.
* Orientation: a uniformly random unit quaternion per molecule; H atoms at
  0.96 Angstrom from O with an H-O-H angle of 104.5 degrees.
* Orbitals, in global order per molecule: O s (-20 eV), O p x3 (-10 eV),
  H1 (-5 eV), H2 (-5 eV).
* Intramolecular hopping: each of the four O orbitals couples with -4 eV to
  each H orbital; no H-H term inside a molecule.
* Intermolecular hopping: every orbital pair on two atoms of different
  molecules at minimum-image distance r < 4.5 Angstrom couples with
  -A exp(-(r - 2.5)/lam), A = 0.5 eV, lam = 0.5 Angstrom.
* Four occupied states per molecule (eight valence electrons).

Seeds: positions come from ``numpy.random.default_rng(seed)``, orientations
from ``default_rng(seed + 1000)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

DENSITY = 0.033          # molecules per cubic Angstrom
MIN_SEP = 3.1            # minimum O-O distance (Angstrom)
R_OH = 0.96              # O-H bond length (Angstrom)
ANGLE_HOH = np.deg2rad(104.5)
ONSITE = np.array([-20.0, -10.0, -10.0, -10.0, -5.0, -5.0])
T_INTRA = -4.0           # O orbital <-> H orbital, same molecule
HOP_A = 0.5              # intermolecular prefactor (eV)
HOP_LAM = 0.5            # intermolecular decay length (Angstrom)
HOP_R0 = 2.5             # reference distance (Angstrom)
HOP_RCUT = 4.5           # hard cutoff (Angstrom)
ORB_PER_MOL = 6
OCC_PER_MOL = 4

# atom kind per atom slot in a molecule (0 = O, 1 = H1, 2 = H2) and the
# orbitals each atom slot owns, as offsets inside the molecule's 6 orbitals
_ATOM_ORBS = (np.array([0, 1, 2, 3]), np.array([4]), np.array([5]))


@dataclass
class WaterSystem:
    """One synthetic system.  Orbital ``6 m + q`` belongs to molecule m."""

    n_mol: int
    box: float
    atoms: np.ndarray            # (3M, 3) positions, atom 3m = O, 3m+1/3m+2 = H
    H: sp.csr_matrix             # (N, N) FP64, symmetric, sorted indices
    n_occ: int
    seed: int
    hop_a: float = HOP_A
    hop_lam: float = HOP_LAM
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n_mol * ORB_PER_MOL

    @property
    def centres(self) -> np.ndarray:
        return self.atoms[0::3]

    def orbital_atom(self) -> np.ndarray:
        """Atom index of every orbital."""
        m = np.repeat(np.arange(self.n_mol), ORB_PER_MOL)
        q = np.tile(np.array([0, 0, 0, 0, 1, 2]), self.n_mol)
        return 3 * m + q


def box_length(n_mol: int) -> float:
    return float((n_mol / DENSITY) ** (1.0 / 3.0))


def _wrap(x: np.ndarray, L: float) -> np.ndarray:
    x = np.mod(x, L)
    x[x >= L] = 0.0
    return x


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def place_centres(n_mol: int, seed: int, max_sweeps: int = 20000) -> tuple[np.ndarray, float]:
    """Uniform random O positions relaxed to a 3.1 Angstrom minimum separation."""
    L = box_length(n_mol)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, size=(n_mol, 3))
    if n_mol == 1:
        return x, L
    target = 1.02 * MIN_SEP
    step = 0.5
    for _ in range(max_sweeps):
        x = _wrap(x, L)
        tree = cKDTree(x, boxsize=L)
        pairs = tree.query_pairs(target, output_type="ndarray")
        if len(pairs) == 0:
            break
        d = _min_image(x[pairs[:, 1]] - x[pairs[:, 0]], L)
        r = np.linalg.norm(d, axis=1)
        if r.min() >= MIN_SEP:
            break
        r_safe = np.maximum(r, 1e-9)
        push = (target - r) / r_safe          # gradient magnitude of the penalty / r
        g = d * push[:, None] * (0.5 * step)
        disp = np.zeros_like(x)
        np.add.at(disp, pairs[:, 0], -g)
        np.add.at(disp, pairs[:, 1], g)
        x = x + disp
    else:
        raise RuntimeError("overlap removal did not converge")
    return _wrap(x, L), L


def random_rotations(n: int, seed: int) -> np.ndarray:
    """Rotation matrices from uniform random unit quaternions (n, 3, 3)."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, a, b, c = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (b * b + c * c)
    R[:, 0, 1] = 2 * (a * b - c * w)
    R[:, 0, 2] = 2 * (a * c + b * w)
    R[:, 1, 0] = 2 * (a * b + c * w)
    R[:, 1, 1] = 1 - 2 * (a * a + c * c)
    R[:, 1, 2] = 2 * (b * c - a * w)
    R[:, 2, 0] = 2 * (a * c - b * w)
    R[:, 2, 1] = 2 * (b * c + a * w)
    R[:, 2, 2] = 1 - 2 * (a * a + b * b)
    return R


def molecule_atoms(centres: np.ndarray, rot: np.ndarray, L: float) -> np.ndarray:
    half = 0.5 * ANGLE_HOH
    local = np.array([[0.0, 0.0, 0.0],
                      [R_OH * np.sin(half), 0.0, R_OH * np.cos(half)],
                      [-R_OH * np.sin(half), 0.0, R_OH * np.cos(half)]])
    atoms = centres[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    return _wrap(atoms.reshape(-1, 3), L)


def hamiltonian(atoms: np.ndarray, L: float, hop_a: float = HOP_A,
                hop_lam: float = HOP_LAM) -> sp.csr_matrix:
    """Tight-binding H (FP64 CSR, symmetric) for the atoms of whole molecules."""
    n_atoms = atoms.shape[0]
    n_mol = n_atoms // 3
    N = n_mol * ORB_PER_MOL
    rows, cols, vals = [], [], []
    # onsite
    idx = np.arange(N)
    rows.append(idx); cols.append(idx); vals.append(np.tile(ONSITE, n_mol))
    # intramolecular O orbital <-> H orbital
    base = ORB_PER_MOL * np.arange(n_mol)
    o = (base[:, None] + np.arange(4)[None, :])            # (M, 4)
    for hq in (4, 5):
        h = np.repeat((base + hq)[:, None], 4, axis=1)
        rows += [o.ravel(), h.ravel()]
        cols += [h.ravel(), o.ravel()]
        vals += [np.full(o.size, T_INTRA)] * 2
    # intermolecular, any orbital pair of two atoms closer than the cutoff
    tree = cKDTree(atoms, boxsize=L)
    pairs = tree.query_pairs(HOP_RCUT, output_type="ndarray")
    if len(pairs):
        pairs = pairs[(pairs[:, 0] // 3) != (pairs[:, 1] // 3)]
    if len(pairs):
        d = _min_image(atoms[pairs[:, 1]] - atoms[pairs[:, 0]], L)
        r = np.linalg.norm(d, axis=1)
        keep = r < HOP_RCUT
        pairs, r = pairs[keep], r[keep]
        t = -hop_a * np.exp(-(r - HOP_R0) / hop_lam)
        for ka in range(3):
            for kb in range(3):
                sel = ((pairs[:, 0] % 3) == ka) & ((pairs[:, 1] % 3) == kb)
                if not sel.any():
                    continue
                pa, pb, tv = pairs[sel, 0], pairs[sel, 1], t[sel]
                oa = ORB_PER_MOL * (pa // 3)[:, None] + _ATOM_ORBS[ka][None, :]
                ob = ORB_PER_MOL * (pb // 3)[:, None] + _ATOM_ORBS[kb][None, :]
                ra = np.repeat(oa, ob.shape[1], axis=1).ravel()
                cb = np.tile(ob, (1, oa.shape[1])).ravel()
                v = np.repeat(tv, oa.shape[1] * ob.shape[1])
                rows += [ra, cb]
                cols += [cb, ra]
                vals += [v, v]
    r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
    H = sp.coo_matrix((v, (r, c)), shape=(N, N)).tocsr()
    H.sum_duplicates()
    H.sort_indices()
    return H


def make_water(n_mol: int, seed: int = 0, hop_a: float = HOP_A,
               hop_lam: float = HOP_LAM) -> WaterSystem:
    centres, L = place_centres(n_mol, seed)
    rot = random_rotations(n_mol, seed + 1000)
    atoms = molecule_atoms(centres, rot, L)
    H = hamiltonian(atoms, L, hop_a, hop_lam)
    return WaterSystem(n_mol=n_mol, box=L, atoms=atoms, H=H,
                       n_occ=OCC_PER_MOL * n_mol, seed=seed, hop_a=hop_a, hop_lam=hop_lam)


def perturb(system: WaterSystem, sigma: float, seed: int) -> WaterSystem:
    """Gaussian displacement of every atom coordinate, H rebuilt.

    The intramolecular hopping does not depend on distance and stays -4 eV;
    intermolecular terms are recomputed from the displaced atoms."""
    rng = np.random.default_rng(seed)
    atoms = _wrap(system.atoms + rng.normal(scale=sigma, size=system.atoms.shape), system.box)
    H = hamiltonian(atoms, system.box, system.hop_a, system.hop_lam)
    return WaterSystem(n_mol=system.n_mol, box=system.box, atoms=atoms, H=H,
                       n_occ=system.n_occ, seed=system.seed, hop_a=system.hop_a,
                       hop_lam=system.hop_lam, meta={"perturbed": sigma, "perturb_seed": seed})


def hopping_derivatives(system: WaterSystem) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """dH/dA and dH/dlam of the intermolecular hopping -A exp(-(r - r0)/lam),
    as CSR matrices on the intermolecular entries of H (input generator
    derivatives, for chain-rule checks of gradients with respect to H)."""
    atoms, L = system.atoms, system.box
    N = system.n
    tree = cKDTree(atoms, boxsize=L)
    pairs = tree.query_pairs(HOP_RCUT, output_type="ndarray")
    if len(pairs):
        pairs = pairs[(pairs[:, 0] // 3) != (pairs[:, 1] // 3)]
    rows, cols, dA, dl = [], [], [], []
    if len(pairs):
        d = _min_image(atoms[pairs[:, 1]] - atoms[pairs[:, 0]], L)
        r = np.linalg.norm(d, axis=1)
        keep = r < HOP_RCUT
        pairs, r = pairs[keep], r[keep]
        ex = np.exp(-(r - HOP_R0) / system.hop_lam)
        ga = -ex
        gl = -system.hop_a * ex * (r - HOP_R0) / system.hop_lam ** 2
        for ka in range(3):
            for kb in range(3):
                sel = ((pairs[:, 0] % 3) == ka) & ((pairs[:, 1] % 3) == kb)
                if not sel.any():
                    continue
                pa, pb = pairs[sel, 0], pairs[sel, 1]
                oa = ORB_PER_MOL * (pa // 3)[:, None] + _ATOM_ORBS[ka][None, :]
                ob = ORB_PER_MOL * (pb // 3)[:, None] + _ATOM_ORBS[kb][None, :]
                ra = np.repeat(oa, ob.shape[1], axis=1).ravel()
                cb = np.tile(ob, (1, oa.shape[1])).ravel()
                m = oa.shape[1] * ob.shape[1]
                va, vl = np.repeat(ga[sel], m), np.repeat(gl[sel], m)
                rows += [ra, cb]; cols += [cb, ra]; dA += [va, va]; dl += [vl, vl]
    if not rows:
        z = sp.csr_matrix((N, N))
        return z, z
    r_, c_ = np.concatenate(rows), np.concatenate(cols)
    DA = sp.coo_matrix((np.concatenate(dA), (r_, c_)), shape=(N, N)).tocsr()
    DL = sp.coo_matrix((np.concatenate(dl), (r_, c_)), shape=(N, N)).tocsr()
    DA.sum_duplicates(); DL.sum_duplicates()
    return DA, DL

"""Spectral references (oracle, test infrastructure only).

The density matrix is the sum of outer products of the occupied eigenstates
of H (Introduction); SP2 reaches it as the limit of eq. (3).  These helpers
compute that target, and the gap between the highest occupied and lowest
unoccupied eigenvalue that makes it unique, by LAPACK diagonalisation.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _dense(H):
    return H.toarray() if sp.issparse(H) else np.asarray(H, dtype=np.float64)


def eig_projector(H, n_occ: int) -> np.ndarray:
    """P* = sum over the n_occ lowest eigenvectors v of v v^T."""
    w, V = np.linalg.eigh(_dense(H))
    Vo = V[:, :int(n_occ)]
    return Vo @ Vo.T


def spectral_gap(H, n_occ: int) -> float:
    """eps_{n_occ + 1} - eps_{n_occ}: lowest unoccupied minus highest occupied
    eigenvalue (eigenvalues ascending, counted from 1)."""
    w = np.linalg.eigvalsh(_dense(H))
    return float(w[int(n_occ)] - w[int(n_occ) - 1])

"""Spectral references (oracle, test infrastructure only).

The density matrix is the sum of outer products of the occupied eigenstates
of H (Introduction); SP2 reaches it as the limit of eq. (3).  These helpers
compute that target by LAPACK diagonalisation, and the scalar recursion of
eq. (2) on eigenvalues, which every iterate must reproduce in H's eigenbasis
(each iterate is a polynomial in H).
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
    w = np.linalg.eigvalsh(_dense(H))
    return float(w[int(n_occ)] - w[int(n_occ) - 1])


def iterate_on_eigenvalues(x0: np.ndarray, alphas) -> np.ndarray:
    """Apply x <- x + a (x - x^2) for each branch a to scalar eigenvalues."""
    x = np.array(x0, dtype=np.float64, copy=True)
    for a in alphas:
        x = x + a * (x - x * x)
    return x

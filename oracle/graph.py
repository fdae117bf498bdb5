"""Graph side of G-SP2 (oracle, test infrastructure only).

Methods, "Graph Theory": the thresholded graph G_tau, core and halo
vertices of a part, and the core-halo cost of eq. (4).

Readings: the graph is undirected, so an edge (u, v), u != v, exists when
|P_uv| > tau or |P_vu| > tau (a computed P need not be bitwise symmetric);
the halo is one hop deep; a part's local order is its core vertices
ascending, then its halo vertices ascending.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def threshold_graph(P_prev, tau: float) -> sp.csr_matrix:
    """Boolean symmetric adjacency (no self loops): edge iff |P_uv| > tau
    (strict), for either orientation of the pair."""
    P = sp.coo_matrix(P_prev)
    keep = (np.abs(P.data.astype(np.float64)) > tau) & (P.row != P.col)
    r, c = P.row[keep], P.col[keep]
    n = P.shape[0]
    A = sp.coo_matrix((np.ones(len(r), dtype=np.int8), (r, c)), shape=(n, n)).tocsr()
    A = ((A + A.T) > 0).astype(np.int8).tocsr()
    A.sort_indices()
    return A


def core_halo(adj: sp.csr_matrix, part: np.ndarray, n_parts: int) -> tuple[list, list]:
    """Core vertices of part k are those with part id k; its halo is every
    vertex outside the part adjacent to one of its core vertices."""
    part = np.asarray(part)
    cores, halos = [], []
    for k in range(n_parts):
        core = np.flatnonzero(part == k)
        if core.size == 0:
            raise ValueError(f"part {k} is empty")
        nbr = np.unique(adj[core].indices) if core.size else np.empty(0, dtype=np.int64)
        halo = np.setdiff1d(nbr, core, assume_unique=True)
        cores.append(core.astype(np.int64))
        halos.append(np.sort(halo).astype(np.int64))
    return cores, halos


def subproblem_index(core: np.ndarray, halo: np.ndarray) -> np.ndarray:
    """Rows/columns of H in a part's dense sub-problem: core first, then halo."""
    return np.concatenate([core, halo])


def ch_cost(sizes) -> int:
    """Eq. (4): C = sum_i (c_i + h_i)^3."""
    return int(sum(int(s) ** 3 for s in sizes))

"""G-SP2 end to end in FP64 (oracle, test infrastructure only).

Follows the pipeline of the paper's Fig. 1 description and the Methods
sections: threshold a previous P into G_tau, take the given partition,
build each part's core+halo index set, extract the dense sub-block of H,
start every block from eq. (1) with the *global* Gershgorin bounds, run the
SP2 recursion on all blocks with one branch sequence chosen from the summed
core trace, and reassemble P from each part's core columns.

Every vertex is core in exactly one part, so P has exactly one source for
each of its columns; entries outside part k's rows in a core column of part
k are zero (not stored).  The assembled P need not be symmetric.  With
``symmetrize`` every stored entry whose mirror is stored too becomes the mean
of the two; an entry whose mirror is not stored is kept as it is (reading of
"collected and reassembled" in the Fig. 1 description: the result keeps the
pattern the parts define).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .graph import core_halo, subproblem_index, threshold_graph
from .sp2 import SP2Result, gershgorin_bounds, initial_guess, sp2_blocks


@dataclass
class GSP2Result:
    cores: list
    halos: list
    index: list              # per part: core + halo global indices (local order)
    core_columns: list       # per part: (s_k, c_k) FP64 block = X_k[:, :c_k]
    sp2: SP2Result
    eps: tuple
    n: int

    @property
    def sizes(self):
        return [len(i) for i in self.index]

    def dense(self, symmetrize: bool = False) -> np.ndarray:
        if symmetrize:
            return self.csc(symmetrize=True).toarray()
        P = np.zeros((self.n, self.n))
        for idx, core, blk in zip(self.index, self.cores, self.core_columns):
            P[np.ix_(idx, core)] = blk
        return P

    def csc(self, symmetrize: bool = False) -> sp.csc_matrix:
        """P with each core column's rows sorted by global index."""
        rows, cols, vals = [], [], []
        for idx, core, blk in zip(self.index, self.cores, self.core_columns):
            for jl, j in enumerate(core):
                rows.append(idx); cols.append(np.full(len(idx), j)); vals.append(blk[:, jl])
        r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
        if symmetrize:
            # position of every stored entry's mirror, or -1 when it is not stored
            key = r.astype(np.int64) * self.n + c
            mirror = c.astype(np.int64) * self.n + r
            order = np.argsort(key)
            pos = np.searchsorted(key[order], mirror)
            pos = np.minimum(pos, len(key) - 1)
            found = key[order][pos] == mirror
            w = np.where(found, v[order][pos], v)
            v = np.where(found, 0.5 * (v + w), v)
        P = sp.coo_matrix((v, (r, c)), shape=(self.n, self.n)).tocsc()
        P.sort_indices()
        return P


def gsp2(H, P_prev, tau: float, part, n_parts: int, n_occ: float, max_iter: int = 60,
         alpha_seq=None, stop_rule: bool = True, trace_tol: float = 0.5,
         parts_subset=None, adjacency=None) -> GSP2Result:
    """G-SP2 P from H (sparse or dense FP64), a previous P (for the graph),
    the threshold tau and a partition (part id per vertex).

    ``parts_subset`` restricts the run to some parts; that is only
    meaningful with ``alpha_seq`` (a replayed branch sequence), because the
    trace rule sums over every part."""
    H = sp.csr_matrix(H)
    n = H.shape[0]
    emin, emax = gershgorin_bounds(H)
    adj = threshold_graph(P_prev, tau) if adjacency is None else adjacency
    cores, halos = core_halo(adj, part, n_parts)
    ks = range(n_parts) if parts_subset is None else list(parts_subset)
    if parts_subset is not None and alpha_seq is None:
        raise ValueError("a subset of parts needs a replayed branch sequence")
    index = [subproblem_index(cores[k], halos[k]) for k in ks]
    X0 = [initial_guess(H[idx][:, idx].toarray(), emin, emax) for idx in index]
    csz = [len(cores[k]) for k in ks]
    res = sp2_blocks(X0, csz, n_occ, max_iter=max_iter, alpha_seq=alpha_seq,
                     stop_rule=stop_rule, trace_tol=trace_tol)
    core_cols = [X[:, :c] for X, c in zip(res.blocks, csz)]
    return GSP2Result([cores[k] for k in ks], [halos[k] for k in ks], index, core_cols,
                      res, (emin, emax), n)

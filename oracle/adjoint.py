"""Adjoint of G-SP2 in FP64 (oracle, test infrastructure only).

Differentiates the map H -> P that the G-SP2 oracle computes for a fixed
branch sequence (the sequence of a forward run, replayed), following the
forward steps in reverse:

* P[idx_k, j] = X_k,n[:, j] for core columns j: the seed of part k is
  dL/dP on those columns, zero elsewhere, symmetrised, since every iterate is
  symmetric and only symmetric perturbations of H are considered.
* Eq. (2), X' = X^2 (alpha = -1) or 2X - X^2 (alpha = +1): for a symmetric
  cotangent G of X', the cotangent of X is GX + XG, or 2G - (GX + XG).
* Eq. (1), X0 = (eps_max I - H_sub) / (eps_max - eps_min): the cotangent of
  H_sub is -G0 / D (D = eps_max - eps_min), and
  dL/d eps_max = sum_k <G0_k, I - X0_k> / D, dL/d eps_min = sum_k <G0_k, X0_k> / D.
* Gershgorin bounds: eps_max = H_ii + sum_{j != i} |H_ij| at its maximising
  row i (the lowest such index), eps_min = H_jj - sum |H_jl| at its
  minimising row j; their derivatives fall on those rows.

The result is the gradient with respect to H under symmetric perturbations,
split evenly between H_uv and H_vu, returned as a dense symmetric matrix
(entries outside H's pattern are zero).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .graph import core_halo, subproblem_index, threshold_graph
from .sp2 import gershgorin_bounds, initial_guess


@dataclass
class GSP2Grad:
    dH: np.ndarray            # dense N x N, symmetric
    d_eps: tuple              # (dL/d eps_min, dL/d eps_max)
    rows: tuple               # (argmin row of eps_min, argmax row of eps_max)
    P: np.ndarray             # the forward P (dense)


def gershgorin_rows(H) -> tuple[int, int]:
    """Rows attaining eps_min and eps_max (lowest index on ties)."""
    H = sp.csr_matrix(H)
    d = H.diagonal()
    r = np.asarray(abs(H).sum(axis=1)).ravel() - np.abs(d)
    return int(np.argmin(d - r)), int(np.argmax(d + r))


def gsp2_grad(H, P_prev, tau: float, part, n_parts: int, alpha_seq, dLdP: np.ndarray,
              adjacency=None) -> GSP2Grad:
    """dL/dH for L depending on P through dLdP (dense N x N; only the stored
    entries of P, the core columns over each part's rows, are read)."""
    H = sp.csr_matrix(H)
    n = H.shape[0]
    emin, emax = gershgorin_bounds(H)
    D = emax - emin
    adj = threshold_graph(P_prev, tau) if adjacency is None else adjacency
    cores, halos = core_halo(adj, part, n_parts)
    dH = np.zeros((n, n))
    P = np.zeros((n, n))
    g_emax = 0.0
    g_emin = 0.0
    for k in range(n_parts):
        idx = subproblem_index(cores[k], halos[k])
        c = len(cores[k])
        X0 = initial_guess(H[idx][:, idx].toarray(), emin, emax)
        # forward, keeping every iterate
        Xs = [X0]
        for a in alpha_seq:
            X = Xs[-1]
            Xs.append(X + a * (X - X @ X))
        P[np.ix_(idx, cores[k])] = Xs[-1][:, :c]
        # seed: dL/dP on the part's core columns, symmetrised
        G = np.zeros_like(X0)
        G[:, :c] = dLdP[np.ix_(idx, cores[k])]
        G = 0.5 * (G + G.T)
        # reverse sweep through eq. (2)
        for t in range(len(alpha_seq) - 1, -1, -1):
            X = Xs[t]
            S = G @ X + X @ G
            G = S if alpha_seq[t] < 0 else 2.0 * G - S
        # eq. (1)
        dH[np.ix_(idx, idx)] += -G / D
        g_emax += float(np.sum(G * (np.eye(len(idx)) - X0))) / D
        g_emin += float(np.sum(G * X0)) / D
    # Gershgorin rows; symmetric perturbations, split evenly over H_uv and H_vu
    jmin, imax = gershgorin_rows(H)
    Hc = H.tocsr()
    for row, g, sgn in ((imax, g_emax, 1.0), (jmin, g_emin, -1.0)):
        cols = Hc.indices[Hc.indptr[row]:Hc.indptr[row + 1]]
        vals = Hc.data[Hc.indptr[row]:Hc.indptr[row + 1]]
        for cidx, v in zip(cols, vals):
            if cidx == row:
                dH[row, row] += g
            else:
                w = g * sgn * np.sign(v)
                dH[row, cidx] += 0.5 * w
                dH[cidx, row] += 0.5 * w
    # only H's stored entries carry a gradient
    pat = sp.csr_matrix((np.ones(Hc.nnz), Hc.indices, Hc.indptr), shape=Hc.shape).toarray() != 0
    dH = np.where(pat, dH, 0.0)
    return GSP2Grad(dH, (g_emin, g_emax), (jmin, imax), P)

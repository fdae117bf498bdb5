"""SP2 purification in FP64 (oracle, test infrastructure only).

Follows Methods, "Second-Order Spectral Projection Method (SP2)":
eq. (1) for the initial guess, eq. (2) for the step, the trace rule for the
branch, eq. (3) for the limit and the idempotency check for convergence.

Readings of points the paper leaves open (each also listed in the design
notes):

* Branch rule.  The paper writes the test on Tr[X_i], the iterate being
  produced; the test is applied to the current iterate instead:
  alpha = +1 (X <- 2X - X^2, raises the trace) iff Tr[X] <= N_occ, else
  alpha = -1 (X <- X^2).  N_occ = N_el / 2 (the paper's 2 Tr[X] <= N_el).
  A tie goes to +1.
* Trace in G-SP2.  "Tr" is the sum over all parts of the diagonal entries
  of each part's *core* rows (every vertex is core in exactly one part).
  Dense SP2 is the single-part case, where it is the ordinary trace.
* Stopping.  e_t = Tr[X_t] - Tr[X_t^2] measures idempotency of the iterate
  that is being squared; the error bound applies to its magnitude, since in
  finite precision e_t turns negative once X_t is idempotent to rounding.
  Stop at the first product t >= 2 with |e_t| >= |e_{t-2}| and
  |e_{t-2}| < max(1, n u) (the error has stopped falling, and has reached
  the level the arithmetic can resolve: n = sum of core sizes, u = unit
  roundoff of the product operands, 2^-53 here, so the floor is 1), and
  return X_t (the square just formed is discarded).  At most ``max_iter``
  products; if the rule never fires the result is the last iterate and the
  run is "not converged".
* Replay.  With a stored branch sequence, exactly that many products are
  applied, no stop rule, and the result is rejected when its trace misses
  N_occ by more than ``trace_tol`` (the paper's check on a stored
  sequence).
* Occupation.  The same check applies when the stop rule fires: a result
  whose trace misses N_occ by more than ``trace_tol`` is a failed run
  (status "wrong_trace"), since the SP2 section ties a correct run to a
  final trace equal to the electron count.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


class NotConverged(RuntimeError):
    pass


class WrongTrace(RuntimeError):
    pass


def gershgorin_bounds(H) -> tuple[float, float]:
    """Spectral bounds from the Gershgorin circle theorem (Methods, SP2 section,
    after eq. (1)): every eigenvalue lies in some disc centred at H_ii with
    radius sum_{j != i} |H_ij|, so eps_min = min_i(H_ii - r_i) and
    eps_max = max_i(H_ii + r_i)."""
    if sp.issparse(H):
        H = sp.csr_matrix(H)
        diag = H.diagonal().astype(np.float64)
        absrow = np.asarray(abs(H).sum(axis=1)).ravel()
    else:
        H = np.asarray(H, dtype=np.float64)
        diag = np.diag(H).copy()
        absrow = np.abs(H).sum(axis=1)
    radius = absrow - np.abs(diag)
    return float(np.min(diag - radius)), float(np.max(diag + radius))


def initial_guess(Hsub: np.ndarray, eps_min: float, eps_max: float) -> np.ndarray:
    """Eq. (1): X0 = (eps_max I - H) / (eps_max - eps_min)."""
    Hsub = np.asarray(Hsub, dtype=np.float64)
    n = Hsub.shape[0]
    return (eps_max * np.eye(n) - Hsub) / (eps_max - eps_min)


def _core_trace(blocks: list[np.ndarray], cores: list[int]) -> float:
    return float(sum(np.trace(b[:c, :c]) for b, c in zip(blocks, cores)))


@dataclass
class SP2Result:
    blocks: list            # final iterate per part
    n_products: int         # matrix products formed (including a discarded last one)
    alphas: list            # branch actually applied after each kept product
    traces: list            # Tr[X_t] for t = 0 .. len(alphas)
    errors: list            # e_t = Tr[X_t] - Tr[X_t^2] for each product t
    converged: bool
    status: str = "ok"
    meta: dict = field(default_factory=dict)


def drop_small(X: np.ndarray, eps: float) -> np.ndarray:
    """Numerical thresholding of sparse-matrix SP2 (the standard scheme that
    gives the initial P, Fig. 1 description; the threshold is the same kind of
    parameter as the graph's tau, Methods, "Graph Theory"): an entry is kept
    iff |x| > eps, the strict comparison of the graph's threshold."""
    return np.where(np.abs(X) > eps, X, 0.0)


def sp2_blocks(X0: list, cores: list, n_occ: float, max_iter: int = 60,
               alpha_seq=None, stop_rule: bool = True, trace_tol: float = 0.5,
               raise_on_failure: bool = False, unit_roundoff: float = 2.0 ** -53,
               eps: float | None = None) -> SP2Result:
    """Run the SP2 recursion eq. (2) on every block at once, all blocks sharing
    one branch sequence chosen from the summed core trace.

    X0: list of square FP64 arrays, part k's core rows first (its first
    cores[k] rows/columns).  eps: if given, every iterate (X0 included) is
    thresholded with drop_small; the products themselves are formed in full."""
    X = [np.array(x, dtype=np.float64, copy=True) for x in X0]
    if eps is not None:
        X = [drop_small(x, eps) for x in X]
    tr = _core_trace(X, cores)
    traces, errors, alphas = [tr], [], []
    replay = alpha_seq is not None
    n_steps = len(alpha_seq) if replay else max_iter
    floor = max(1.0, sum(cores) * unit_roundoff)
    for t in range(n_steps):
        Y = [x @ x for x in X]                 # the product of eq. (2)
        trY = _core_trace(Y, cores)
        errors.append(tr - trY)
        if (not replay and stop_rule and t >= 2 and abs(errors[t]) >= abs(errors[t - 2])
                and abs(errors[t - 2]) < floor):
            if abs(tr - n_occ) <= trace_tol:
                return SP2Result(X, t + 1, alphas, traces, errors, True)
            if raise_on_failure:
                raise WrongTrace(f"trace {tr} vs N_occ {n_occ}")
            return SP2Result(X, t + 1, alphas, traces, errors, False, "wrong_trace")
        if replay:
            alpha = int(alpha_seq[t])
        else:
            alpha = 1 if tr <= n_occ else -1
        # eq. (2): X_i = [I + alpha (I - X)] X = X + alpha (X - X^2)
        X = [x + alpha * (x - y) for x, y in zip(X, Y)]
        if eps is not None:
            X = [drop_small(x, eps) for x in X]
        alphas.append(alpha)
        tr = _core_trace(X, cores)
        traces.append(tr)
    if replay:
        ok = abs(tr - n_occ) <= trace_tol
        res = SP2Result(X, n_steps, alphas, traces, errors, ok, "ok" if ok else "wrong_trace")
        if not ok and raise_on_failure:
            raise WrongTrace(f"trace {tr} vs N_occ {n_occ}")
        return res
    res = SP2Result(X, n_steps, alphas, traces, errors, False, "not_converged")
    if raise_on_failure:
        raise NotConverged(f"no stop after {n_steps} products")
    return res


def dense_sp2(H, n_occ: float, max_iter: int = 60, **kw) -> tuple[np.ndarray, SP2Result]:
    """Plain SP2 on the whole matrix: Gershgorin bounds, eq. (1), eq. (2)."""
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H, dtype=np.float64)
    emin, emax = gershgorin_bounds(Hd)
    X0 = initial_guess(Hd, emin, emax)
    res = sp2_blocks([X0], [Hd.shape[0]], n_occ, max_iter=max_iter, **kw)
    return res.blocks[0], res


def thresholded_sp2(H, n_occ: float, eps: float, max_iter: int = 60, **kw) -> tuple[np.ndarray, SP2Result]:
    """SP2 of the whole matrix in numerically thresholded algebra, the scheme
    that computes the initial density matrix before any graph exists (Fig. 1
    description): dense SP2 (Gershgorin bounds, eq. (1), eq. (2), the trace
    rule and the stop rule) with every iterate thresholded by drop_small;
    each product is formed from the thresholded iterate, and the stop
    measure e_t from that full product."""
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H, dtype=np.float64)
    emin, emax = gershgorin_bounds(Hd)
    X0 = initial_guess(Hd, emin, emax)
    res = sp2_blocks([X0], [Hd.shape[0]], n_occ, max_iter=max_iter, eps=eps, **kw)
    return res.blocks[0], res

"""Planted mistakes in a copy of the oracle must each break a pin.

Each mutant edits one line of the oracle's source in a temporary copy; the
pin battery then runs in a child process that imports the copy in place of
the real oracle.  The unmodified copy is the control and must pass."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "x0_orientation": ("sp2.py", "(eps_max * np.eye(n) - Hsub)", "(Hsub - eps_min * np.eye(n))"),
    "branch_swapped": ("sp2.py", "alpha = 1 if tr <= n_occ else -1", "alpha = -1 if tr <= n_occ else 1"),
    "step_sign": ("sp2.py", "x + alpha * (x - y)", "x - alpha * (x - y)"),
    "step_elementwise": ("sp2.py", "Y = [x @ x for x in X]", "Y = [x * x for x in X]"),
    "radius_keeps_diag": ("sp2.py", "radius = absrow - np.abs(diag)", "radius = absrow"),
    "radius_no_abs": ("sp2.py", "absrow = np.abs(H).sum(axis=1)", "absrow = H.sum(axis=1)"),
    "trace_all_rows": ("sp2.py", "np.trace(b[:c, :c])", "np.trace(b)"),
    "stop_no_safeguard": ("sp2.py", "and abs(errors[t - 2]) < floor", "and abs(errors[t - 2]) < 1e300"),
    "stop_inverted": ("sp2.py", "abs(errors[t]) >= abs(errors[t - 2])", "abs(errors[t]) <= abs(errors[t - 2])"),
    "threshold_not_strict": ("graph.py", "> tau)", ">= tau)"),
    "graph_not_symmetrised": ("graph.py", "A = ((A + A.T) > 0)", "A = ((A + 0 * A.T) > 0)"),
    "halo_keeps_core": ("graph.py", "halo = np.setdiff1d(nbr, core, assume_unique=True)", "halo = nbr"),
    "index_halo_first": ("graph.py", "np.concatenate([core, halo])", "np.concatenate([halo, core])"),
    "assemble_rows": ("gsp2.py", "P[np.ix_(idx, core)] = blk", "P[np.ix_(core, idx)] = blk.T"),
    "bounds_local": ("gsp2.py", "X0 = [initial_guess(H[idx][:, idx].toarray(), emin, emax) for idx in index]",
                     "X0 = [initial_guess(H[idx][:, idx].toarray(), *gershgorin_bounds(H[idx][:, idx])) for idx in index]"),
    "adjoint_step_sign": ("adjoint.py", "G = S if alpha_seq[t] < 0 else 2.0 * G - S", "G = S if alpha_seq[t] > 0 else 2.0 * G - S"),
    "adjoint_one_sided": ("adjoint.py", "S = G @ X + X @ G", "S = 2.0 * (G @ X)"),
    "adjoint_no_symmetrise": ("adjoint.py", "G = 0.5 * (G + G.T)", "G = G"),
    "adjoint_x0_sign": ("adjoint.py", "dH[np.ix_(idx, idx)] += -G / D", "dH[np.ix_(idx, idx)] += G / D"),
    "symmetrize_mirror_ignored": ("gsp2.py", "v = np.where(found, 0.5 * (v + w), v)", "v = np.where(found, 0.5 * (v + v), v)"),
    "gap_off_by_one": ("spectral.py", "return float(w[int(n_occ)] - w[int(n_occ) - 1])",
                       "return float(w[int(n_occ) + 1] - w[int(n_occ)])"),
    "occupation_unchecked": ("sp2.py", "            if abs(tr - n_occ) <= trace_tol:", "            if True:"),
    "drop_signed": ("sp2.py", "np.where(np.abs(X) > eps, X, 0.0)", "np.where(X > eps, X, 0.0)"),
    "drop_x0_only": ("sp2.py", "            X = [drop_small(x, eps) for x in X]\n        alphas.append",
                     "            X = [x for x in X]\n        alphas.append"),
    "adjoint_no_bound_terms": ("adjoint.py", "                dH[row, row] += g", "                dH[row, row] += 0.0"),
}


def _run_battery(tmp_path, mutant):
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst)
    if mutant is not None:
        fname, old, new = MUTANTS[mutant]
        path = dst / fname
        src = path.read_text()
        assert src.count(old) == 1, f"mutation site not unique in {fname}: {old}"
        path.write_text(src.replace(old, new))
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(1, %r);"
            "import oracle; assert oracle.__file__.startswith(%r);"
            "from tests import _pins; _pins.battery()") % (str(tmp_path), ROOT, str(tmp_path))
    env = dict(os.environ, OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


def test_control_copy_passes(tmp_path):
    r = _run_battery(tmp_path, None)
    assert r.returncode == 0, r.stderr[-2000:]


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, mutant):
    r = _run_battery(tmp_path, mutant)
    assert r.returncode != 0, f"planted mistake {mutant} passed every pin"

"""FP64 CPU oracle for graph-partitioned SP2 (G-SP2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The GPU library
and its Python binding never import, call or link anything here, and this
package never imports the GPU library.  Each function follows the passage of
arXiv:1801.10016 named in its docstring, written as the plain definition
(or the algorithm's steps in the paper's order), in float64 numpy, with no
blocking, fusion or reordering of its own.
"""
from .sp2 import (gershgorin_bounds, initial_guess, sp2_blocks, dense_sp2, thresholded_sp2, drop_small,
                  SP2Result, NotConverged, WrongTrace)
from .graph import threshold_graph, core_halo, ch_cost, subproblem_index
from .gsp2 import gsp2, GSP2Result
from .spectral import eig_projector, spectral_gap
from .adjoint import gsp2_grad, gershgorin_rows, GSP2Grad

__all__ = [
    "gershgorin_bounds", "initial_guess", "sp2_blocks", "dense_sp2", "thresholded_sp2", "drop_small", "SP2Result",
    "NotConverged", "WrongTrace", "threshold_graph", "core_halo", "ch_cost",
    "subproblem_index", "gsp2", "GSP2Result", "eig_projector", "spectral_gap",
    "gsp2_grad", "gershgorin_rows", "GSP2Grad",
]

"""Seeded Gaussian probe matrices for comparing large results through sketches.

This module only draws random numbers; it holds none of the density-matrix
arithmetic.  Both sides of a comparison (the FP64 oracle's stored
expectations and a test reading the GPU result) draw the same probes from the
same seeds and form the same plain product S B R of their own block B.

For a block B (rows x cols) and Gaussian S (m x rows), R (cols x r), the
sketch S B R is linear in B, so the sketch of a difference is the difference
of the sketches, and ||S D R||_F / sqrt(m r) estimates ||D||_F to within a
few tens of percent for m r >= 64.  Any change of B that is not tiny against
its norm (a permuted, transposed or sign-flipped sub-block, a dropped term)
moves the sketch by about its own size.
"""
from __future__ import annotations

import numpy as np

SKETCH_M = 16          # left probe rows
SKETCH_R = 8           # right probe columns
SKETCH_SEED = 1801_10016


def probes(key: int, n_rows: int, n_cols: int, m: int = SKETCH_M, r: int = SKETCH_R,
           seed: int = SKETCH_SEED) -> tuple[np.ndarray, np.ndarray]:
    """Gaussian S (m x n_rows) and R (n_cols x r) for the block named `key`
    (a part number, or -1 for a whole matrix)."""
    rng = np.random.default_rng([seed, key + 1])
    S = rng.standard_normal((m, n_rows))
    R = rng.standard_normal((n_cols, r))
    return S, R

"""Dense brute-force checker for the pressure operator (test infrastructure).

Assembles the matrix of the oracle's matrix-free operator column by column
(tiny meshes only) and solves it with a dense Cholesky factorisation from
numpy/scipy, so that the iterative solve can be compared with a direct one.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def assemble(oracle, c, D) -> np.ndarray:
    n = oracle.nc
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = oracle.apply_A(c, D, e)
    return A


def direct_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    cf = sla.cho_factor(A, lower=True)
    return sla.cho_solve(cf, b)

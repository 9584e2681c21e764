"""Linear solves for the oracle: SciPy sparse direct (SuperLU) or dense LU.

The discrete solution, not an iteration history, is what the oracle
provides; a zero right-hand side gives x = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def direct(A, b):
    if not np.any(b):
        return np.zeros_like(b)
    return spla.spsolve(A.tocsc(), b)


def dense(A, b):
    return np.linalg.solve(A.toarray(), b)


def rel_residual(A, x, b):
    nb = np.linalg.norm(b)
    r = b - A @ x
    return np.linalg.norm(r) / nb if nb > 0 else np.linalg.norm(r)

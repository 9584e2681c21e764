"""Linear solves for the oracle.

The oracle's operators are sums of link fluxes: (A x)_i = m_i x_i +
sum_j w_ij (x_i - x_j), with m_i the mass / interface / wall terms and w_ij
the symmetric link couplings (FluxOp).  A CSR matrix of the same operator is
factorised by SciPy SuperLU; the factorised solution is then refined with
residuals evaluated in the flux form in extended precision (numpy longdouble),
the textbook iterative refinement.  This removes the rounding of the CSR
diagonal (a sum of couplings), which at density ratios of 1e3 moves the
solution by ~1e-11.  The discrete solution, not an iteration history, is what
the oracle provides; a zero right-hand side gives x = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class FluxOp:
    """(A x)_i = mexc_i x_i + sum_j w_ij (x_i - x_j); rows/cols/w list every
    coupling in both directions.

    ``plus`` (optional) holds the same couplings per axis on the grid: plus[a][c]
    is the weight of the link from cell c to its +a neighbour (wrapping on a
    periodic axis), 0 where there is no link.  ``shape`` is (n, periodic) of
    the grid.  The structured multigrid solve reads this form."""

    def __init__(self, mexc, rows, cols, w, plus=None, shape=None):
        self.mexc = np.asarray(mexc, dtype=float)
        self.rows = np.asarray(rows)
        self.cols = np.asarray(cols)
        self.w = np.asarray(w, dtype=float)
        self.plus = plus
        self.shape = shape

    def matvec(self, x, dtype=np.float64):
        x = np.asarray(x, dtype=dtype)
        y = self.mexc.astype(dtype) * x
        np.add.at(y, self.rows, self.w.astype(dtype) * (x[self.rows] - x[self.cols]))
        return y

    def to_csr(self):
        N = self.mexc.size
        diag = self.mexc.copy()
        np.add.at(diag, self.rows, self.w)
        A = sp.csr_matrix((np.concatenate([-self.w, diag]),
                           (np.concatenate([self.rows, np.arange(N)]),
                            np.concatenate([self.cols, np.arange(N)]))), shape=(N, N))
        return A


def direct(A, b, op: FluxOp = None, refine: int = 3):
    if not np.any(b):
        return np.zeros_like(b)
    lu = spla.splu(sp.csc_matrix(A))
    x = lu.solve(b)
    if op is None or refine <= 0:
        return x
    bl = np.asarray(b, dtype=np.longdouble)
    xl = x.astype(np.longdouble)
    for _ in range(refine):
        r = bl - op.matvec(xl, np.longdouble)
        xl = xl + lu.solve(r.astype(np.float64)).astype(np.longdouble)
    return xl.astype(np.float64)


def dense(A, b):
    return np.linalg.solve(A.toarray(), b)


def rel_residual(A, x, b):
    nb = np.linalg.norm(b)
    r = b - A @ x
    return np.linalg.norm(r) / nb if nb > 0 else np.linalg.norm(r)

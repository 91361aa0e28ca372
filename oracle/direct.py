"""Reference solutions of the linear systems (TEST INFRASTRUCTURE ONLY).

The method's result is the solution x* of the nonsingular system A x = b
(the linearized monolithic system of Section 2.2 in the ordering of eq.
matrix_J2); any iterate within the stated residual is correct.  The oracle's
reference for x* is a sparse LU solve (SciPy ``splu``, partial pivoting)
followed by classical iterative refinement (Wilkinson): the residual of the
current iterate is formed with every product and sum in extended precision
(``numpy.longdouble``, 64-bit significand on x86), the correction solved with
the same LU factors, and the iterate updated in extended precision.  When
kappa(A) * eps64 < 1 this converges to x* rounded to FP64, independently of
how ill-conditioned individual fields are, down to a limiting error of
about kappa(A) * eps_ld (eps_ld = 5.4e-20, the residual's precision) in the
worst case.  On the channel workloads the plain LU solution carries a
relative error of ~5e-8 in the solid pressure (the nearly incompressible
solid makes that field sensitive); after refinement the corrections fall
to ~1e-17 of every field and FGMRES run to 1e-12 agrees with the refined
solution to ~1e-11 in every field (an independent route to the same x*).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def residual_ld(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """b - A x with every product and row sum in numpy.longdouble."""
    A = sp.csr_matrix(A)
    xl = np.asarray(x, dtype=np.longdouble)
    prod = A.data.astype(np.longdouble) * xl[A.indices]
    rows = np.zeros(A.shape[0], dtype=np.longdouble)
    nz = np.diff(A.indptr) > 0
    if A.nnz:
        rows[nz] = np.add.reduceat(prod, A.indptr[:-1][nz])
    return np.asarray(b, dtype=np.longdouble) - rows


def direct_solve(A: sp.spmatrix, b: np.ndarray, refine: int = 10,
                 transpose: bool = False) -> np.ndarray:
    """x with A x = b (A^T x = b when transpose) by sparse LU plus up to
    `refine` steps of iterative refinement with extended-precision residuals,
    stopping once a correction is below the extended-precision rounding of
    x (each step shrinks the error by about kappa * eps64); returned rounded
    to FP64."""
    M = sp.csr_matrix(A.T if transpose else A)
    lu = spla.splu(sp.csc_matrix(M))
    x = lu.solve(np.asarray(b, dtype=np.float64)).astype(np.longdouble)
    tiny = np.finfo(np.longdouble).eps
    for _ in range(refine):
        r = residual_ld(M, x, b)
        dx = lu.solve(np.asarray(r, dtype=np.float64)).astype(np.longdouble)
        x = x + dx
        if np.abs(dx).max() <= tiny * np.abs(x).max():
            break
    return np.asarray(x, dtype=np.float64)

"""Pins of the oracle's reference solve (oracle/direct.py): sparse LU plus
iterative refinement with extended-precision residuals must return the exact
solution, rounded to FP64, of systems whose exact solution is known, also
where plain LU loses many digits."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.direct import direct_solve, residual_ld
from paper_1909_13201_amd import inputs


def test_two_by_two_near_singular():
    """[[F(n+1), F(n)], [F(n), F(n-1)]] of Fibonacci numbers has determinant
    +-1 and kappa ~ F(n+1)^2 (2.8e10 at n = 25); with an integer solution every
    entry of A, x* and b is exact in FP64."""
    F = [0, 1]
    for _ in range(30):
        F.append(F[-1] + F[-2])
    n = 25
    A = sp.csr_matrix(np.array([[F[n + 1], F[n]], [F[n], F[n - 1]]], dtype=np.float64))
    xs = np.array([7.0, -5.0])
    b = A @ xs
    x = direct_solve(A, b)
    kappa = np.linalg.cond(A.toarray())
    u_ld = np.finfo(np.longdouble).eps
    err = np.abs(x - xs).max() / np.abs(xs).max()
    # refinement's limiting accuracy: kappa times the residual's precision
    assert err <= kappa * u_ld
    # sharpness: plain LU loses far more digits, and refine=0 is plain LU
    x0 = spla.splu(sp.csc_matrix(A)).solve(b)
    assert np.abs(x0 - xs).max() / np.abs(xs).max() >= 1e3 * max(err, 1e-300)
    assert np.array_equal(direct_solve(A, b, refine=0), x0)
    bt = A.T @ xs
    assert np.abs(direct_solve(A, bt, transpose=True) - xs).max() <= kappa * u_ld * 7


def _integer_system(n, seed):
    """A = L U with unit-triangular sparse integer factors (so det A = 1 and
    A, x*, b = A x* are exact integers below 2^53)."""
    rng = np.random.default_rng(seed)
    L = np.eye(n, dtype=np.int64)
    U = np.eye(n, dtype=np.int64)
    for k in range(1, 3):
        L += np.diag(rng.integers(-1, 2, n - k), -k)
        U += np.diag(rng.integers(-1, 2, n - k), k)
    A = L @ U
    P = rng.permutation(n)
    A = A[P]                       # row permutation: LU must pivot
    xs = rng.integers(-1000, 1001, n)
    b = A @ xs
    assert np.abs(b).max() < 2 ** 53
    return A, xs, b


def test_integer_systems_solved_exactly():
    for seed in range(3):
        A, xs, b = _integer_system(60, seed)
        assert np.linalg.cond(A.astype(np.float64)) < 1e12   # refinement's premise
        As = sp.csr_matrix(A.astype(np.float64))
        x = direct_solve(As, b.astype(np.float64))
        assert np.array_equal(x, xs.astype(np.float64)), np.abs(x - xs).max()
        xt = direct_solve(sp.csr_matrix(A.T.astype(np.float64)), b.astype(np.float64),
                          transpose=True)
        assert np.array_equal(xt, xs.astype(np.float64))


def test_residual_ld_exact_on_integers():
    A, xs, b = _integer_system(30, 7)
    r = residual_ld(sp.csr_matrix(A.astype(np.float64)), xs.astype(np.float64),
                    b.astype(np.float64))
    assert np.all(r == 0)
    r1 = residual_ld(sp.csr_matrix(A.astype(np.float64)), xs.astype(np.float64) + 1.0,
                     b.astype(np.float64))
    assert np.array_equal(np.asarray(r1, np.float64), -A.sum(1).astype(np.float64))


def test_channel_operator_refined_residual():
    """On the c1 operator (kappa ~ 2e9) the refinement has converged: two more
    steps change no field by more than the FP64 rounding of the solution,
    the extended-precision residual is at that rounding level (normwise),
    and the plain LU solution is within kappa eps of it."""
    from oracle.multigrid import Hierarchy
    cfg = inputs.config("c1")
    O = Hierarchy(cfg, None, build_smoothers=False)
    A = O.A[-1]
    b = O.rhs(inputs.body_force(cfg))
    x = direct_solve(A, b)
    x4 = direct_solve(A, b, refine=4)
    lv = O.finest
    for sl in (slice(0, lv.off_ps), slice(lv.off_ps, lv.off_u), slice(lv.off_u, lv.off_pf),
               slice(lv.off_pf, lv.N)):
        assert np.linalg.norm(x4[sl] - x[sl]) <= 1e-15 * np.linalg.norm(x[sl])
    r = np.asarray(residual_ld(A, x, b), np.float64)
    assert np.linalg.norm(r) <= 4 * np.finfo(float).eps * np.linalg.norm(abs(A) @ abs(x))
    x0 = spla.splu(sp.csc_matrix(A)).solve(b)
    assert np.linalg.norm(x - x0) <= 1e-6 * np.linalg.norm(x)

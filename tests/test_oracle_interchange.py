"""Pins of the interchanged cascade (oracle): GMRES preconditioned by the
field split P_2 of eq. FS, each diagonal block by one GMG cycle on it (the
paper's future work, Section 5, with its GMG and FS boxes swapped).

* the cycle's operators are exactly the field split's diagonal blocks: no
  entry coupling [d, p^s] with [u, p^f], every other entry of A kept, and
  the removed coupling is real (the interface traction in the solid-momentum
  rows, the kinematic rows with a time step);
* the restriction keeps R_2's routing inside each group and drops only the
  fluid-momentum rows it routes into coarse solid-momentum rows;
* the preconditioner is block diagonal: a residual in one group gives a
  correction in that group only (a structural invariant any wrong operator,
  restriction or coarse solve breaks), and it is linear;
* two levels on a small mesh: the cycle equals its closed-form error
  propagation (I - B A)^nu2 (I - P A_0^{-1} R A)(I - B A)^nu1 built from the
  diagonal blocks and the explicit smoother;
* FGMRES with it converges to the same solution as the direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.direct import direct_solve
from oracle.krylov import fgmres
from oracle.multigrid import Hierarchy, diagonal_blocks, field_groups
from paper_1909_13201_amd import inputs


def _pair(name="c2", L=3, **kw):
    cfg = dict(inputs.with_levels(inputs.config(name), L), **kw)
    w = inputs.advecting_field(cfg)
    return (Hierarchy(dict(cfg, interchange=True), w),
            Hierarchy(dict(cfg, interchange=False), w, build_smoothers=False))


@pytest.fixture(scope="module")
def c2():
    return _pair("c2", 3)


def test_diagonal_blocks(c2):
    H, O = c2
    for l in range(H.L):
        g = field_groups(H.levels[l])
        C = sp.coo_matrix(H.Ac[l])
        assert np.all(g[C.row] == g[C.col])
        X = sp.coo_matrix(O.A[l] - H.Ac[l])
        X.eliminate_zeros()
        assert X.nnz > 0 and np.all(g[X.row] != g[X.col])      # only coupling removed
        lv = H.levels[l]
        assert np.all(X.row < lv.off_ps)      # steady: the solid-momentum rows' traction
    # with a time step the kinematic rows couple u to d^s as well
    Ht, _ = _pair("c5", 2)
    lv = Ht.finest
    X = sp.coo_matrix(Ht.A[-1] - Ht.Ac[-1])
    X.eliminate_zeros()
    assert np.any((X.row >= lv.off_u) & (X.row < lv.off_pf))


def test_restriction_inside_groups(c2):
    H, O = c2
    for l in range(1, H.L):
        gf, gc = field_groups(H.levels[l]), field_groups(H.levels[l - 1])
        C = sp.coo_matrix(H.Rc[l])
        assert np.all(gc[C.row] == gf[C.col])
        X = sp.coo_matrix(O.R[l] - H.Rc[l])
        X.eliminate_zeros()
        assert X.nnz > 0
        # the dropped entries send fine fluid-momentum (u) rows into coarse
        # solid-momentum (d) rows
        fl, cl = H.levels[l], H.levels[l - 1]
        assert np.all(X.row < cl.off_ps) and np.all((X.col >= fl.off_u) & (X.col < fl.off_pf))
        # the prolongation never mixes the groups
        P = sp.coo_matrix(H.P[l])
        assert np.all(gf[P.row] == gc[P.col])


def test_block_diagonal_and_linear(c2):
    H, _ = c2
    lv = H.finest
    g = field_groups(lv)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(lv.N)
    r1, r2 = np.where(g == 0, r, 0.0), np.where(g == 1, r, 0.0)
    z1, z2, z = H.vcycle(r1), H.vcycle(r2), H.vcycle(r)
    assert np.abs(z1[g == 1]).max() == 0.0 and np.abs(z2[g == 0]).max() == 0.0
    assert np.abs(z1[g == 0]).max() > 0 and np.abs(z2[g == 1]).max() > 0
    assert np.allclose(z, z1 + z2, rtol=0, atol=1e-12 * np.abs(z).max())
    # the standard cascade is not block diagonal: a residual in the [u, p^f]
    # group moves the [d, p^s] group (the interface traction of the solid
    # momentum rows and R_2's routing); the steady operator is block upper
    # triangular, so the other direction stays zero there too
    Hs = Hierarchy(dict(H.cfg, interchange=False), H.w_finest)
    zs = Hs.vcycle(r2)
    assert np.linalg.norm(zs[g == 0]) > 1e-2 * np.linalg.norm(zs[g == 1])


def test_two_level_closed_form():
    cfg = dict(inputs.config("c1"), interchange=True)
    H = Hierarchy(cfg, None)
    A, P, R = H.Ac[1].toarray(), H.P[1].toarray(), H.Rc[1].toarray()
    N = A.shape[0]
    B = H.smoothers[1].dense(H.Ac[1])
    om = cfg["omega"]
    S = np.eye(N) - om * B @ A
    C = np.eye(N) - P @ np.linalg.solve(H.Ac[0].toarray(), R @ A)
    E = np.linalg.matrix_power(S, cfg["nu_post"]) @ C @ np.linalg.matrix_power(S, cfg["nu_pre"])
    M = (np.eye(N) - E) @ np.linalg.inv(A)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(N)
    z = H.vcycle(r)
    assert np.allclose(z, M @ r, rtol=0, atol=1e-9 * np.abs(z).max())


def test_fgmres_converges(c2):
    H, O = c2
    b = O.rhs(inputs.body_force(H.cfg))
    A = O.A[-1]
    x, info = fgmres(lambda v: A @ v, H.vcycle, b, restart=30, rtol=1e-10, max_restarts=40)
    assert info["converged"]
    xd = direct_solve(A, b)
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)

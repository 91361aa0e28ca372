"""Pins of the oracle's smoother, V-cycle, FGMRES and adjoint.

* every Schwarz block is a principal submatrix of the level operator with
  the field structure of AS_1 / AS_2 (Section 3.2);
* the sweep equals the dense operator sum_j E_j inv(A_j) R_j + Jacobi built
  with numpy.linalg.inv (independent of the LU path), applied to unit vectors;
* two-level V-cycle = (I - E_TG) A^{-1} with E_TG = S^nu2 (I - P A0^{-1} R A) S^nu1;
* a one-level hierarchy makes FGMRES converge in one iteration;
* FGMRES agrees with a sparse direct solve, its residual estimates never
  increase and the final estimate equals the true residual;
* the transposed V-cycle is the exact transpose; the adjoint matches a direct
  solve of A^T; parameter gradients match central finite differences.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import adjoint, fem
from oracle.krylov import fgmres
from oracle.multigrid import Hierarchy
from oracle.schwarz import build_blocks
from paper_1909_13201_amd import inputs


@pytest.fixture(scope="module")
def c1():
    cfg = inputs.config("c1")
    return cfg, Hierarchy(cfg)


def test_blocks_structure(c1):
    cfg, H = c1
    lv = H.finest
    blocks, kinds = build_blocks(lv, cfg["core"], cfg["halo"])
    A = H.A[-1].tocsr()
    N2D = 2 * lv.N2
    sizes = []
    for I, (field, region) in zip(blocks, kinds):
        isd = I < N2D
        isps = (I >= lv.off_ps) & (I < lv.off_u)
        isu = (I >= lv.off_u) & (I < lv.off_pf)
        ispf = I >= lv.off_pf
        if field == 0 and region == 1:
            assert np.all(isd | isps) and isps.any()
            assert np.all(lv.solid_side[I[isd] // 2])
        elif field == 0:
            assert np.all(isd) and not np.any(lv.solid_side[I // 2])
        else:
            assert np.all(isu | ispf) and ispf.any()
            assert not np.any(lv.solid_side[(I[isu] - lv.off_u) // 2])
        assert not np.any(lv.dir_mask[I])
        sizes.append(len(I))
    # 2x2 cores with a one-element halo: 4x4 elements -> 9x9 nodes, 9 pressures
    assert max(sizes) == 9 * 9 * 2 + 9
    # u^s and Dirichlet unknowns are in no block
    cover = np.zeros(lv.N, bool)
    for I in blocks:
        cover[I] = True
    us = lv.u(np.where(lv.solid_side)[0][:, None], np.arange(2)).ravel()
    assert not cover[us].any()
    assert np.all(cover | lv.dir_mask | np.isin(np.arange(lv.N), us))


def test_enlarged_interface_cores_counted_by_hand():
    """c3 at 4 levels: 128 x 64 elements, solid rows [0,16) and [48,64), 4x4
    tiles (32 columns x 16 rows).  With iface_mult = 3 the tile rows touching
    the interface (3 and 12 solid, 4 and 11 fluid) take over two rows each
    away from the interface, leaving per tile column 2 + 2 solid, 4 fluid-d
    and 4 fluid-u cores; the enlarged fluid cores are 4 x 12 elements, so
    their u-blocks carry 5 x 13 pressures instead of 5 x 5."""
    cfg = inputs.with_levels(inputs.config("c3"), 4)
    H = Hierarchy(cfg, None, build_smoothers=False)
    lv = H.finest
    assert tuple(lv.ne) == (128, 64)
    plain, _ = build_blocks(lv, cfg["core"], cfg["halo"], 1)
    blocks, kinds = build_blocks(lv, cfg["core"], cfg["halo"], 3)
    assert len(plain) == 32 * (8 + 8 + 8)
    assert len(blocks) == 32 * (4 + 4 + 4)
    assert sum(k == (0, 1) for k in kinds) == 32 * 4
    npf = sorted(int(np.sum(I >= lv.off_pf)) for I, k in zip(blocks, kinds) if k[0] == 1)
    assert npf == [25] * 64 + [65] * 64
    # interior u-block: 6x6 elements with the halo -> 13x13 nodes x 2 + 25;
    # enlarged: 6x13 elements, the interface node row excluded -> 13x26 x 2 + 65
    small = [len(I) for I, k in zip(blocks, kinds) if k[0] == 1 and np.sum(I >= lv.off_pf) == 25]
    big = [len(I) for I, k in zip(blocks, kinds) if k[0] == 1 and np.sum(I >= lv.off_pf) == 65]
    assert max(small) == 13 * 13 * 2 + 25 and max(big) == 13 * 26 * 2 + 65


def test_monolithic_blocks_structure():
    """The comparator's blocks (the AS formula of Section 3.2): per core and
    region one block over d, u and p of that region, so u^s and the kinematic
    rows sit in the solid blocks and only Dirichlet unknowns are left to the
    Jacobi step; the principal submatrices have the zero pattern of P^s_1j
    (p^s rows see no u, kinematic rows no p) and P^f_1j (ALE rows see only d).
    The field-split index sets of the same cores are subsets of them."""
    cfg = inputs.with_levels(inputs.config("c2"), 3)
    H = Hierarchy(cfg, inputs.advecting_field(cfg), build_smoothers=False)
    lv, A = H.finest, H.A[-1].tocsr()
    mono, kinds = build_blocks(lv, cfg["core"], cfg["halo"], 1, True)
    fs, _ = build_blocks(lv, cfg["core"], cfg["halo"], 1, False)
    assert all(k[0] == 2 for k in kinds)
    cover = np.zeros(lv.N, bool)
    for I in mono:
        cover[I] = True
    assert np.array_equal(~cover, lv.dir_mask)
    N2D = 2 * lv.N2
    for I, (_, region) in zip(mono, kinds):
        isd = I < N2D
        isu = (I >= lv.off_u) & (I < lv.off_pf)
        isp = ~(isd | isu)
        Aj = A[I][:, I].toarray()
        if region == 1:
            assert np.all(Aj[np.ix_(isp, isu)] == 0) and np.all(Aj[np.ix_(isu, isp)] == 0)
        else:
            assert np.all(Aj[np.ix_(isd, isu | isp)] == 0)
    # every field-split block lies inside the monolithic block of its core
    mono_sets = [set(I.tolist()) for I in mono]
    for I in fs:
        assert any(set(I.tolist()) <= M for M in mono_sets)


def test_smoother_matches_dense_inverse(c1):
    cfg, H = c1
    S = H.smoothers[-1]
    A = H.A[-1]
    B = S.dense(A)
    rng = np.random.default_rng(3)
    R = rng.standard_normal((A.shape[0], 5))
    for k in range(5):
        assert np.allclose(S.apply(R[:, k]), B @ R[:, k], rtol=1e-10, atol=1e-10 * abs(B).max())
        assert np.allclose(S.apply_transpose(R[:, k]), B.T @ R[:, k], rtol=1e-10,
                           atol=1e-10 * abs(B).max())
    # last-writer rule: each row of B only has entries inside its owner block
    own = S.owner
    for i in rng.choice(np.where(own >= 0)[0], 20, replace=False):
        nz = np.nonzero(B[i])[0]
        assert np.all(np.isin(nz, S.blocks[own[i]]))


def test_two_level_exact_composition(c1):
    cfg, H = c1
    A = H.A[-1].toarray()
    N = A.shape[0]
    B = H.smoothers[-1].dense(H.A[-1])
    om = cfg["omega"]
    Sm = np.eye(N) - om * B @ A
    P = H.P[1].toarray()
    R = H.R[1].toarray()
    A0inv = np.linalg.inv(H.A[0].toarray())
    E = (np.linalg.matrix_power(Sm, cfg["nu_post"]) @ (np.eye(N) - P @ A0inv @ R @ A)
         @ np.linalg.matrix_power(Sm, cfg["nu_pre"]))
    M_expected = (np.eye(N) - E) @ np.linalg.inv(A)
    M = H.dense_preconditioner()
    assert np.allclose(M, M_expected, rtol=0, atol=1e-9 * abs(M_expected).max())
    MT = H.dense_preconditioner(transpose=True)
    assert np.allclose(MT, M.T, rtol=0, atol=1e-12 * abs(M).max())


@pytest.mark.parametrize("kind", ["V", "W", "F"])
def test_three_level_cycle_compositions(kind):
    """Three levels (coarse 2x2 with a solid bottom row -> 8x8): the cycle
    equals (I - E_2) A_2^-1 with the closed-form error propagation
        E_l = S_l^nu2 (I - P_l (I - E_c) A_{l-1}^-1 R_l A_l) S_l^nu1,
        E_c = E_{l-1} (V),  E_{l-1}^2 (W),  E^V_{l-1} E^F_{l-1} (F),  E_0 = 0,
    S_l = I - omega B_l A_l with B_l the dense smoother (numpy.linalg.inv
    blocks); and the transposed cycle is its transpose."""
    import tests.cfgs as cfgs
    cfg = cfgs.small(nc=(2, 2), solid_rows=(0,), levels=3, yb=[0.0, 0.25, 1.0],
                     core=(2, 2), halo=1, omega=0.8, cycle=kind,
                     bc_d=inputs.config("c1")["bc_d"], bc_u=inputs.config("c1")["bc_u"])
    H = Hierarchy(cfg)
    A = [a.toarray() for a in H.A]
    om = cfg["omega"]

    def S(l):
        B = H.smoothers[l].dense(H.A[l])
        return np.eye(A[l].shape[0]) - om * B @ A[l]

    def E(l, k):
        if l == 0:
            return np.zeros_like(A[0])
        P, R = H.P[l].toarray(), H.R[l].toarray()
        Ec = {"V": lambda: E(l - 1, "V"), "W": lambda: np.linalg.matrix_power(E(l - 1, "W"), 2),
              "F": lambda: E(l - 1, "V") @ E(l - 1, "F")}[k]()
        n = A[l].shape[0]
        cgc = np.eye(n) - P @ (np.eye(Ec.shape[0]) - Ec) @ np.linalg.inv(A[l - 1]) @ R @ A[l]
        Sl = S(l)
        return (np.linalg.matrix_power(Sl, cfg["nu_post"]) @ cgc
                @ np.linalg.matrix_power(Sl, cfg["nu_pre"]))

    N = A[2].shape[0]
    M_expected = (np.eye(N) - E(2, kind)) @ np.linalg.inv(A[2])
    M = H.dense_preconditioner()
    assert np.allclose(M, M_expected, rtol=0, atol=1e-9 * abs(M_expected).max())
    MT = H.dense_preconditioner(transpose=True)
    assert np.allclose(MT, M.T, rtol=0, atol=1e-11 * abs(M).max())
    if kind != "V":    # the cycles differ once there are three levels
        Hv = Hierarchy(dict(cfg, cycle="V"))
        assert not np.allclose(M, Hv.dense_preconditioner(), rtol=0, atol=1e-6 * abs(M).max())


def test_one_level_gmres_one_iteration():
    cfg = inputs.with_levels(inputs.config("c1"), 1)
    H = Hierarchy(cfg)
    b = H.rhs(inputs.body_force(inputs.config("c1"))[:H.finest.N2] * 0 + 1.0)
    x, info = fgmres(lambda v: H.A[-1] @ v, H.vcycle, b, rtol=1e-10)
    assert info["converged"] and info["iters"] == 1


def test_fgmres_vs_direct_and_monotone(c1):
    cfg, H = c1
    A = H.A[-1]
    b = H.rhs(inputs.body_force(cfg))
    xd = spla.splu(A.tocsc()).solve(b)
    x, info = fgmres(lambda v: A @ v, H.vcycle, b, rtol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    hist = np.array(info["history"])
    assert np.all(np.diff(hist) <= 1e-14)
    assert info["rel_res_true"] == pytest.approx(hist[-1], rel=1e-3)
    kappa = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - xd) <= kappa * 1e-10 * np.linalg.norm(xd)
    # Dirichlet values are met
    lv = H.finest
    assert np.allclose(x[lv.dir_mask], lv.dir_val[lv.dir_mask], atol=1e-12)


def test_fgmres_restart_still_monotone(c1):
    cfg, H = c1
    A = H.A[-1]
    b = H.rhs(inputs.body_force(cfg))
    x, info = fgmres(lambda v: A @ v, H.vcycle, b, restart=3, rtol=1e-10)
    assert info["converged"] and info["restarts"] > 0
    hist = np.array(info["history"])
    assert np.all(np.diff(hist) <= 1e-12)


def _small_c5():
    cfg = inputs.with_levels(inputs.config("c5"), 2)
    return cfg, inputs.advecting_field(cfg)


def test_steady_outlet_flux_equals_inflow():
    """Steady: walls are impermeable (K rows give u = 0 on the solid) and the
    fluid continuity rows hold for the constant pressure test function, so the
    outlet flux equals the prescribed parabolic inflow flux, peak * (2/3) *
    height = 0.8 * 2/3 for the channel, whatever the load and parameters."""
    for E, mu, seed in ((1e4, 3.5e-3, 0), (3e3, 2e-2, 7)):
        cfg = inputs.with_levels(inputs.config("c2"), 2)
        cfg.update(E=E, mu=mu)
        w = inputs.advecting_field(cfg)
        H = Hierarchy(cfg, w, build_smoothers=False)
        b = H.rhs(inputs.body_force(cfg, seed=seed))
        x = spla.splu(H.A[-1].tocsc()).solve(b)
        J = adjoint.outlet_flux_vector(H.finest) @ x
        assert J == pytest.approx(0.8 * 2.0 / 3.0, rel=1e-10)


def test_adjoint_and_gradients_vs_fd():
    cfg, w = _small_c5()
    H = Hierarchy(cfg, w)
    lv = H.finest
    f = inputs.body_force(cfg)
    b = H.rhs(f)
    A = H.A[-1]
    c = adjoint.outlet_flux_vector(lv)
    x, info = fgmres(lambda v: A @ v, H.vcycle, b, rtol=1e-12, max_restarts=40)
    assert info["converged"]
    lam, ainfo = adjoint.adjoint_solve(H, c, rtol=1e-11, max_restarts=40)
    assert ainfo["converged"]
    lam_d = spla.splu(A.T.tocsc()).solve(c)
    assert np.linalg.norm(lam - lam_d) <= 1e-8 * np.linalg.norm(lam_d)
    gE, gmu = adjoint.gradients(H, x, lam)
    taus = [p["tau"] for p in H.parts]

    def J(E, mu):
        c2 = dict(cfg, E=E, mu=mu)
        asm = fem.assemble_level(lv, c2, lv.inject_from_finest(w, H.L), taus[-1])
        Ar = fem.dirichlet_reduce(lv, asm["A"])
        bb = fem.dirichlet_rhs(lv, asm["A"], fem.load_vector(lv, c2, f, w, taus[-1]))
        return c @ spla.splu(Ar.tocsc()).solve(bb)

    # FD noise: direct solves carry relative error ~1e-11 in J at this
    # conditioning (~2e12), so a central difference with h = 1e-6 has noise
    # ~1e-5; a 4-point stencil in log-parameters at h = 1e-2 has truncation
    # error ~h^4 and noise ~1e-9, both far below the 1e-6 tolerance.
    h = 1e-2
    E0, mu0 = cfg["E"], cfg["mu"]
    d4 = lambda g: (-g(2 * h) + 8 * g(h) - 8 * g(-h) + g(-2 * h)) / (12 * h)
    fdE = d4(lambda t: J(E0 * np.exp(t), mu0))
    fdmu = d4(lambda t: J(E0, mu0 * np.exp(t)))
    assert E0 * gE == pytest.approx(fdE, rel=1e-6)
    assert mu0 * gmu == pytest.approx(fdmu, rel=1e-6)
    # dJ/db = lambda: directional check against a perturbed right-hand side
    rng = np.random.default_rng(5)
    db = rng.standard_normal(lv.N)
    Ad = spla.splu(A.tocsc())
    assert c @ Ad.solve(db) == pytest.approx(lam @ db, rel=1e-8)

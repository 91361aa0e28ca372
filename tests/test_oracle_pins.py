"""Pins of the oracle's remaining assembly and transfer parts.

Each test checks the oracle against something fixed by the paper and the
mathematics, never against the oracle itself:

* ALE coefficient k = 1/V_el (Section 2.2, the choice of k after eq.
  newtonian), with V_el the volume of the coarsest-mesh element containing
  the point: for a displacement of constant gradient on a fluid-only graded
  mesh, d^T A_dd d = sum_e k_e V_e (grad d + grad d^T) : grad d, which is
  (number of coarse elements) x (grad d + grad d^T) : grad d on every level
  with k = 1/V_coarse, the total volume times it with k = 1; the volumes
  are written out from the breakpoints by hand.
* Galerkin identity R A_f P = A_c on free rows and columns (Section 3.3)
  with the level-independent ALE coefficient, consistent kinematic mass,
  a backward-Euler step and three levels, in 2D and 3D: every coarse test
  and trial function is a fine one and k is constant on coarse elements.
* backward-Euler terms (eqs. kinsld, momentum_supg with one backward
  difference): polynomial d, u, p in the discrete spaces with u = d/dt on
  the solid and f built from the strong form including rho u/dt make every
  K row and every interior S, V, F, W row (SUPG time term included) vanish;
  a perturbed dt breaks them.
* 3D (hexahedral Q2/Q1): the solid, Oseen + SUPG and ALE patch tests, the
  SUPG lambda_k of a cube (64/h^2, derived by exact integration of the
  definition), reproduction of triquadratic / trilinear fields by P and the
  R_2 zero pattern.
* mapped geometry (circular and smooth bulge, mappings 1 and 2): fields
  linear in the physical coordinates are reproduced exactly by isoparametric
  Q2, so constant-stress solid, fluid and ALE states leave zero residual on
  interior test functions.  SUPG is off there: its second derivatives use
  the element Jacobian only, exact on affine elements alone.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import sympy as sy

from oracle import fem, transfer
from oracle.mesh import Level
from tests.cfgs import channel3d, small

SYM = sy.symbols("x y z")


# --------------------------------------------------------------------------
# helpers (generic in the dimension)
# --------------------------------------------------------------------------
def _interior_nodes(lv):
    m = np.ones(lv.N2, bool)
    for a in range(lv.D):
        m &= (lv.nidx[:, a] > 0) & (lv.nidx[:, a] < lv.nn[a] - 1)
    return m


def _eval(expr, X):
    """Evaluate a sympy expression of x, y(, z) at points X (n, D)."""
    D = X.shape[1]
    f = sy.lambdify(SYM[:D], expr, "numpy")
    return np.broadcast_to(np.asarray(f(*[X[:, a] for a in range(D)]), float), (X.shape[0],)).copy()


def _nodal(lv, exprs):
    return np.stack([_eval(e, lv.X) for e in exprs], axis=1)


def _vertex_X(lv, flags):
    return lv.X[lv.node_of_vertex(np.where(flags)[0])]


def _state(lv, d=None, u=None, ps=None, pf=None):
    D = lv.D
    x = np.zeros(lv.N)
    if d is not None:
        x[:D * lv.N2] = _nodal(lv, d).ravel()
    if u is not None:
        x[lv.off_u:lv.off_u + D * lv.N2] = _nodal(lv, u).ravel()
    if ps is not None and lv.Nps:
        x[lv.off_ps:lv.off_ps + lv.Nps] = _eval(ps, _vertex_X(lv, lv.vert_solid))
    if pf is not None and lv.Npf:
        x[lv.off_pf:lv.off_pf + lv.Npf] = _eval(pf, _vertex_X(lv, lv.vert_fluid))
    return x


def _grad(v, D):
    return sy.Matrix(D, D, lambda i, j: sy.diff(v[i], SYM[j]))


def _div_tensor(T, D):
    return [sum(sy.diff(T[i, j], SYM[j]) for j in range(D)) for i in range(D)]


def _solid_force(d, p, G, D, rho=1.0, u=None, dt=None):
    """f = (rho u/dt - div(-p I + G (grad d + grad d^T))) / rho."""
    gd = _grad(d, D)
    sig = -p * sy.eye(D) + G * (gd + gd.T)
    dv = _div_tensor(sig, D)
    f = [-dv[i] / rho for i in range(D)]
    if dt is not None:
        f = [f[i] + u[i] / dt for i in range(D)]
    return [sy.expand(e) for e in f]


def _fluid_force(u, p, mu, w, D, rho=1.0, dt=None):
    """f = (rho u/dt + rho (w.grad) u - div(-p I + mu (grad u + grad u^T))) / rho."""
    gu = _grad(u, D)
    sig = -p * sy.eye(D) + mu * (gu + gu.T)
    dv = _div_tensor(sig, D)
    conv = [sum(w[j] * gu[i, j] for j in range(D)) for i in range(D)]
    f = [(rho * conv[i] - dv[i]) / rho for i in range(D)]
    if dt is not None:
        f = [f[i] + u[i] / dt for i in range(D)]
    return [sy.expand(e) for e in f]


def _rows(lv, r, which):
    D = lv.D
    if which == "d":
        return r[:D * lv.N2].reshape(-1, D)
    if which == "u":
        return r[lv.off_u:lv.off_u + D * lv.N2].reshape(-1, D)
    if which == "ps":
        return r[lv.off_ps:lv.off_ps + lv.Nps]
    return r[lv.off_pf:lv.off_pf + lv.Npf]


def _region_cfg3(nc, solid_layers, levels=1, **kw):
    """3D box [0,1]^3 (graded when breaks are given) with solid y-layers."""
    region = np.zeros((nc[2], nc[1], nc[0]), np.int8)
    for r in solid_layers:
        region[:, r, :] = 1
    cfg = channel3d(levels=levels, nc=nc)
    cfg.update(region=region.ravel(), bc_d=[[0, 0] for _ in range(6)],
               bc_u=[[0, 0] for _ in range(6)], supg=False)
    cfg.update(kw)
    return cfg


# --------------------------------------------------------------------------
# ALE coefficient k = 1/V of the coarsest element containing the point
# --------------------------------------------------------------------------
def _coarse_volumes_by_hand(cfg):
    """Products of breakpoint differences, x fastest (affine meshes only)."""
    D = cfg["dim"]
    widths = [np.diff(np.asarray(cfg["breaks"][a], float)) for a in range(D)]
    V = widths[0]
    for a in range(1, D):
        V = np.multiply.outer(widths[a], V).ravel()
    return V


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_ale_coefficient_energy_identity(dim, level):
    if dim == 2:
        cfg = small(nc=(3, 4), solid_rows=(), levels=3,
                    xb=[0, 0.15, 0.55, 1.0], yb=[0, 0.1, 0.35, 0.6, 1.0])
    else:
        if level == 2:
            pytest.skip("3D level 2 is covered by levels 0 and 1 (size)")
        cfg = _region_cfg3((2, 3, 2), (), levels=2)
        cfg["breaks"] = ([0, 0.3, 1.0], [0, 0.2, 0.45, 1.0], [0, 0.7, 1.0])
    D = dim
    Vc = _coarse_volumes_by_hand(cfg)
    assert np.allclose(Vc, fem.coarse_element_volumes(cfg), rtol=1e-13, atol=0)
    lv = Level(cfg, level)
    rng = np.random.default_rng(7)
    Gm = rng.standard_normal((D, D))
    d = [sum(float(Gm[i, j]) * SYM[j] for j in range(D)) + 0.3 * i for i in range(D)]
    x = _state(lv, d=d)
    energy = float((Gm + Gm.T).ravel() @ Gm.ravel())
    Dn = D * lv.N2
    for ale_k, expect in ((0, len(Vc) * energy), (1, Vc.sum() * energy)):
        A = fem.assemble_level(lv, dict(cfg, ale_k=ale_k))["A"].tocsr()
        Add = A[:Dn][:, :Dn]
        got = x[:Dn] @ (Add @ x[:Dn])
        assert got == pytest.approx(expect, rel=1e-11)
    # per-level element volumes would give (elements on this level) x energy
    if level > 0:
        assert abs(lv.nE * energy - len(Vc) * energy) > 1e-3 * abs(energy)


def _galerkin_cfg(dim, ale_k, dt):
    if dim == 2:
        cfg = small(nc=(2, 3), solid_rows=(0,), levels=3, ale_k=ale_k, k_mass=1,
                    xb=[0, 0.4, 1.0], yb=[0, 0.15, 0.55, 1.0])
        cfg["bc_d"][0][0] = cfg["bc_d"][0][1] = 1
        cfg["bc_u"][0][0] = 2
        cfg["bc_u"][3][0] = 1
    else:
        cfg = _region_cfg3((1, 2, 1), (0,), levels=2, ale_k=ale_k, k_mass=1)
        cfg["breaks"] = ([0, 1.0], [0, 0.3, 1.0], [0, 1.0])
        cfg["bc_d"][0][0] = cfg["bc_d"][0][1] = 1
        cfg["bc_u"][0][0] = 2
        cfg["bc_u"][3][0] = 1
    if dt is not None:
        cfg["dt"] = dt
    return cfg


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("ale_k", [0, 1])
@pytest.mark.parametrize("dt", [None, 0.05])
def test_galerkin_identity_ale_and_time_step(dim, ale_k, dt):
    cfg = _galerkin_cfg(dim, ale_k, dt)
    L = cfg["n_levels"]
    for lf in range(1, L):
        fine, coarse = Level(cfg, lf), Level(cfg, lf - 1)
        Af = fem.dirichlet_reduce(fine, fem.assemble_level(fine, cfg)["A"])
        Ac = fem.dirichlet_reduce(coarse, fem.assemble_level(coarse, cfg)["A"])
        P = transfer.prolongation(fine, coarse)
        R = transfer.restriction(fine, coarse)
        G = (R @ Af @ P).toarray()
        fr = coarse.free
        ref = Ac.toarray()[np.ix_(fr, fr)]
        assert np.allclose(G[np.ix_(fr, fr)], ref, atol=1e-10 * abs(ref).max(), rtol=0), lf


# --------------------------------------------------------------------------
# backward-Euler step
# --------------------------------------------------------------------------
def _be_solid_case(dim):
    x, y, z = SYM
    if dim == 2:
        cfg = small(nc=(3, 4), solid_rows=(0, 1, 2, 3), E=7.0, nu=0.3, rho=1.7,
                    xb=[0, 0.2, 0.7, 1.0], yb=[0, 0.1, 0.5, 0.6, 1.0])
        d = [x * x + 2 * x * y - y * y, 3 * x * x - x * y + 2 * y * y]
    else:
        cfg = _region_cfg3((2, 2, 2), (0, 1), E=7.0, nu=0.3, rho=1.7)
        cfg["breaks"] = ([0, 0.3, 1.0], [0, 0.6, 1.0], [0, 0.45, 1.0])
        d = [x * x + 2 * x * y - y * y + z * z, 3 * x * x - x * y + 2 * y * z,
             x * z - z * z + y * y]
    return cfg, d


@pytest.mark.parametrize("dim", [2, 3])
def test_backward_euler_solid_patch(dim):
    cfg, d = _be_solid_case(dim)
    dt = 0.37
    cfg["dt"] = dt
    D = dim
    G, inv_lam = fem.lame_constants(cfg["E"], cfg["nu"])
    divd = sum(sy.diff(d[i], SYM[i]) for i in range(D))
    p = sy.expand(-divd / inv_lam)
    u = [sy.expand(e / dt) for e in d]                       # kinematic: u = dd/dt
    f = _solid_force(d, p, G, D, rho=cfg["rho"], u=u, dt=dt)
    lv = Level(cfg, 0)
    x = _state(lv, d=d, u=u, ps=p)
    fn = _nodal(lv, f)
    inner = _interior_nodes(lv)

    def residual(c):
        return fem.assemble_level(lv, c)["A"] @ x - fem.load_vector(lv, cfg, fn)

    r = residual(cfg)
    scale = abs(fem.assemble_level(lv, cfg)["A"]).max() * abs(x).max()
    assert abs(_rows(lv, r, "u")[lv.solid_side]).max() < 1e-12 * scale      # K rows, all nodes
    assert abs(_rows(lv, r, "d")[inner]).max() < 1e-12 * scale              # S rows
    assert abs(_rows(lv, r, "ps")).max() < 1e-12 * scale                    # V rows
    # sharpness: the K_ds = -K_us / dt and rho M / dt terms
    r2 = residual(dict(cfg, dt=dt * 1.01))
    assert abs(_rows(lv, r2, "u")[lv.solid_side]).max() > 1e-6 * scale
    assert abs(_rows(lv, r2, "d")[inner]).max() > 1e-6 * scale
    # the steady operator (no K_ds, no inertia) does not satisfy it either
    r3 = residual(dict(cfg, dt=np.inf))
    assert abs(_rows(lv, r3, "u")[lv.solid_side]).max() > 1e-6 * scale


def _be_fluid_case(dim):
    x, y, z = SYM
    if dim == 2:
        cfg = small(nc=(4, 3), solid_rows=(), mu=0.05, rho=1.3, supg=True, ale_k=1,
                    xb=[0, 0.3, 0.5, 0.8, 1.0], yb=[0, 0.25, 0.7, 1.0])
        u = [y * y + x * y, x * x - sy.Rational(1, 2) * y * y]
        d = [x * x - y * y, -2 * x * y]
        p = x + 2 * y
        w = (0.3, -0.2)
    else:
        cfg = _region_cfg3((2, 2, 2), (), mu=0.05, rho=1.3, supg=True, ale_k=1)
        cfg["breaks"] = ([0, 0.4, 1.0], [0, 0.55, 1.0], [0, 0.3, 1.0])
        u = [y * y + x * y + z * z, x * x - sy.Rational(1, 2) * y * y + x * z, x * x + y * y]
        d = [x * x - y * y, -2 * x * y, 0 * z]
        p = x + 2 * y - z
        w = (0.3, -0.2, 0.25)
    return cfg, u, d, p, w


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dt", [None, 0.21])
def test_oseen_supg_ale_patch(dim, dt):
    """Fluid momentum (inertia, convection, viscous, pressure, SUPG including
    its time term), continuity and ALE rows vanish for polynomial states."""
    cfg, u, d, p, w = _be_fluid_case(dim)
    D = dim
    if dt is not None:
        cfg["dt"] = dt
    assert sum(sy.diff(u[i], SYM[i]) for i in range(D)) == 0
    f = _fluid_force(u, p, cfg["mu"], w, D, rho=cfg["rho"], dt=dt)
    lv = Level(cfg, 0)
    x = _state(lv, d=d, u=u, pf=p)
    wn = np.tile(np.asarray(w, float), (lv.N2, 1))
    fn = _nodal(lv, f)
    asm = fem.assemble_level(lv, cfg, wn)
    assert asm["tau"] is not None
    r = asm["A"] @ x - fem.load_vector(lv, cfg, fn, wn, asm["tau"])
    inner = _interior_nodes(lv)
    scale = abs(asm["A"]).max() * abs(x).max()
    assert abs(_rows(lv, r, "u")[inner]).max() < 1e-11 * scale             # F rows
    assert abs(_rows(lv, r, "d")[inner]).max() < 1e-11 * scale             # A rows
    assert abs(_rows(lv, r, "pf")).max() < 1e-11 * scale                   # W rows
    # sharpness: a wrong viscosity, and for the time step a wrong dt
    r2 = (fem.assemble_level(lv, dict(cfg, mu=cfg["mu"] * 1.1), wn)["A"] @ x
          - fem.load_vector(lv, cfg, fn, wn, asm["tau"]))
    assert abs(_rows(lv, r2, "u")[inner]).max() > 1e-6 * scale
    if dt is not None:
        c3 = dict(cfg, dt=dt * 1.01)
        r3 = (fem.assemble_level(lv, c3, wn, asm["tau"])["A"] @ x
              - fem.load_vector(lv, cfg, fn, wn, asm["tau"]))
        assert abs(_rows(lv, r3, "u")[inner]).max() > 1e-6 * scale


def test_supg_time_term_is_tested():
    """The SUPG counterpart of rho u/dt is what makes the fluid rows vanish
    above: without it (SUPG built with the steady operator but the inertia
    kept) the interior residual is of the order of tau rho^2 |u|/dt."""
    cfg, u, d, p, w = _be_fluid_case(2)
    dt = 0.21
    cfg["dt"] = dt
    f = _fluid_force(u, p, cfg["mu"], w, 2, rho=cfg["rho"], dt=dt)
    lv = Level(cfg, 0)
    x = _state(lv, d=d, u=u, pf=p)
    wn = np.tile(np.asarray(w, float), (lv.N2, 1))
    fn = _nodal(lv, f)
    full = fem.assemble_level(lv, cfg, wn)
    steady = fem.assemble_level(lv, dict(cfg, dt=np.inf), wn, full["tau"])
    Mi = fem.assemble_level(lv, dict(cfg, dt=dt, supg=False), None)["A"] - \
        fem.assemble_level(lv, dict(cfg, supg=False, dt=np.inf), None)["A"]
    A_no_supg_time = steady["A"] + Mi
    r = A_no_supg_time @ x - fem.load_vector(lv, cfg, fn, wn, full["tau"])
    inner = _interior_nodes(lv)
    scale = abs(full["A"]).max() * abs(x).max()
    assert abs(_rows(lv, r, "u")[inner]).max() > 1e-8 * scale


# --------------------------------------------------------------------------
# 3D solid patch, SUPG lambda on a cube, transfers in 3D
# --------------------------------------------------------------------------
def test_patch_linear_elastic_solid_3d():
    x, y, z = SYM
    cfg = _region_cfg3((2, 3, 2), (0, 1, 2), E=7.0, nu=0.3)
    cfg["breaks"] = ([0, 0.35, 1.0], [0, 0.2, 0.5, 1.0], [0, 0.6, 1.0])
    G, inv_lam = fem.lame_constants(cfg["E"], cfg["nu"])
    d = [x * x + 2 * x * y - y * y + z * z, 3 * x * x - x * y + 2 * y * z, x * z - z * z + y * y]
    divd = sum(sy.diff(d[i], SYM[i]) for i in range(3))
    p = sy.expand(-divd / inv_lam)
    f = _solid_force(d, p, G, 3)
    lv = Level(cfg, 0)
    xv = _state(lv, d=d, ps=p)
    asm = fem.assemble_level(lv, cfg)
    r = asm["A"] @ xv - fem.load_vector(lv, cfg, _nodal(lv, f))
    inner = _interior_nodes(lv)
    assert inner.sum() > 0
    scale = abs(asm["A"]).max() * abs(xv).max()
    assert abs(_rows(lv, r, "d")[inner]).max() < 1e-12 * scale
    assert abs(_rows(lv, r, "ps")).max() < 1e-12 * scale
    r2 = fem.assemble_level(lv, dict(cfg, E=7.07))["A"] @ xv - fem.load_vector(lv, cfg, _nodal(lv, f))
    assert abs(_rows(lv, r2, "d")[inner]).max() > 1e-6 * scale


def _lambda_cube_exact():
    """lambda_k of eq. (lambda_k) on [0, h]^3 from its definition: the
    element's interior Q2 space is spanned by b e_a with the bubble
    b = x(h-x) y(h-y) z(h-z); v_a = div(grad(b e_a) + grad(b e_a)^T) =
    lap(b) e_a + grad(d_a b); lambda = max eig [int v_a.v_c] / int |grad b|^2."""
    x, y, z = SYM
    h = sy.symbols("h", positive=True)
    b = x * (h - x) * y * (h - y) * z * (h - z)
    X = (x, y, z)
    lap = sum(sy.diff(b, t, 2) for t in X)
    v = [[(lap if i == a else 0) + sy.diff(b, X[a], X[i]) for i in range(3)] for a in range(3)]
    box = [(t, 0, h) for t in X]
    M = sy.Matrix(3, 3, lambda a, c: sy.integrate(sum(v[a][i] * v[c][i] for i in range(3)), *box))
    Nb = sy.integrate(sum(sy.diff(b, t) ** 2 for t in X), *box)
    ev = [sy.simplify(e * h ** 2 / Nb) for e in M.eigenvals()]
    return max(float(e) for e in ev)


def test_supg_lambda_cube_closed_form():
    c = _lambda_cube_exact()
    assert c == pytest.approx(64.0, rel=1e-14)
    for h in (1.0, 0.25, 0.03):
        cfg = _region_cfg3((1, 1, 1), ())
        cfg["breaks"] = ([0, h], [0, h], [0, h])
        lv = Level(cfg, 0)
        ref = fem.RefElement(3)
        dV, Gr, H, _ = fem.geometry(ref, lv.X[lv.elem_nodes])
        lam = fem.supg_lambda(ref, dV, Gr, H)
        assert lam[0] == pytest.approx(64.0 / h ** 2, rel=1e-12)


def test_prolongation_reproduces_polynomials_3d():
    cfg = _region_cfg3((2, 3, 2), (0,), levels=2)
    cfg["breaks"] = ([0, 0.3, 1.0], [0, 0.2, 0.5, 1.0], [0, 0.6, 1.0])
    fine, coarse = Level(cfg, 1), Level(cfg, 0)
    P = transfer.prolongation(fine, coarse, masked=False)
    x, y, z = SYM
    q2 = [1 + x * x * y * y * z * z - 3 * x * y * z, y * y - 2 * x * x * y * z + x, z * z * x - y]
    q1 = 2 + x - 3 * y + 5 * x * y - x * y * z + 0.5 * z

    def vec(lv):
        v = np.zeros(lv.N)
        v[:3 * lv.N2] = _nodal(lv, q2).ravel()
        v[lv.off_u:lv.off_u + 3 * lv.N2] = 2 * _nodal(lv, q2).ravel()
        for flags, off, n in ((lv.vert_solid, lv.off_ps, lv.Nps),
                              (lv.vert_fluid, lv.off_pf, lv.Npf)):
            v[off:off + n] = _eval(q1, _vertex_X(lv, flags))
        return v

    assert np.allclose(P @ vec(coarse), vec(fine), atol=1e-13, rtol=0)
    # a non-Q2 field (x^3) is not reproduced: the test can fail
    cub = [x ** 3, 0 * x, 0 * x]
    vc = np.zeros(coarse.N)
    vc[:3 * coarse.N2] = _nodal(coarse, cub).ravel()
    vf = np.zeros(fine.N)
    vf[:3 * fine.N2] = _nodal(fine, cub).ravel()
    assert abs(P @ vc - vf).max() > 1e-4


def test_restriction_zero_pattern_3d():
    cfg = _region_cfg3((2, 2, 2), (0,), levels=2)
    fine, coarse = Level(cfg, 1), Level(cfg, 0)
    D = 3
    R = transfer.restriction(fine, coarse, masked=False).tocsr()
    Rdu = R[:D * coarse.N2][:, fine.off_u:fine.off_u + D * fine.N2].tocoo()
    assert Rdu.nnz > 0
    assert np.all(coarse.solid_side[Rdu.row // D])
    assert np.all(~fine.solid_side[Rdu.col // D])
    Ruu = R[coarse.off_u:coarse.off_u + D * coarse.N2][:, fine.off_u:fine.off_u + D * fine.N2].tocoo()
    assert not np.any(coarse.solid_side[Ruu.row // D] & ~fine.solid_side[Ruu.col // D])
    assert R[coarse.off_u:coarse.off_u + D * coarse.N2][:, :D * fine.N2].nnz == 0
    Rdd = R[:D * coarse.N2][:, :D * fine.N2].tocoo()
    fl = ~coarse.solid_side[Rdd.row // D]
    assert np.all(~fine.solid_side[Rdd.col[fl] // D])
    # every weight of R's momentum block is a P weight (transposed)
    P = transfer.prolongation(fine, coarse, masked=False)
    assert abs(R - P.T).max() > 0.1


# --------------------------------------------------------------------------
# mapped geometry
# --------------------------------------------------------------------------
def _bulge_cfg(mapping, **kw):
    cfg = small(nc=(6, 4), solid_rows=(0, 3), levels=2, xb=list(np.linspace(0, 2, 7)),
                yb=[0, 0.1, 0.5, 0.9, 1.0], **kw)
    cfg["mapping"] = mapping
    cfg["map_params"] = [1.0, 0.3, 0.5, 0.9]
    return cfg


@pytest.mark.parametrize("mapping", [1, 2])
def test_mapped_mesh_is_curved(mapping):
    """The bulge map makes non-affine elements (so the patch tests below
    exercise the isoparametric geometry, not an affine shortcut)."""
    cfg = _bulge_cfg(mapping)
    lv = Level(cfg, 1)
    Xe = lv.X[lv.elem_nodes]                                   # (nE, 9, 2)
    # an affine element has its centre node at the mean of its corners
    corners = Xe[:, [0, 2, 6, 8]].mean(axis=1)
    assert abs(Xe[:, 4] - corners).max() > 1e-4


@pytest.mark.parametrize("mapping", [1, 2])
def test_patch_mapped_solid(mapping):
    cfg = _bulge_cfg(mapping, E=7.0, nu=0.3)
    cfg["region"] = np.ones_like(cfg["region"])
    lv = Level(cfg, 1)
    G, inv_lam = fem.lame_constants(cfg["E"], cfg["nu"])
    x, y, _ = SYM
    d = [0.3 * x - 0.7 * y + 0.1, 0.2 * x + 0.5 * y]
    p = -(0.3 + 0.5) / inv_lam
    xv = _state(lv, d=d, ps=sy.Float(p))
    asm = fem.assemble_level(lv, cfg)
    r = asm["A"] @ xv
    inner = _interior_nodes(lv)
    scale = abs(asm["A"]).max() * abs(xv).max()
    assert abs(_rows(lv, r, "d")[inner]).max() < 1e-11 * scale
    assert abs(_rows(lv, r, "ps")).max() < 1e-11 * scale
    # a quadratic field in x is not in the mapped space's kernel: nonzero
    d2 = [x * x, 0 * y]
    r2 = asm["A"] @ _state(lv, d=d2, ps=sy.Float(0.0))
    assert abs(_rows(lv, r2, "d")[inner]).max() > 1e-6 * scale


@pytest.mark.parametrize("mapping", [1, 2])
@pytest.mark.parametrize("ale_k", [0, 1])
def test_patch_mapped_fluid_and_ale(mapping, ale_k):
    cfg = _bulge_cfg(mapping, mu=0.05, rho=1.3, supg=False, ale_k=ale_k)
    cfg["region"] = np.zeros_like(cfg["region"])
    lv = Level(cfg, 1)
    x, y, _ = SYM
    B = np.array([[0.4, -0.3], [0.6, -0.4]])                   # trace 0
    u = [float(B[0, 0]) * x + float(B[0, 1]) * y + 0.2, float(B[1, 0]) * x + float(B[1, 1]) * y]
    d = [0.3 * x - 0.7 * y, 0.2 * x + 0.5 * y]
    w = np.array([0.3, -0.2])
    rho = cfg["rho"]
    f = B @ w                                                  # (w.grad) u, p constant
    xv = _state(lv, d=d, u=u, pf=sy.Float(1.5))
    wn = np.tile(w, (lv.N2, 1))
    asm = fem.assemble_level(lv, cfg, wn)
    r = asm["A"] @ xv - fem.load_vector(lv, cfg, np.tile(f, (lv.N2, 1)), wn)
    inner = _interior_nodes(lv)
    scale = abs(asm["A"]).max() * abs(xv).max()
    assert abs(_rows(lv, r, "u")[inner]).max() < 1e-11 * scale
    assert abs(_rows(lv, r, "pf")).max() < 1e-11 * scale
    rd = _rows(lv, r, "d")
    if ale_k == 1:
        assert abs(rd[inner]).max() < 1e-11 * scale
    else:
        # k jumps across coarse elements: only test functions supported in
        # one coarse element see a constant k (level-1 nodes strictly inside
        # a coarse element: odd node-line indices on the level-0 grid x2)
        one = inner.copy()
        for a in range(2):
            one &= (lv.nidx[:, a] % 4) != 0
        assert one.sum() > 0
        assert abs(rd[one]).max() < 1e-11 * scale
        edge = inner & ~one
        assert abs(rd[edge]).max() > 1e-9 * scale           # where k jumps
    # sharpness: a wrong convection (rho doubled in the operator only)
    r2 = (fem.assemble_level(lv, dict(cfg, rho=2 * rho), wn)["A"] @ xv
          - fem.load_vector(lv, cfg, np.tile(f, (lv.N2, 1)), wn))
    assert abs(_rows(lv, r2, "u")[inner]).max() > 1e-6 * scale


@pytest.mark.parametrize("mapping", [1, 2])
def test_mapped_area_closed_form(mapping):
    """Areas of the mapped coarse element rows from the isoparametric element
    volumes against the closed form.  The map moves a point of reference
    height eta up by b(x) s(eta), b the bulge profile (circle: sqrt(R^2 -
    (x - xc)^2), integral pi R^2 / 2; smooth: R cos^2(pi (x - xc) / (2R)),
    integral R^2) and s the linear blend from 0 at ya to 1 at yb, so a row
    between reference heights e0 < e1 gains int b dx * (s(e1) - s(e0)):
    the rows below ya and above yb keep their area, the row from 0.5 to 0.9
    gains the whole bulge."""
    cfg = _bulge_cfg(mapping)
    xc, R, ya, yb = cfg["map_params"]
    bump_area = np.pi * R * R / 2 if mapping == 1 else R * R
    rows = np.diff(np.asarray(cfg["breaks"][1]))
    s = lambda e: np.clip((e - ya) / (yb - ya), 0.0, 1.0)
    e = np.asarray(cfg["breaks"][1])
    expect = 2.0 * rows + bump_area * (s(e[1:]) - s(e[:-1]))
    errs = []
    for L in (1, 2, 3, 4):
        lv = Level(dict(cfg, n_levels=L), L - 1)
        dV = fem.geometry(fem.RefElement(2), lv.X[lv.elem_nodes])[0].sum(axis=1)
        crow = (lv.eidx[:, 1] >> (L - 1))
        got = np.bincount(crow, weights=dV, minlength=len(rows))
        errs.append(abs(got - expect).max())
    # converges to the closed form (the circle meets the wall with a vertical
    # tangent, so its rate is lower); a wrong height or blend would stall
    assert errs[-1] < (2e-3 if mapping == 1 else 1e-5)
    assert errs[-1] < errs[-2] / (1.5 if mapping == 1 else 4.0)


# --------------------------------------------------------------------------
# the disc cross-section map of the 3D tube (mapping 3) and the 3D outlet
# flux functional
# --------------------------------------------------------------------------
def _tube_cfg(levels=1, nc=(4, 4, 2), **kw):
    cfg = _region_cfg3(nc, (), levels=levels, **kw)
    cfg["breaks"] = ([0, 0.05, 0.5, 0.95, 1.0][:nc[0] + 1] if nc[0] == 4 else
                     list(np.linspace(0, 1, nc[0] + 1)),
                     [0, 0.05, 0.5, 0.95, 1.0][:nc[1] + 1] if nc[1] == 4 else
                     list(np.linspace(0, 1, nc[1] + 1)),
                     list(np.linspace(0, 0.6, nc[2] + 1)))
    cfg["mapping"] = 3
    cfg["map_params"] = [0.5, 0.5, 0.5]
    return cfg


def test_disc_map_section_area_closed_form():
    """The map sends the square section onto the disc of radius R: the
    isoparametric element volumes of one element layer converge to
    pi R^2 times the layer height (a wrong scale, centre or square-root
    factor would stall away from it)."""
    errs = []
    for L in (1, 2, 3):
        cfg = _tube_cfg(levels=L, nc=(4, 4, 1))
        cfg["breaks"] = (cfg["breaks"][0], cfg["breaks"][1], [0.0, 0.6])
        lv = Level(cfg, L - 1)
        dV = fem.geometry(fem.RefElement(3), lv.X[lv.elem_nodes])[0].sum(axis=1)
        errs.append(abs(dV.sum() - np.pi * 0.25 * 0.6))
    assert errs[-1] < 2e-4
    assert errs[-1] < errs[-2] / 8.0
    # the mapped elements are curved (the map is not affine)
    lv = Level(_tube_cfg(levels=1, nc=(4, 4, 1)), 0)
    Xe = lv.X[lv.elem_nodes]
    corners = Xe[:, [0, 2, 6, 8, 18, 20, 24, 26]].mean(axis=1)
    assert abs(Xe[:, 13] - corners).max() > 1e-4


def test_patch_disc_mapped_solid_3d():
    """Isoparametric Q2 on the disc-mapped tube reproduces fields linear in
    the physical coordinates: a constant-stress solid state leaves zero
    residual on interior test functions."""
    x, y, z = SYM
    cfg = _tube_cfg(levels=1, nc=(4, 4, 2), E=7.0, nu=0.3)
    cfg["region"] = np.ones_like(cfg["region"])
    lv = Level(cfg, 0)
    G, inv_lam = fem.lame_constants(cfg["E"], cfg["nu"])
    d = [0.3 * x - 0.7 * y + 0.1 * z, 0.2 * x + 0.5 * y, -0.4 * z + 0.1 * x]
    p = -(0.3 + 0.5 - 0.4) / inv_lam
    xv = _state(lv, d=d, ps=sy.Float(p))
    asm = fem.assemble_level(lv, cfg)
    r = asm["A"] @ xv
    inner = _interior_nodes(lv)
    assert inner.sum() > 0
    scale = abs(asm["A"]).max() * abs(xv).max()
    assert abs(_rows(lv, r, "d")[inner]).max() < 1e-11 * scale
    assert abs(_rows(lv, r, "ps")).max() < 1e-11 * scale
    d2 = [x * x, 0 * y, 0 * z]
    r2 = asm["A"] @ _state(lv, d=d2, ps=sy.Float(0.0))
    assert abs(_rows(lv, r2, "d")[inner]).max() > 1e-6 * scale


def test_outlet_flux_3d_closed_forms():
    """c^T x = int over the fluid part of the z-max face of u.n: with u
    constant along z it is the fluid section's area, with u_z = x the first
    moment, with tangential u zero; solid elements of the last layer do not
    count (a solid ring around the fluid)."""
    from oracle import adjoint
    x, y, z = SYM
    cfg = _region_cfg3((3, 4, 2), (0,), levels=1)
    cfg["breaks"] = ([0, 0.2, 0.7, 1.1], [0, 0.1, 0.4, 0.8, 1.0], [0, 0.3, 0.9])
    lv = Level(cfg, 0)
    c = adjoint.outlet_flux_vector(lv)
    y0, y1 = 0.1, 1.0                              # fluid rows (solid y-layer 0)
    area = 1.1 * (y1 - y0)
    assert c @ _state(lv, u=[0 * x, 0 * y, 1 + 0 * z]) == pytest.approx(area, rel=1e-13)
    assert c @ _state(lv, u=[0 * x, 0 * y, x]) == pytest.approx(0.5 * 1.1 ** 2 * (y1 - y0),
                                                                 rel=1e-13)
    assert c @ _state(lv, u=[1 + 0 * x, y, 0 * z]) == pytest.approx(0.0, abs=1e-14)
    # Q2 traces are exact for quadratic profiles: u_z = y^2 on the fluid rows
    assert c @ _state(lv, u=[0 * x, 0 * y, y * y]) == pytest.approx(
        1.1 * (y1 ** 3 - y0 ** 3) / 3, rel=1e-13)
    # on the disc-mapped tube the flux of u = e_z converges to the section area
    errs = []
    for L in (1, 2):
        cfg = _tube_cfg(levels=L, nc=(4, 4, 1))
        lv = Level(cfg, L - 1)
        c = adjoint.outlet_flux_vector(lv)
        errs.append(abs(c @ _state(lv, u=[0 * x, 0 * y, 1 + 0 * z]) - np.pi * 0.25))
    assert errs[-1] < 1e-3 and errs[-1] < errs[0]

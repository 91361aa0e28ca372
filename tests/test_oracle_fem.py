"""Pins of the oracle's finite-element layer against closed forms.

* 1D Q2 / Q1 Lagrange bases: nodal interpolation and the quarter-point
  weights (3/8, 3/4, -1/8) of the natural injection.
* the 3-point Gauss rule integrates polynomials up to degree 5 exactly.
* SUPG lambda_k of a square element of side h equals 55/h^2 (hand-derived
  from the element bubble, see test docstring).
* polynomial consistency (patch tests): for fields inside the discrete space
  whose strong residual vanishes, every assembled equation whose test
  function does not touch the boundary has zero residual.  This pins the
  solid (S, V), fluid (F, W, convection, SUPG), ALE (A) and interface
  routing (S rows collecting fluid stresses) terms entry by entry.
* manufactured solution for the mixed linear-elastic solid: L2 error rates
  ~3 (d, Q2) and ~2 (p, Q1).
* the lumped kinematic mass sums to the solid area per component.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sy

from oracle import fem
from oracle.mesh import Level
from tests.cfgs import small


def test_q2_q1_1d_bases():
    v, d, dd = fem.q2_1d(np.array([-1.0, 0.0, 1.0]))
    assert np.allclose(v, np.eye(3))
    v, _, _ = fem.q2_1d(np.array([-0.5, 0.5]))
    assert np.allclose(v[0], [3 / 8, 3 / 4, -1 / 8])
    assert np.allclose(v[1], [-1 / 8, 3 / 4, 3 / 8])
    xs = np.linspace(-1, 1, 7)
    v, d, dd = fem.q2_1d(xs)
    assert np.allclose(v.sum(1), 1.0) and np.allclose(d.sum(1), 0.0)
    assert np.allclose(v @ np.array([-1.0, 0.0, 1.0]), xs)          # reproduces x
    assert np.allclose(v @ np.array([1.0, 0.0, 1.0]), xs ** 2)      # reproduces x^2
    w, _ = fem.q1_1d(np.array([-1.0, 0.0, 1.0]))
    assert np.allclose(w, [[1, 0], [0.5, 0.5], [0, 1]])


def test_gauss_rule_degree_5():
    for k in range(6):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((fem.GAUSS_W * fem.GAUSS_PTS ** k).sum() - exact) < 1e-14
    k = 6
    assert abs((fem.GAUSS_W * fem.GAUSS_PTS ** k).sum() - 2.0 / 7) > 1e-3


@pytest.mark.parametrize("h", [1.0, 0.25, 0.03])
def test_supg_lambda_square_closed_form(h):
    """Bubble b = (1-xi^2)(1-eta^2) on a square of side h.  With v_a =
    lap(b) e_a + grad(d_a b), int v_a.v_b = delta_ab 2816/(9 h^2) and
    int |grad b|^2 = 256/45, so lambda_k = 55 / h^2."""
    cfg = small(nc=(1, 1), solid_rows=(), xb=[0, h], yb=[0, h])
    lv = Level(cfg, 0)
    ref = fem.RefElement(2)
    dV, G, H, _ = fem.geometry(ref, lv.X[lv.elem_nodes])
    lam = fem.supg_lambda(ref, dV, G, H)
    assert lam[0] == pytest.approx(55.0 / h ** 2, rel=1e-12)
    tau = fem.supg_tau(lam, np.array([[0.0, 1.0, 1e4]]), mu=2e-3, rho=1.0)
    nu = 2e-3
    expect = [1 / (4 * lam[0] * nu), min(1 / (4 * lam[0] * nu), 1 / np.sqrt(lam[0])),
              1 / (np.sqrt(lam[0]) * 1e4)]
    assert np.allclose(tau[0], expect)


def _interior_node_mask(lv):
    m = np.ones(lv.N2, bool)
    for a in range(lv.D):
        m &= (lv.nidx[:, a] > 0) & (lv.nidx[:, a] < lv.nn[a] - 1)
    return m


def _nodal(lv, fun):
    return np.stack(fun(lv.X[:, 0], lv.X[:, 1]), axis=1)


def _vertex_xy(lv, flags):
    nodes = lv.node_of_vertex(np.where(flags)[0])
    return lv.X[nodes, 0], lv.X[nodes, 1]


def _state(lv, d, u, ps, pf):
    x = np.zeros(lv.N)
    x[:2 * lv.N2] = d.ravel()
    x[lv.off_u:lv.off_u + 2 * lv.N2] = u.ravel()
    if lv.Nps:
        x[lv.off_ps:lv.off_ps + lv.Nps] = ps(*_vertex_xy(lv, lv.vert_solid))
    if lv.Npf:
        x[lv.off_pf:lv.off_pf + lv.Npf] = pf(*_vertex_xy(lv, lv.vert_fluid))
    return x


def test_patch_linear_elastic_solid():
    E, nu = 7.0, 0.3
    G, inv_lam = fem.lame_constants(E, nu)
    lamL = 1.0 / inv_lam
    cfg = small(nc=(3, 4), solid_rows=(0, 1, 2, 3), E=E, nu=nu,
                xb=[0, 0.2, 0.7, 1.0], yb=[0, 0.1, 0.5, 0.6, 1.0])
    lv = Level(cfg, 0)
    d = _nodal(lv, lambda x, y: (x * x + 2 * x * y - y * y, 3 * x * x - x * y + 2 * y * y))
    # div d = 2x + 2y - x + 4y = x + 6y ; p = -lambda div d
    ps = lambda x, y: -lamL * (x + 6 * y)
    # f = -[(lambda+G) grad div d + G lap d], grad div d = (1, 6), lap d = (0, 10)
    fx, fy = -((lamL + G) * 1.0 + G * 0.0), -((lamL + G) * 6.0 + G * 10.0)
    x = _state(lv, d, np.zeros_like(d), ps, None)
    asm = fem.assemble_level(lv, cfg)
    f = np.tile([fx, fy], (lv.N2, 1))
    r = asm["A"] @ x - fem.load_vector(lv, cfg, f)
    inner = _interior_node_mask(lv)
    rd = r[:2 * lv.N2].reshape(-1, 2)[inner]
    scale = abs(asm["A"]).max() * abs(x).max()
    assert abs(rd).max() < 1e-12 * scale
    assert abs(r[lv.off_ps:lv.off_ps + lv.Nps]).max() < 1e-12 * scale
    # the test is sharp: a wrong shear modulus breaks it
    cfg2 = dict(cfg, E=E * 1.01)
    r2 = fem.assemble_level(lv, cfg2)["A"] @ x - fem.load_vector(lv, cfg, f)
    assert abs(r2[:2 * lv.N2].reshape(-1, 2)[inner]).max() > 1e-6 * scale


def test_patch_oseen_supg_and_ale():
    mu, rho = 0.05, 1.3
    wx, wy = 0.3, -0.2
    cfg = small(nc=(4, 3), solid_rows=(), mu=mu, rho=rho, supg=True, ale_k=1,
                xb=[0, 0.3, 0.5, 0.8, 1.0], yb=[0, 0.25, 0.7, 1.0])
    lv = Level(cfg, 0)
    u = _nodal(lv, lambda x, y: (y * y + x * y, x * x - 0.5 * y * y))   # div u = 0
    d = _nodal(lv, lambda x, y: (x * x - y * y, -2 * x * y))           # lap d = 0, div d = 0
    pf = lambda x, y: x + 2 * y
    w = np.tile([wx, wy], (lv.N2, 1))
    # f = (w.grad) u - mu lap u + grad p  (div u = 0), divided by rho
    fun_f = lambda x, y: ((rho * (wx * y + wy * (2 * y + x)) - mu * 2.0 + 1.0) / rho,
                          (rho * (wx * 2 * x + wy * (-y)) - mu * 1.0 + 2.0) / rho)
    f = _nodal(lv, fun_f)
    x = _state(lv, d, u, None, pf)
    asm = fem.assemble_level(lv, cfg, w)
    assert asm["tau"] is not None
    r = asm["A"] @ x - fem.load_vector(lv, cfg, f, w, asm["tau"])
    inner = _interior_node_mask(lv)
    scale = abs(asm["A"]).max() * abs(x).max()
    ru = r[lv.off_u:lv.off_u + 2 * lv.N2].reshape(-1, 2)[inner]
    rA = r[:2 * lv.N2].reshape(-1, 2)[inner]
    rW = r[lv.off_pf:]
    assert abs(ru).max() < 1e-11 * scale
    assert abs(rA).max() < 1e-11 * scale
    assert abs(rW).max() < 1e-11 * scale
    # sharpness: dropping SUPG changes the fluid rows only through tau-terms,
    # which vanish for the exact solution; a wrong viscosity does not.
    r2 = (fem.assemble_level(lv, dict(cfg, mu=mu * 1.1), w)["A"] @ x
          - fem.load_vector(lv, cfg, f, w, asm["tau"]))
    assert abs(r2[lv.off_u:lv.off_u + 2 * lv.N2].reshape(-1, 2)[inner]).max() > 1e-6 * scale


def test_patch_interface_traction_routing():
    """Uniform shear: d = (a y, 0) in the solid, u = (b y, 0) in the fluid with
    G a = mu b, no pressure, no load.  Both stresses equal, so the solid-side
    momentum rows (including interface nodes, which collect the fluid stress
    through the fluid elements) and the fluid rows have zero residual."""
    E, nu, mu = 10.0, 0.3, 0.2
    G, _ = fem.lame_constants(E, nu)
    a = 0.7
    b = G * a / mu
    cfg = small(nc=(4, 4), solid_rows=(0,), E=E, nu=nu, mu=mu,
                yb=[0, 0.15, 0.5, 0.8, 1.0])
    lv = Level(cfg, 0)
    d = _nodal(lv, lambda x, y: (a * y, 0 * y))
    u = _nodal(lv, lambda x, y: (b * y, 0 * y))
    x = _state(lv, d, u, lambda x, y: 0 * x, lambda x, y: 0 * x)
    asm = fem.assemble_level(lv, cfg)
    r = asm["A"] @ x
    inner = _interior_node_mask(lv)
    scale = abs(asm["A"]).max() * abs(x).max()
    iface = lv.solid_side & lv.fluid_touch & inner
    assert iface.sum() > 0
    rS = r[:2 * lv.N2].reshape(-1, 2)
    assert abs(rS[lv.solid_side & inner]).max() < 1e-12 * scale
    rF = r[lv.off_u:lv.off_u + 2 * lv.N2].reshape(-1, 2)
    assert abs(rF[~lv.solid_side & inner]).max() < 1e-12 * scale
    # without the fluid stress on interface rows the residual is G a * length
    x2 = _state(lv, d, 0 * u, lambda x, y: 0 * x, lambda x, y: 0 * x)
    r2 = (asm["A"] @ x2)[:2 * lv.N2].reshape(-1, 2)
    assert abs(r2[iface]).max() > 1e-3 * G * a


def test_lumped_kinematic_mass_area():
    cfg = small(nc=(4, 4), solid_rows=(0, 1), yb=[0, 0.1, 0.3, 0.6, 1.0])
    lv = Level(cfg, 0)
    A = fem.assemble_level(lv, cfg)["A"].tocsr()
    rows = lv.u(np.where(lv.solid_side)[0], 0)
    sub = A[rows][:, lv.off_u:lv.off_u + 2 * lv.N2]
    assert sub.nnz == len(rows)                       # diagonal only
    diag = A.diagonal()[rows]
    assert np.all(diag > 0)
    assert diag.sum() == pytest.approx(0.3, rel=1e-13)  # solid area


@pytest.mark.parametrize("dummy", [0])
def test_mms_elastic_rates(dummy):
    X, Y = sy.symbols("x y")
    E, nu = 5.0, 0.3
    G, inv_lam = fem.lame_constants(E, nu)
    lamL = 1.0 / inv_lam
    dx = sy.sin(sy.pi * X) * sy.sin(sy.pi * Y)
    dy = 4 * X * (1 - X) * Y * (1 - Y) * sy.exp(X)
    div = sy.diff(dx, X) + sy.diff(dy, Y)
    fx = -((lamL + G) * sy.diff(div, X) + G * (sy.diff(dx, X, 2) + sy.diff(dx, Y, 2)))
    fy = -((lamL + G) * sy.diff(div, Y) + G * (sy.diff(dy, X, 2) + sy.diff(dy, Y, 2)))
    p = -lamL * div
    F = sy.lambdify((X, Y), [fx, fy], "numpy")
    Dx = sy.lambdify((X, Y), [dx, dy], "numpy")
    Pf = sy.lambdify((X, Y), p, "numpy")
    errs_d, errs_p = [], []
    for L in (2, 3, 4):
        cfg = small(nc=(2, 2), solid_rows=(0, 1), levels=L, E=E, nu=nu)
        for f_ in range(4):
            cfg["bc_d"][f_][1] = 1
        lv = Level(cfg, L - 1)
        asm = fem.assemble_level(lv, cfg)
        fn = np.stack([np.broadcast_to(v, lv.X[:, 0].shape)
                       for v in F(lv.X[:, 0], lv.X[:, 1])], 1)
        b = fem.dirichlet_rhs(lv, asm["A"], fem.load_vector(lv, cfg, fn))
        x = spla.spsolve(fem.dirichlet_reduce(lv, asm["A"]).tocsc(), b)
        ref = fem.RefElement(2)
        dV, _, _, _ = fem.geometry(ref, lv.X[lv.elem_nodes])
        xq = np.einsum("qa,eai->eqi", ref.phi, lv.X[lv.elem_nodes])
        dh = x[:2 * lv.N2].reshape(-1, 2)[lv.elem_nodes]
        dq = np.einsum("qa,eai->eqi", ref.phi, dh)
        ex = np.stack(Dx(xq[..., 0], xq[..., 1]), -1)
        errs_d.append(np.sqrt((dV[..., None] * (dq - ex) ** 2).sum()))
        ph = x[lv.ps_of_vert[lv.elem_verts]]
        pq = np.einsum("qm,em->eq", ref.psi, ph)
        errs_p.append(np.sqrt((dV * (pq - Pf(xq[..., 0], xq[..., 1])) ** 2).sum()))
    rd = np.log2(np.array(errs_d[:-1]) / np.array(errs_d[1:]))
    rp = np.log2(np.array(errs_p[:-1]) / np.array(errs_p[1:]))
    assert rd[-1] > 2.8, rd
    assert rp[-1] > 1.8, rp

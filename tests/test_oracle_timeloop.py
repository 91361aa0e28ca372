"""Pins of the oracle's time stepping (oracle/timeloop.py): the time operator
against the difference of two assemblies, the steady state as a fixed point
of a backward-Euler step, the inflow factor, the linearity of one step in the
Dirichlet data, the Picard fixed point and the period statistics of
Section 4."""
import numpy as np
import pytest

from oracle import fem
from oracle.direct import direct_solve
from oracle.mesh import hierarchy_levels
from oracle.multigrid import Hierarchy
from oracle.timeloop import (inflow_scale, period, period_statistics, step_rhs,
                             velocity_field)
from paper_1909_13201_amd import inputs


def _cfg(levels=2, dt=1.0 / 32.0):
    cfg = inputs.with_levels(inputs.config("c5"), levels)
    cfg["dt"] = dt
    return cfg


def test_inflow_scale_closed_form():
    assert inflow_scale(0.0) == pytest.approx(1.0, abs=1e-15)
    assert inflow_scale(0.25) == pytest.approx(1.75, abs=1e-15)
    assert inflow_scale(0.75) == pytest.approx(0.25, abs=1e-15)
    assert inflow_scale(1.0) == pytest.approx(1.0, abs=1e-14)
    assert inflow_scale(0.25, amp=0.0) == 1.0


def test_velocity_field_is_the_u_block_node_major():
    lv = hierarchy_levels(_cfg())[-1]
    w = np.random.default_rng(1).standard_normal((lv.N2, lv.D))
    x = np.zeros(lv.N)
    for n in range(lv.N2):
        for c in range(lv.D):
            x[lv.off_u + lv.D * n + c] = w[n, c]
    assert np.array_equal(velocity_field(lv, x), w)


@pytest.mark.parametrize("supg", [False, True])
def test_time_operator_is_the_part_carrying_one_over_dt(supg):
    """T = A(dt) - A(inf) up to the rounding of the two assemblies, and it
    scales with 1/dt (every term of it carries 1/dt once)."""
    cfg = _cfg()
    cfg["supg"] = supg
    lv = hierarchy_levels(cfg)[-1]
    w = inputs.advecting_field(inputs.with_levels(inputs.config("c5"), 2))
    a = fem.assemble_level(lv, cfg, w)
    steady = dict(cfg, dt=np.inf)
    b = fem.assemble_level(lv, steady, w, a["tau"])
    D = (a["A"] - b["A"]).tocsr()
    scale = abs(a["A"]).max()
    assert abs(D - a["T"]).max() <= 1e-14 * scale
    assert abs(a["T"]).max() > 1e-6 * scale           # not trivially empty
    assert b["T"].nnz == 0
    half = fem.assemble_level(lv, dict(cfg, dt=2 * cfg["dt"]), w, a["tau"])
    assert abs(2 * half["T"] - a["T"]).max() <= 1e-13 * abs(a["T"]).max()


def test_steady_state_is_a_fixed_point_of_a_step():
    """With constant inflow, a backward-Euler step from the steady solution of
    the same (frozen-w) problem returns that solution."""
    cfg = _cfg()
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    Hs = Hierarchy(dict(cfg, dt=np.inf), w_finest=w, build_smoothers=False)
    xs = direct_solve(Hs.A[-1], Hs.rhs(f))
    Ht = Hierarchy(cfg, w_finest=w, taus=[p["tau"] for p in Hs.parts], build_smoothers=False)
    x1 = direct_solve(Ht.A[-1], step_rhs(Ht, f, 1.0, xs))
    assert np.linalg.norm(x1 - xs) <= 1e-9 * np.linalg.norm(xs)
    # and the step moves a state that is not steady
    x0 = 0.5 * xs
    x2 = direct_solve(Ht.A[-1], step_rhs(Ht, f, 1.0, x0))
    assert np.linalg.norm(x2 - x0) > 1e-3 * np.linalg.norm(xs)


def test_step_is_linear_in_the_dirichlet_factor():
    cfg = _cfg()
    w = inputs.advecting_field(cfg)
    H = Hierarchy(cfg, w_finest=w, build_smoothers=False)
    lv = H.finest
    zf = np.zeros((lv.N2, lv.D))
    z = np.zeros(lv.N)
    b1 = step_rhs(H, zf, 1.0, z)
    b3 = step_rhs(H, zf, 1.75, z)
    assert np.abs(b3 - 1.75 * b1).max() <= 1e-13 * np.abs(b1).max()
    assert np.abs(b1).max() > 0
    # Dirichlet rows carry the scaled data, free rows the lift -A_fD g u_D
    g = np.where(lv.dir_mask, lv.dir_val, 0.0)
    assert np.array_equal(b1[lv.dir_mask], g[lv.dir_mask])
    ref = -(H.A_full[-1] @ g)
    assert np.abs(b1[~lv.dir_mask] - ref[~lv.dir_mask]).max() <= 1e-13 * np.abs(ref).max()


def test_picard_converges_to_a_fixed_point():
    """After the Picard loop has converged, the last iterate solves the
    system assembled about its own velocity."""
    cfg = _cfg()
    f = inputs.body_force(cfg)
    x, recs, states = period(cfg, f, steps=2, picard_max=12, picard_tol=1e-10)
    assert len(states) == 2
    last = [r for r in recs if r["step"] == 2]
    assert last[-1]["change"] <= 1e-10 and len(last) < 12
    changes = [r["change"] for r in last]
    assert all(b < a for a, b in zip(changes, changes[1:]))   # contracting
    lvf = hierarchy_levels(cfg)[-1]
    H = Hierarchy(cfg, w_finest=velocity_field(lvf, x), build_smoothers=False)
    b = step_rhs(H, f, inflow_scale(2 * cfg["dt"]), states[0])
    r = H.A[-1] @ x - b
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)


def test_fgmres_period_matches_direct_period():
    cfg = _cfg()
    f = inputs.body_force(cfg)
    xd, rd, sd = period(cfg, f, steps=3, picard_max=2)
    xg, rg, sg = period(cfg, f, steps=3, picard_max=2, solver="fgmres")
    for a, b in zip(sd, sg):
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(a)
    st = period_statistics(rg, 3)
    assert st["solves"] == 6 and st["s_max"] == 2.0
    assert 1 <= st["N"] <= 30 and 0 < st["rho"] < 1


def test_period_statistics_by_hand():
    recs = [dict(step=1, s=1, iters=10, rate=0.1, change=1.0),
            dict(step=1, s=2, iters=8, rate=0.2, change=0.1),
            dict(step=2, s=1, iters=6, rate=0.3, change=1.0)]
    st = period_statistics(recs, 2)
    assert st["N"] == pytest.approx(8.0)
    assert st["rho"] == pytest.approx(0.2)
    assert st["s_max"] == pytest.approx(1.5)
    assert st["solves"] == 3


def _momentum_rows(lv):
    """Rows of the momentum balance: d rows of solid-side nodes (the solid
    momentum equation sits on d) and u rows of the other nodes."""
    m = np.zeros(lv.N, bool)
    ss = np.asarray(lv.solid_side, bool)
    for c in range(lv.D):
        m[lv.D * np.arange(lv.N2) + c] = ss
        m[lv.off_u + lv.D * np.arange(lv.N2) + c] = ~ss
    return m


@pytest.mark.parametrize("theta", [0.5, 0.7])
def test_theta_scheme_operators(theta):
    """A_theta = T + theta A_inf on the momentum rows (A_inf elsewhere) and
    Tx = T - (1 - theta) A_inf on the momentum rows, A_inf assembled
    separately without dt."""
    import scipy.sparse as sp
    cfg = dict(_cfg(), theta=theta)
    lv = hierarchy_levels(cfg)[-1]
    w = inputs.advecting_field(inputs.with_levels(inputs.config("c5"), 2))
    a = fem.assemble_level(lv, cfg, w)
    b = fem.assemble_level(lv, dict(cfg, dt=np.inf, theta=1.0), w, a["tau"])
    m = _momentum_rows(lv)
    S = sp.diags(np.where(m, theta, 1.0))
    Mm = sp.diags(m.astype(float))
    scale = abs(a["A"]).max()
    assert abs(a["A"] - a["T"] - S @ b["A"]).max() <= 1e-13 * scale
    assert abs(a["Tx"] - (a["T"] - (1 - theta) * (Mm @ b["A"]))).max() <= 1e-13 * scale
    # theta = 1 is backward Euler: the same operator and Tx = T
    one = fem.assemble_level(lv, dict(cfg, theta=1.0), w, a["tau"])
    ref = fem.assemble_level(lv, {k: v for k, v in cfg.items() if k != "theta"}, w, a["tau"])
    assert abs(one["A"] - ref["A"]).max() == 0 and abs(one["Tx"] - one["T"]).max() == 0


def test_theta_steady_state_is_a_fixed_point():
    cfg = dict(_cfg(), theta=0.5)
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    Hs = Hierarchy(dict(cfg, dt=np.inf, theta=1.0), w_finest=w, build_smoothers=False)
    xs = direct_solve(Hs.A[-1], Hs.rhs(f))
    Ht = Hierarchy(cfg, w_finest=w, taus=[p["tau"] for p in Hs.parts], build_smoothers=False)
    x1 = direct_solve(Ht.A[-1], step_rhs(Ht, f, 1.0, xs))
    assert np.linalg.norm(x1 - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("theta,order", [(1.0, 1), (0.5, 2)])
def test_theta_scheme_convergence_order(theta, order):
    """A channel without solid (Stokes, parabolic inflow scaled by the
    pulsatile factor, from the steady state at t = 0): successive
    differences of the velocity at t = 1/4 for dt = 1/16 ... 1/128 shrink
    by 2 (backward Euler) or 4 (Crank-Nicolson)."""
    import scipy.sparse.linalg as spla
    from tests.cfgs import small
    cfg0 = small(nc=(4, 4), solid_rows=(), levels=1,
                 bc_u=[[2, 0], [0, 0], [1, 0], [1, 0], [0, 0], [0, 0]], bc_d=[[1, 0]] * 6)
    Hs = Hierarchy(dict(cfg0, dt=np.inf), None, build_smoothers=False)
    lv = Hs.finest
    f = np.zeros((lv.N2, lv.D))
    x0 = direct_solve(Hs.A[-1], Hs.rhs(f))
    us = []
    for dt in (1 / 16, 1 / 32, 1 / 64, 1 / 128):
        H = Hierarchy(dict(cfg0, dt=dt, theta=theta), None, build_smoothers=False)
        lu = spla.splu(H.A[-1].tocsc())
        x = x0
        for i in range(1, int(round(0.25 / dt)) + 1):
            x = lu.solve(step_rhs(H, f, inflow_scale(i * dt), x))
        us.append(x[lv.off_u:lv.off_pf])
    e = [np.linalg.norm(us[k] - us[k + 1]) for k in range(3)]
    ratios = [e[k] / e[k + 1] for k in range(2)]
    assert all(abs(r - 2 ** order) < 0.35 * 2 ** order for r in ratios), ratios

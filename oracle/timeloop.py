"""Time stepping of the linearized FSI system (TEST INFRASTRUCTURE ONLY:
imported by tests/, the smoke check and the bench's CPU baseline, never by
the library's product path).

The paper integrates the monolithic system of Section 2.2 in time (a
backward difference for the time derivatives in the integrands, Crank-
Nicolson for the momentum balance) and solves every time step by Newton's
method, each Newton step by the preconditioned GMRES of Section 3; Section 4
reports, per period of 1 s with t_step time steps, the mean number of
nonlinear steps per time step (s^max), the mean GMRES iterations per linear
solve (N) and the mean convergence rate (rho).

Readings (the linearization here is Oseen about a frozen advecting
velocity, solid linearized at the stress-free state):
* the time derivatives by backward differences with step dt = cfg["dt"];
  the steady terms of the momentum rows carry the weight theta =
  cfg["theta"] (1, the default, is backward Euler throughout; 1/2 is
  Crank-Nicolson for the momentum balance, as the paper uses it), the
  assembled operator A carries the implicit part and Tx = T - (1 - theta) M
  the explicit one (T the terms that multiply 1/dt, M the steady momentum-
  row terms), so one step solves
      A x_n = F L f + Tx x_{n-1}
  on the free rows, x_n = g(t_n) u_D on the Dirichlet rows;
* the nonlinear steps are Picard (fixed-point) steps on the advecting
  velocity: step s of time step n assembles every level about w = the
  velocity of the latest iterate (w = u(x_{n-1}) for s = 1) and solves the
  linear system above; the loop ends after picard_max steps or once
  ||x_s - x_{s-1}|| <= picard_tol ||x_s||;
* the inflow is pulsatile with the 2D aneurysm's profile of Section 4.1:
  the Dirichlet data scale by g(t) = 1 + amp sin(2 pi t), amp = 0.75, so
  every nonzero prescribed value (the parabolic inflow) follows g;
* rho_{i,s} is quoted per iteration, (r_N / r_0)^(1 / N), with r the true
  residual of the solve started from x = 0 (r_0 = ||b||).
"""
from __future__ import annotations

import numpy as np

from . import fem
from .direct import direct_solve
from .krylov import fgmres
from .mesh import hierarchy_levels
from .multigrid import Hierarchy


def inflow_scale(t: float, amp: float = 0.75) -> float:
    """Pulsatile factor of the inflow profile (Section 4.1, period 1 s)."""
    return 1.0 + amp * np.sin(2.0 * np.pi * t)


def velocity_field(lv, x: np.ndarray) -> np.ndarray:
    """The velocity part of a level vector as nodal (N2, D) values."""
    return np.asarray(x[lv.off_u: lv.off_u + lv.D * lv.N2]).reshape(lv.N2, lv.D)


def step_rhs(H: Hierarchy, fnodal: np.ndarray, g: float, x_prev: np.ndarray) -> np.ndarray:
    """Right-hand side of one backward-Euler step at inflow factor g: on the
    free rows the load, the lift of the scaled Dirichlet data through the
    unreduced operator and the time operator applied to the previous state;
    on the Dirichlet rows the scaled data."""
    lv = H.finest
    asm = H.parts[-1]
    b_raw = fem.load_vector(lv, H.cfg, fnodal, H.w_finest, asm["tau"])
    gD = np.where(lv.dir_mask, g * lv.dir_val, 0.0)
    b = b_raw - H.A_full[-1] @ gD + asm["Tx"] @ x_prev
    return np.where(lv.dir_mask, gD, b)


def period(cfg: dict, fnodal: np.ndarray, steps: int, picard_max: int = 1,
           picard_tol: float = 0.0, amp: float = 0.75, t0: float = 0.0,
           x0: np.ndarray | None = None, solver: str = "direct", rtol: float = 1e-10,
           restart: int = 30):
    """Run `steps` time steps from x0 (zeros by default) at t0.  solver:
    "direct" (refined LU, the reference solution of every linear system) or
    "fgmres" (the paper's GMRES preconditioned by the FS-AS V-cycle).
    Returns (x, records, states): one record per linear solve (step i,
    nonlinear step s, iterations, rate, relative change), states[i] = x_i."""
    dt = float(cfg["dt"])
    if not np.isfinite(dt) or dt <= 0:
        raise ValueError("time stepping needs a finite dt > 0")
    lvf = hierarchy_levels(cfg)[-1]
    x_prev = np.zeros(lvf.N) if x0 is None else np.array(x0, dtype=np.float64)
    records, states = [], []
    for i in range(1, steps + 1):
        g = inflow_scale(t0 + i * dt, amp)
        x_cur = x_prev
        for s in range(1, picard_max + 1):
            H = Hierarchy(cfg, w_finest=velocity_field(lvf, x_cur),
                          build_smoothers=(solver == "fgmres"))
            b = step_rhs(H, fnodal, g, x_prev)
            if solver == "direct":
                x_new = direct_solve(H.A[-1], b)
                iters, rate = 0, float("nan")
            else:
                A = H.A[-1]
                x_new, info = fgmres(lambda v: A @ v, H.vcycle, b, restart=restart, rtol=rtol)
                if not info["converged"]:
                    raise RuntimeError(f"step {i}, nonlinear step {s}: FGMRES did not converge")
                iters = info["iters"]
                rate = info["rel_res_true"] ** (1.0 / iters) if iters else 0.0
            change = float(np.linalg.norm(x_new - x_cur) / max(np.linalg.norm(x_new), 1e-300))
            records.append(dict(step=i, s=s, iters=iters, rate=rate, change=change))
            x_cur = x_new
            if picard_tol > 0 and change <= picard_tol:
                break
        x_prev = x_cur
        states.append(x_prev.copy())
    return x_prev, records, states


def period_statistics(records: list, steps: int) -> dict:
    """N, rho and s^max of Section 4 over the records of `steps` time steps."""
    n = len(records)
    return dict(N=sum(r["iters"] for r in records) / n,
                rho=sum(r["rate"] for r in records) / n,
                s_max=n / steps, solves=n)

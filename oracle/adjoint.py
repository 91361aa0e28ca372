"""Adjoint solve and parameter gradients of a linear functional (oracle).

For the reduced system A(theta) x = b(theta) (Dirichlet rows eliminated
symmetrically, so x already carries the Dirichlet values) and J = c^T x:

* adjoint: A^T lambda = c, solved by FGMRES preconditioned with the
  transposed V-cycle M^{-T};
* dJ/db = lambda;
* dJ/dtheta = -(F lambda)^T (dA_full/dtheta) x, where F zeroes Dirichlet
  entries and A_full is the unreduced operator; this includes the
  dependence of the Dirichlet lift on theta.  theta in {E, mu}; the SUPG
  parameter tau is held fixed (the operator is affine in G, 1/lambda_L, mu).

The functional used for the differentiation workload is the outlet flux
J = int_{outlet, fluid} u.n ds (the flux definition of Section 4.1), exact
Gauss quadrature of the Q2 trace.
"""
from __future__ import annotations

import numpy as np

from .fem import GAUSS_PTS, GAUSS_W, q2_1d
from .krylov import fgmres
from .mesh import Level


def outlet_flux_vector(lv: Level) -> np.ndarray:
    """c with c^T x = int over the fluid part of the outlet face of u.n ds:
    the x-max face in 2D, the z-max face in 3D (the tube's axis)."""
    if lv.D == 3:
        return _outlet_flux_vector_3d(lv)
    c = np.zeros(lv.N)
    nx, ny = lv.ne
    L, dL, _ = q2_1d(GAUSS_PTS)
    for ey in range(ny):
        e = (nx - 1) + nx * ey
        if lv.region[e] != 0:
            continue
        # face nodes: local x index 2, local y index 0..2
        nodes = lv.elem_nodes[e][[2, 5, 8]]
        X = lv.X[nodes]                                   # (3, 2)
        for q in range(3):
            t = dL[q] @ X                                 # dX/deta at the point
            for a in range(3):
                wphi = GAUSS_W[q] * L[q, a]
                c[lv.u(nodes[a], 0)] += wphi * t[1]
                c[lv.u(nodes[a], 1)] += -wphi * t[0]
    return c


def _outlet_flux_vector_3d(lv: Level) -> np.ndarray:
    """The z-max face of every fluid element of the last element layer: the
    face's 3 x 3 Q2 trace nodes (local z index 2), 3 x 3 Gauss points, and
    n dS = (dX/dxi x dX/deta) dxi deta on the face parametrized by the
    element's reference (xi, eta), which points along +z (outward)."""
    c = np.zeros(lv.N)
    nx, ny, nz = lv.ne
    L, dL, _ = q2_1d(GAUSS_PTS)
    for ey in range(ny):
        for ex in range(nx):
            e = ex + nx * (ey + ny * (nz - 1))
            if lv.region[e] != 0:
                continue
            # local node (a, b, 2) with a, b in 0..2, x fastest
            loc = np.array([a + 3 * b + 18 for b in range(3) for a in range(3)])
            nodes = lv.elem_nodes[e][loc]
            X = lv.X[nodes].reshape(3, 3, 3)              # (b, a, xyz)
            for qa in range(3):
                for qb in range(3):
                    t1 = np.einsum("a,bac->c", dL[qa], X * L[qb][:, None, None])
                    t2 = np.einsum("b,bac->c", dL[qb], X * L[qa][None, :, None])
                    n = np.cross(t1, t2)
                    wq = GAUSS_W[qa] * GAUSS_W[qb]
                    for b in range(3):
                        for a in range(3):
                            phi = wq * L[qa, a] * L[qb, b]
                            node = nodes[a + 3 * b]
                            for comp in range(3):
                                c[lv.u(node, comp)] += phi * n[comp]
    return c


def parameter_derivatives(parts: dict, E: float, nu: float):
    """dA_full/dE and dA_full/dmu from the affine pieces."""
    dG_dE = 1.0 / (2.0 * (1.0 + nu))
    dinv_dE = 0.0 if nu >= 0.5 else -(1.0 + nu) * (1.0 - 2.0 * nu) / (nu * E * E)
    dA_dE = dG_dE * parts["AG"] + dinv_dE * parts["AC"]
    dA_dmu = parts["Amu"]
    return dA_dE, dA_dmu


def adjoint_solve(H, c, rtol=1e-10, restart=30, max_restarts=20):
    A = H.A[-1]
    return fgmres(lambda v: A.T @ v, lambda v: H.vcycle(v, transpose=True), c,
                  restart=restart, rtol=rtol, max_restarts=max_restarts)


def gradients(H, x: np.ndarray, lam: np.ndarray):
    """(dJ/dE, dJ/dmu) for J = c^T x given the forward x and adjoint lambda."""
    lv = H.finest
    cfg = H.cfg
    dA_dE, dA_dmu = parameter_derivatives(H.parts[-1], cfg["E"], cfg["nu"])
    lf = np.where(lv.free, lam, 0.0)
    return -lf @ (dA_dE @ x), -lf @ (dA_dmu @ x)

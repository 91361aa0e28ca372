"""Prolongation and equation-routed restriction (paper Section 3.3).

P_{l,l-1} is the natural injection of the coarse Q2 x Q2 x Q1 space into the
fine one: componentwise Q2 interpolation for d and u, Q1 interpolation inside
each region for p^s and p^f.  In the J2 ordering it is block lower
triangular (P_{d^f,d^s} and P_{u^f,u^s} present, P_{d^s,d^f} = 0).

The restriction is NOT P^T.  Its blocks are R_SS = R_KK = P_{d^s d^s}^T,
R_AA = R_FF = P_{d^f d^f}^T, R_VV = P_{p^s p^s}^T, R_WW = P_{p^f p^f}^T and
R_SF = P_{d^f,d^s}^T, and the transpose of P_{u^f,u^s} appears nowhere: the
coarse solid/interface momentum row collects the fine solid momentum rows
(S) and the fine fluid momentum rows (F), while the coarse kinematic row K
collects only fine K rows and the coarse ALE row A only fine A rows.

Coarse Dirichlet rows of the restricted residual are zeroed and fine
Dirichlet entries of a prolonged correction are zeroed (the masked operators
D_c R and D_f P are what the V-cycle applies).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import q2_1d, q1_1d
from .mesh import Level


def _interp_1d(n_coarse_el: int, quadratic: bool) -> sp.csr_matrix:
    """1D interpolation from a coarse line of n elements to its midpoint refinement."""
    if quadratic:
        nf, nc, per = 4 * n_coarse_el + 1, 2 * n_coarse_el + 1, 4
    else:
        nf, nc, per = 2 * n_coarse_el + 1, n_coarse_el + 1, 2
    rows, cols, vals = [], [], []
    for k in range(nf):
        c = min(k // per, n_coarse_el - 1)
        if quadratic:
            xi = (k - 4 * c) / 2.0 - 1.0
            w = q2_1d(np.array([xi]))[0][0]
            base = 2 * c
        else:
            xi = float(k - 2 * c) - 1.0
            w = q1_1d(np.array([xi]))[0][0]
            base = c
        for j, wj in enumerate(w):
            if wj != 0.0:
                rows.append(k)
                cols.append(base + j)
                vals.append(wj)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def _kron_axes(mats):
    """Kronecker product for x-fastest numbering: kron(M_z, M_y, M_x)."""
    out = mats[0]
    for M in mats[1:]:
        out = sp.kron(M, out, format="csr")
    return out


def node_interpolation(fine: Level, coarse: Level) -> sp.csr_matrix:
    """Scalar Q2 node interpolation matrix (N2_fine x N2_coarse)."""
    return _kron_axes([_interp_1d(n, True) for n in coarse.ne]).tocsr()


def vertex_interpolation(fine: Level, coarse: Level) -> sp.csr_matrix:
    return _kron_axes([_interp_1d(n, False) for n in coarse.ne]).tocsr()


def prolongation(fine: Level, coarse: Level, masked: bool = True) -> sp.csr_matrix:
    """Full P_{l,l-1} in the level layout (fine N x coarse N)."""
    D = fine.D
    Pn = node_interpolation(fine, coarse)
    Pv = vertex_interpolation(fine, coarse)
    PnD = sp.kron(Pn, sp.identity(D), format="csr")
    # pressures: rows of fine region vertices, columns of coarse region vertices
    Pps = Pv[fine.vert_solid][:, coarse.vert_solid]
    Ppf = Pv[fine.vert_fluid][:, coarse.vert_fluid]
    # every weight of a region vertex must land on a coarse vertex of that region
    assert np.allclose(abs(Pv[fine.vert_solid]).sum(axis=1).A1, abs(Pps).sum(axis=1).A1)
    assert np.allclose(abs(Pv[fine.vert_fluid]).sum(axis=1).A1, abs(Ppf).sum(axis=1).A1)
    P = sp.block_diag([PnD, Pps, PnD, Ppf], format="csr")
    if masked:
        P = sp.diags(fine.free.astype(np.float64)) @ P
    return P.tocsr()


def restriction(fine: Level, coarse: Level, masked: bool = True) -> sp.csr_matrix:
    """Equation-routed R_{l-1,l} (coarse N x fine N) in the level layout."""
    D = fine.D
    Pn = node_interpolation(fine, coarse)
    Pv = vertex_interpolation(fine, coarse)
    PnT = Pn.T.tocsr()
    Sc = sp.diags(coarse.solid_side.astype(np.float64))
    Fc = sp.diags((~coarse.solid_side).astype(np.float64))
    Sf = sp.diags(fine.solid_side.astype(np.float64))
    Ff = sp.diags((~fine.solid_side).astype(np.float64))
    I = sp.identity(D)
    R_dd = sp.kron(Sc @ PnT @ Sf + Fc @ PnT @ Ff, I)      # R_SS (+) R_AA
    R_du = sp.kron(Sc @ PnT @ Ff, I)                      # R_SF: coarse S <- fine F
    R_uu = sp.kron(Sc @ PnT @ Sf + Fc @ PnT @ Ff, I)      # R_KK (+) R_FF
    R_ps = Pv[fine.vert_solid][:, coarse.vert_solid].T
    R_pf = Pv[fine.vert_fluid][:, coarse.vert_fluid].T
    Nc2, Nf2 = coarse.N2 * D, fine.N2 * D
    Z = lambda m, n: sp.csr_matrix((m, n))
    R = sp.bmat([
        [R_dd, Z(Nc2, fine.Nps), R_du, Z(Nc2, fine.Npf)],
        [Z(coarse.Nps, Nf2), R_ps, Z(coarse.Nps, Nf2), Z(coarse.Nps, fine.Npf)],
        [Z(Nc2, Nf2), Z(Nc2, fine.Nps), R_uu, Z(Nc2, fine.Npf)],
        [Z(coarse.Npf, Nf2), Z(coarse.Npf, fine.Nps), Z(coarse.Npf, Nf2), R_pf],
    ], format="csr")
    if masked:
        R = sp.diags(coarse.free.astype(np.float64)) @ R
    return R.tocsr()

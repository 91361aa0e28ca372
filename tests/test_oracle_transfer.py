"""Pins of the oracle's inter-grid transfers.

* P reproduces every biquadratic (d, u) and bilinear (p^s, p^f) field exactly
  (natural injection of nested Q2/Q1 spaces).
* P is block lower triangular in J2 order: P_{d^s,d^f} = 0.
* R has the zero pattern of R_2 (Section 3.3): coarse S rows receive fine F
  rows (R_SF), coarse K rows receive no fine F rows (no transpose of
  P_{u^f,u^s}), coarse A rows receive only fine A rows.
* Galerkin identity: with constant ALE coefficient, consistent kinematic
  mass and no convection, re-discretized coarse operators equal
  (D_c R) A_fine (D_f P) on free rows and columns.  The naive P^T fails it.
"""
import numpy as np
import pytest

from oracle import fem, transfer
from oracle.mesh import Level
from tests.cfgs import small


def _two_levels(**kw):
    cfg = small(levels=2, **kw)
    return cfg, Level(cfg, 1), Level(cfg, 0)


def test_prolongation_reproduces_polynomials():
    cfg, fine, coarse = _two_levels(nc=(3, 4), solid_rows=(0, 3),
                                    xb=[0, 0.2, 0.7, 1.0], yb=[0, 0.1, 0.5, 0.9, 1.0])
    P = transfer.prolongation(fine, coarse, masked=False)
    q2 = lambda X: np.stack([1 + X[:, 0] ** 2 * X[:, 1] ** 2 - 3 * X[:, 0] * X[:, 1],
                             X[:, 1] ** 2 - 2 * X[:, 0] ** 2 * X[:, 1] + X[:, 0]], 1)
    q1 = lambda x, y: 2 + x - 3 * y + 5 * x * y

    def vec(lv):
        v = np.zeros(lv.N)
        v[:2 * lv.N2] = q2(lv.X).ravel()
        v[lv.off_u:lv.off_u + 2 * lv.N2] = 2 * q2(lv.X).ravel()
        for flags, off, n in ((lv.vert_solid, lv.off_ps, lv.Nps),
                              (lv.vert_fluid, lv.off_pf, lv.Npf)):
            xy = lv.X[lv.node_of_vertex(np.where(flags)[0])]
            v[off:off + n] = q1(xy[:, 0], xy[:, 1])
        return v

    assert np.allclose(P @ vec(coarse), vec(fine), atol=1e-13, rtol=0)


def test_prolongation_block_lower_triangular():
    cfg, fine, coarse = _two_levels(nc=(4, 4), solid_rows=(0,))
    P = transfer.prolongation(fine, coarse, masked=False).tocsr()
    Pd = P[:2 * fine.N2][:, :2 * coarse.N2].tocoo()
    fine_node, coarse_node = Pd.row // 2, Pd.col // 2
    # P_{d^s, d^f} = 0: solid-side fine nodes never read coarse fluid nodes
    assert not np.any(fine.solid_side[fine_node] & ~coarse.solid_side[coarse_node])
    # P_{d^f, d^s} != 0: fluid fine nodes next to the interface read interface nodes
    assert np.any(~fine.solid_side[fine_node] & coarse.solid_side[coarse_node])


def test_restriction_zero_pattern():
    cfg, fine, coarse = _two_levels(nc=(4, 4), solid_rows=(0,))
    R = transfer.restriction(fine, coarse, masked=False).tocsr()
    D = 2
    Rdu = R[:D * coarse.N2][:, fine.off_u:fine.off_u + D * fine.N2].tocoo()
    # R_SF: coarse solid-side momentum rows from fine fluid momentum rows only
    assert Rdu.nnz > 0
    assert np.all(coarse.solid_side[Rdu.row // D])
    assert np.all(~fine.solid_side[Rdu.col // D])
    Ruu = R[coarse.off_u:coarse.off_u + D * coarse.N2][:, fine.off_u:fine.off_u + D * fine.N2].tocoo()
    # no transpose of P_{u^f,u^s}: coarse K rows never receive fine F rows
    bad = coarse.solid_side[Ruu.row // D] & ~fine.solid_side[Ruu.col // D]
    assert not np.any(bad)
    Rud = R[coarse.off_u:coarse.off_u + D * coarse.N2][:, :D * fine.N2]
    assert Rud.nnz == 0
    Rdd = R[:D * coarse.N2][:, :D * fine.N2].tocoo()
    # coarse A rows (fluid) only from fine A rows (fluid)
    fl = ~coarse.solid_side[Rdd.row // D]
    assert np.all(~fine.solid_side[Rdd.col[fl] // D])
    # R != P^T
    P = transfer.prolongation(fine, coarse, masked=False)
    assert abs(R - P.T).max() > 0.1


@pytest.mark.parametrize("solid_rows", [(0,), (0, 3)])
def test_galerkin_identity(solid_rows):
    cfg, fine, coarse = _two_levels(nc=(4, 4), solid_rows=solid_rows, ale_k=1, k_mass=1,
                                    yb=[0, 0.1, 0.5, 0.9, 1.0])
    cfg["bc_d"][0][0] = cfg["bc_d"][0][1] = 1
    cfg["bc_u"][0][0] = 2
    cfg["bc_u"][3][0] = 1 if solid_rows == (0,) else 0
    fine, coarse = Level(cfg, 1), Level(cfg, 0)
    Af = fem.dirichlet_reduce(fine, fem.assemble_level(fine, cfg)["A"])
    Ac = fem.dirichlet_reduce(coarse, fem.assemble_level(coarse, cfg)["A"])
    P = transfer.prolongation(fine, coarse)
    R = transfer.restriction(fine, coarse)
    G = (R @ Af @ P).toarray()
    fr = coarse.free
    ref = Ac.toarray()[np.ix_(fr, fr)]
    assert np.allclose(G[np.ix_(fr, fr)], ref, atol=1e-10 * abs(ref).max(), rtol=0)
    # the classical restriction P^T does not reproduce the coarse operator
    Gn = (P.T @ Af @ P).toarray()
    assert not np.allclose(Gn[np.ix_(fr, fr)], ref, atol=1e-6 * abs(ref).max(), rtol=0)

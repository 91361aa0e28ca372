"""Field-split additive Schwarz smoother (paper Section 3.2).

Field split (eq. P_2): the level system in J2 order is split into the fields
[d, p^s] and [u, p^f] and the off-diagonal field blocks are dropped.  Each
field is then solved by its own additive Schwarz strategy:

* AS_1 on [d, p^s]: solid Vanka blocks [S_ds S_ps; V_ds 0]_j and fluid
  overlapping blocks [A_df]_j;
* AS_2 on [u, p^f]: the lumped-mass block K_us (diagonal, one Jacobi step)
  and fluid Vanka blocks [F_uf F_pf; W_uf 0]_j.

Because the two fields never share an unknown, the field split followed by
AS on each field is one additive Schwarz iteration over the union of the
blocks.  Each block matrix is the principal submatrix of the level operator
on the block's unknowns (it only contains the equations listed above because
of the J2 routing).

Vanka block selection (Section 3.2): the domain is split into solid and fluid
sub-domains, each tiled by non-overlapping element-aligned cores.  A block
takes the pressures whose support meets its core and the displacements /
velocities whose support meets those pressures' supports.  With continuous Q1
pressure inside a region this is parametrised by a halo ``h``: pressures at
vertices of the core's elements, d/u at the Q2 nodes of the core's elements
grown by ``h`` element layers of the same region (``h = 1`` is the rule
taken literally, ``h = 0`` the element closure).  Fluid d blocks take the same
geometric sets without pressure and only fluid nodes (interface d belongs to
the solid equations).  Dirichlet unknowns belong to no block.

Additive update (the formula following eq. P^f_{1j}): every block uses the
same residual f - J x^k and entry i takes the value of the LAST block that
contains it, i.e. owner(i) = max{j : i in I_j}.  Unknowns in no block (u^s and
Dirichlet rows, whose rows are identity) get one Jacobi step r_i / A_ii.
Blocks are ordered field d before field u, tiles lexicographically (x
fastest), solid before fluid inside a tile.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp
from scipy import ndimage

from .mesh import Level


def build_blocks(lv: Level, core, halo: int):
    """Return (blocks, kinds): blocks is a list of sorted global index arrays;
    kinds[j] = (field, region) with field 0 = [d,p^s], 1 = [u,p^f]."""
    D = lv.D
    ne = lv.ne
    reg = lv.region.reshape(ne[::-1])                # [z][y][x]
    nt = [-(-ne[a] // core[a]) for a in range(D)]
    tiles = Level._x_fastest(tuple(nt))
    struct = np.ones((3,) * D, bool)
    blocks, kinds = [], []
    for field in (0, 1):
        for t in tiles:
            for region in ((1, 0) if field == 0 else (0,)):
                box = np.zeros(ne[::-1], bool)
                sl = tuple(slice(t[a] * core[a], min((t[a] + 1) * core[a], ne[a]))
                           for a in reversed(range(D)))
                box[sl] = True
                core_mask = box & (reg == region)
                if not core_mask.any():
                    continue
                blk_mask = core_mask
                if halo > 0:
                    blk_mask = ndimage.binary_dilation(core_mask, structure=struct,
                                                       iterations=halo) & (reg == region)
                core_el = np.where(core_mask.ravel())[0]
                blk_el = np.where(blk_mask.ravel())[0]
                nodes = np.unique(lv.elem_nodes[blk_el])
                verts = np.unique(lv.elem_verts[core_el])
                if field == 0 and region == 1:
                    dofs = np.concatenate([(D * nodes[:, None] + np.arange(D)).ravel(),
                                           lv.ps_of_vert[verts]])
                elif field == 0:
                    fn = nodes[~lv.solid_side[nodes]]
                    dofs = (D * fn[:, None] + np.arange(D)).ravel()
                else:
                    fn = nodes[~lv.solid_side[nodes]]
                    dofs = np.concatenate([(lv.off_u + D * fn[:, None] + np.arange(D)).ravel(),
                                           lv.pf_of_vert[verts]])
                assert np.all(dofs >= 0)
                dofs = np.sort(dofs[lv.free[dofs]])
                if len(dofs) == 0:
                    continue
                blocks.append(dofs)
                kinds.append((field, region))
    return blocks, kinds


def owners(N: int, blocks) -> np.ndarray:
    """owner(i) = index of the last block containing i, -1 if none."""
    own = -np.ones(N, np.int64)
    for j, I in enumerate(blocks):
        own[I] = j
    return own


class FieldSplitSchwarz:
    """B = sum_j E_j A_j^{-1} R_j (last-writer extension) + Jacobi on the rest."""

    def __init__(self, A: sp.csr_matrix, blocks):
        self.N = A.shape[0]
        self.blocks = blocks
        self.owner = owners(self.N, blocks)
        A = A.tocsr()
        self.lu = [la.lu_factor(A[I][:, I].toarray()) for I in blocks]
        self.owned = [self.owner[I] == j for j, I in enumerate(blocks)]
        self.jac = np.where(self.owner < 0)[0]
        self.jac_inv = 1.0 / A.diagonal()[self.jac]

    def apply(self, r: np.ndarray) -> np.ndarray:
        delta = np.zeros(self.N)
        for lu, I, own in zip(self.lu, self.blocks, self.owned):
            y = la.lu_solve(lu, r[I])
            delta[I[own]] = y[own]
        delta[self.jac] = r[self.jac] * self.jac_inv
        return delta

    def apply_transpose(self, r: np.ndarray) -> np.ndarray:
        delta = np.zeros(self.N)
        for lu, I, own in zip(self.lu, self.blocks, self.owned):
            s = np.where(own, r[I], 0.0)
            delta[I] += la.lu_solve(lu, s, trans=1)
        delta[self.jac] += r[self.jac] * self.jac_inv
        return delta

    def dense(self, A: sp.csr_matrix) -> np.ndarray:
        """B as a dense matrix built from explicit inverses (numpy.linalg.inv)."""
        B = np.zeros((self.N, self.N))
        A = A.tocsr()
        for j, I in enumerate(self.blocks):
            Ainv = np.linalg.inv(A[I][:, I].toarray())
            own = self.owned[j]
            B[np.ix_(I[own], I)] = Ainv[own]
        B[self.jac, self.jac] = self.jac_inv
        return B

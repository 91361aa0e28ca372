"""Nested structured meshes, node types and the J2 unknown layout.

Paper passages followed:

* Section 3.3 (Geometric Multigrid Preconditioner): every level is the
  midpoint refinement of a conforming coarse mesh, and the fluid/solid split
  is the same on every level.
* Section 3.1 / eq. (matrix_J2): unknowns d^s d^f p^s | u^s u^f p^f; the
  kinematic and momentum test functions of interface nodes belong to the
  solid-side equations (K, S), those of the remaining fluid nodes to A, F.
* Section 2.2: the fluid ALE test functions vanish on the interface.

Layout of a level vector (the library uses the same documented format)::

    [ d : node-major, component-minor, all Q2 nodes     (dim * N2)
    | p^s : Q1 vertices of solid elements, vertex order (Nps)
    | u : node-major, component-minor, all Q2 nodes     (dim * N2)
    | p^f : Q1 vertices of fluid elements, vertex order (Npf) ]

The d-row of a solid-side node carries the S equation, of a fluid node the A
equation; the u-row carries K or F respectively.  Pressures are continuous Q1
inside each region, duplicated on interface vertices (pressures are free at
the interface, Section 3.3).
"""
from __future__ import annotations

import numpy as np


def multi_index(n: int, dim: int) -> np.ndarray:
    """All tuples in {0..n-1}^dim, first component fastest, shape (n**dim, dim)."""
    k = np.arange(n ** dim)
    return np.stack([(k // n ** a) % n for a in range(dim)], axis=1)


def refine_breaks(b, times: int) -> np.ndarray:
    """Insert midpoints ``times`` times (midpoint refinement in reference space)."""
    b = np.asarray(b, dtype=np.float64)
    for _ in range(times):
        out = np.empty(2 * len(b) - 1)
        out[0::2] = b
        out[1::2] = 0.5 * (b[:-1] + b[1:])
        b = out
    return b


def physical_map(cfg: dict, xref: np.ndarray) -> np.ndarray:
    """Map reference coordinates (n, dim) to physical coordinates."""
    x = np.array(xref, dtype=np.float64, copy=True)
    if cfg["mapping"] == 0:
        return x
    if cfg["mapping"] == 1:
        # circular bulge of radius R centred at xc on the top of the channel;
        # the shift is blended in linearly between reference heights ya and yb
        xc, R, ya, yb = cfg["map_params"]
        bump = np.sqrt(np.maximum(R * R - (xref[:, 0] - xc) ** 2, 0.0))
        s = np.clip((xref[:, 1] - ya) / (yb - ya), 0.0, 1.0)
        x[:, 1] = xref[:, 1] + bump * s
        return x
    if cfg["mapping"] == 2:
        # smooth bulge of height and half-width R centred at xc: the profile
        # R cos^2(pi (x - xc) / (2R)) is tangent to the straight wall at
        # |x - xc| = R, so the shear of the mapped elements is bounded under
        # refinement (the circular profile meets the wall vertically and
        # shears the elements there without bound); same blending as above
        xc, R, ya, yb = cfg["map_params"]
        dx = xref[:, 0] - xc
        bump = np.where(np.abs(dx) < R, R * np.cos(np.pi * dx / (2.0 * R)) ** 2, 0.0)
        s = np.clip((xref[:, 1] - ya) / (yb - ya), 0.0, 1.0)
        x[:, 1] = xref[:, 1] + bump * s
        return x
    if cfg["mapping"] == 3:
        # the square cross-section [0,1]^2 onto a disc of centre (cx, cy) and
        # radius R: with a, b the section coordinates scaled to [-1, 1],
        # x' = a sqrt(1 - b^2/2), y' = b sqrt(1 - a^2/2) sends each edge of
        # the square onto the circle; the axis coordinate is unchanged
        cx, cy, R = cfg["map_params"][:3]
        a = 2.0 * xref[:, 0] - 1.0
        b = 2.0 * xref[:, 1] - 1.0
        x[:, 0] = cx + R * a * np.sqrt(1.0 - 0.5 * b * b)
        x[:, 1] = cy + R * b * np.sqrt(1.0 - 0.5 * a * a)
        return x
    raise ValueError("unknown mapping %r" % cfg["mapping"])


class Level:
    """One level of the nested hierarchy (level 0 = coarsest)."""

    def __init__(self, cfg: dict, l: int):
        D = int(cfg["dim"])
        self.cfg, self.l, self.D = cfg, l, D
        self.ne = tuple(int(n) << l for n in cfg["nc"])       # elements per axis
        self.nn = tuple(2 * n + 1 for n in self.ne)           # Q2 node lines
        self.nv = tuple(n + 1 for n in self.ne)               # Q1 vertex lines
        self.nE = int(np.prod(self.ne))
        self.N2 = int(np.prod(self.nn))
        self.NV = int(np.prod(self.nv))

        # element multi-indices, x fastest
        eidx = self._x_fastest(self.ne)
        self.eidx = eidx
        # region inherited from the coarse parent element
        creg = np.asarray(cfg["region"], dtype=np.int64)
        cidx = eidx >> l
        self.region = creg[self._lin(cidx, cfg["nc"])]

        # Q2 nodes of each element (local index x fastest over {0,1,2}^D)
        loc2 = multi_index(3, D)
        self.elem_nodes = self._lin(2 * eidx[:, None, :] + loc2[None, :, :], self.nn)
        loc1 = multi_index(2, D)
        self.elem_verts = self._lin(eidx[:, None, :] + loc1[None, :, :], self.nv)

        # reference and physical coordinates of Q2 nodes
        self.xref_lines = [refine_breaks(cfg["breaks"][a], l + 1) for a in range(D)]
        nidx = self._x_fastest(self.nn)
        self.nidx = nidx
        xref = np.stack([self.xref_lines[a][nidx[:, a]] for a in range(D)], axis=1)
        self.xref = xref
        self.X = physical_map(cfg, xref)

        # node types: solid-side = belongs to at least one solid element
        solid_el = self.region == 1
        self.solid_side = np.zeros(self.N2, bool)
        self.solid_side[self.elem_nodes[solid_el].ravel()] = True
        self.fluid_touch = np.zeros(self.N2, bool)
        self.fluid_touch[self.elem_nodes[~solid_el].ravel()] = True
        self.vert_solid = np.zeros(self.NV, bool)
        self.vert_solid[self.elem_verts[solid_el].ravel()] = True
        self.vert_fluid = np.zeros(self.NV, bool)
        self.vert_fluid[self.elem_verts[~solid_el].ravel()] = True

        # unknown layout
        self.Nps = int(self.vert_solid.sum())
        self.Npf = int(self.vert_fluid.sum())
        self.off_ps = D * self.N2
        self.off_u = D * self.N2 + self.Nps
        self.off_pf = 2 * D * self.N2 + self.Nps
        self.N = 2 * D * self.N2 + self.Nps + self.Npf
        self.ps_of_vert = -np.ones(self.NV, np.int64)
        self.ps_of_vert[self.vert_solid] = self.off_ps + np.arange(self.Nps)
        self.pf_of_vert = -np.ones(self.NV, np.int64)
        self.pf_of_vert[self.vert_fluid] = self.off_pf + np.arange(self.Npf)

        self._dirichlet()

    # ------------------------------------------------------------------
    @staticmethod
    def _x_fastest(shape):
        D = len(shape)
        n = int(np.prod(shape))
        k = np.arange(n)
        out = np.empty((n, D), np.int64)
        stride = 1
        for a in range(D):
            out[:, a] = (k // stride) % shape[a]
            stride *= shape[a]
        return out

    @staticmethod
    def _lin(idx, shape):
        idx = np.asarray(idx, np.int64)
        out = np.zeros(idx.shape[:-1], np.int64)
        stride = 1
        for a in range(len(shape)):
            out = out + idx[..., a] * stride
            stride *= int(shape[a])
        return out

    def d(self, node, comp):
        return self.D * np.asarray(node) + np.asarray(comp)

    def u(self, node, comp):
        return self.off_u + self.D * np.asarray(node) + np.asarray(comp)

    def node_of_vertex(self, v):
        vidx = self._x_fastest(self.nv)[v]
        return self._lin(2 * vidx, self.nn)

    # ------------------------------------------------------------------
    def _dirichlet(self):
        """Dirichlet DOFs and values from the per-face, per-region tags.

        A tag bc[face][region] constrains every node on that face that belongs
        to an element of that region (the condition holds on the closure of
        the region's boundary part), so interface nodes at the end of a fluid
        inflow or wall face are constrained as well; the parabolic inflow
        profile vanishes there."""
        cfg, D = self.cfg, self.D
        self.dir_mask = np.zeros(self.N, bool)
        self.dir_val = np.zeros(self.N)
        touch = (self.fluid_touch, self.solid_side)      # indexed by region 0 / 1
        wall = np.zeros(self.N2, bool)
        inflow = np.zeros(self.N2, bool)
        inflow_val = np.zeros((self.N2, D))
        for f in range(2 * D):
            a, side = f // 2, f % 2
            on = self.nidx[:, a] == (0 if side == 0 else self.nn[a] - 1)
            if not on.any():
                continue
            dmask = np.zeros(self.N2, bool)
            wmask = np.zeros(self.N2, bool)
            imask = np.zeros(self.N2, bool)
            for r in (0, 1):
                dmask |= on & touch[r] & (cfg["bc_d"][f][r] == 1)
                wmask |= on & touch[r] & (cfg["bc_u"][f][r] == 1)
                imask |= on & touch[r] & (cfg["bc_u"][f][r] == 2)
            for c in range(D):
                self.dir_mask[self.d(np.where(dmask)[0], c)] = True
            wall |= wmask
            if imask.any():
                # parabolic profile over the fluid extent of this face
                prof = np.ones(self.N2)
                sel = on & self.fluid_touch
                for b in range(D):
                    if b == a:
                        continue
                    lo = self.xref[sel, b].min()
                    hi = self.xref[sel, b].max()
                    s = (self.xref[:, b] - lo) / (hi - lo)
                    prof = prof * 4.0 * s * (1.0 - s)
                sign = 1.0 if side == 0 else -1.0
                inflow_val[imask, a] = sign * cfg["inflow_peak"] * prof[imask]
                inflow |= imask
        umask = wall | inflow
        for c in range(D):
            ud = self.u(np.where(umask)[0], c)
            self.dir_mask[ud] = True
            val = np.where(wall[umask], 0.0, inflow_val[umask, c])
            self.dir_val[ud] = val
        self.free = ~self.dir_mask

    # ------------------------------------------------------------------
    def inject_from_finest(self, arr_finest: np.ndarray, L: int) -> np.ndarray:
        """Values of a finest-level nodal field at this level's Q2 nodes.

        Level-l Q2 node lines are every 2**(L-1-l)-th finest node line."""
        step = 2 ** (L - 1 - self.l)
        nn_f = tuple((n - 1) * step + 1 for n in self.nn)
        fidx = self._lin(self.nidx * step, nn_f)
        return arr_finest[fidx]


def hierarchy_levels(cfg: dict) -> list:
    return [Level(cfg, l) for l in range(int(cfg["n_levels"]))]

"""Geometric multigrid V-cycle with the FS-AS smoother (paper Section 3).

GMRES is preconditioned by GMG; on every level l >= 1 a damped Richardson
iteration preconditioned by the field-split smoother is used, on level 0 a
direct solver (Section 3.2, after eq. matrix_J2).  Level operators are
re-discretized on each level.  The coarse solve is a dense LU with partial
pivoting.

The transposed cycle applies M^T exactly: it is the V-cycle of A^T with the
smoother B^T, restriction by (D_f P)^T, prolongation by (D_c R)^T and the
numbers of pre- and post-sweeps exchanged.

The interchange the paper names as future work (Section 5: the GMG and FS
boxes of its solver cascade swapped) is built as cfg["interchange"]: GMRES
preconditioned by the field split P_2 (eq. FS), which is block diagonal over
the field groups [d, p^s] and [u, p^f], each diagonal block approximated by
one GMG cycle on that block.  Both diagonal-block cycles share the levels,
so they are one cycle on blockdiag(D_1, D_2) of every level operator: the
residuals use the level operators with every entry coupling the two groups
removed, the restriction keeps only the routing inside a group (R_2 sends
fine fluid-momentum rows, which belong to D_2, into coarse solid-momentum
rows of D_1; those entries are dropped), the prolongation never mixes the
groups, the FS-AS blocks lie inside one group, and level 0 solves its own
diagonal blocks directly.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

from . import fem, transfer
from .mesh import Level, hierarchy_levels
from .schwarz import (FieldSplitSchwarz, MultiplicativeSchwarz, block_colouring,
                      build_blocks, colour_major, coupling_pattern)


def field_groups(lv: Level) -> np.ndarray:
    """Group of every unknown: 0 for d and p^s (the first row / column block
    of J_2), 1 for u and p^f."""
    g = np.zeros(lv.N, np.int8)
    g[lv.off_u:] = 1
    return g


def diagonal_blocks(M: sp.spmatrix, grow: np.ndarray, gcol: np.ndarray) -> sp.csr_matrix:
    """M with every entry that couples the two field groups removed."""
    C = sp.coo_matrix(M)
    keep = grow[C.row] == gcol[C.col]
    return sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=M.shape)


class Hierarchy:
    def __init__(self, cfg: dict, w_finest: np.ndarray | None = None,
                 taus: list | None = None, build_smoothers: bool = True):
        self.cfg = cfg
        self.L = int(cfg["n_levels"])
        self.levels = hierarchy_levels(cfg)
        self.w_finest = w_finest
        self.A_full, self.A, self.parts = [], [], []
        for l, lv in enumerate(self.levels):
            w = None if w_finest is None else lv.inject_from_finest(w_finest, self.L)
            tau = None if taus is None else taus[l]
            asm = fem.assemble_level(lv, cfg, w, tau)
            self.parts.append(asm)
            self.A_full.append(asm["A"])
            self.A.append(fem.dirichlet_reduce(lv, asm["A"]))
        self.P = [None] + [transfer.prolongation(self.levels[l], self.levels[l - 1])
                           for l in range(1, self.L)]
        self.R = [None] + [transfer.restriction(self.levels[l], self.levels[l - 1])
                           for l in range(1, self.L)]
        # operators and restriction of the cycle: the level operators and R_2,
        # or their field-group diagonal blocks for the interchanged cascade
        self.interchange = bool(cfg.get("interchange", False))
        if self.interchange:
            g = [field_groups(lv) for lv in self.levels]
            self.Ac = [diagonal_blocks(self.A[l], g[l], g[l]) for l in range(self.L)]
            self.Rc = [None] + [diagonal_blocks(self.R[l], g[l - 1], g[l])
                                for l in range(1, self.L)]
        else:
            self.Ac, self.Rc = self.A, self.R
        self.coarse_lu = la.lu_factor(self.Ac[0].toarray())
        self.smoothers = [None] * self.L
        if build_smoothers:
            self.build_smoothers()

    @property
    def finest(self) -> Level:
        return self.levels[-1]

    def build_smoothers(self, core=None, halo=None, iface_mult=None, monolithic=None,
                        schwarz=None):
        """schwarz: "additive" (default) or "multiplicative"; the
        multiplicative sweep takes the blocks colour by colour (greedy
        colouring in block order), the block order inside a colour kept."""
        cfg = self.cfg
        core = tuple(cfg["core"]) if core is None else tuple(core)
        halo = int(cfg["halo"]) if halo is None else int(halo)
        mult = int(cfg.get("iface_mult", 1)) if iface_mult is None else int(iface_mult)
        mono = bool(cfg.get("monolithic", False)) if monolithic is None else bool(monolithic)
        kind = cfg.get("schwarz", "additive") if schwarz is None else schwarz
        if kind not in ("additive", "multiplicative"):
            raise ValueError(f"unknown Schwarz kind {kind!r}")
        self.colours = [None] * self.L
        for l in range(1, self.L):
            blocks, _ = build_blocks(self.levels[l], core, halo, mult, mono)
            if kind == "additive":
                self.smoothers[l] = FieldSplitSchwarz(self.Ac[l], blocks)
            else:
                blocks, self.colours[l] = colour_major(
                    blocks, block_colouring(self.coupling_pattern(l), blocks))
                self.smoothers[l] = MultiplicativeSchwarz(self.Ac[l], blocks)

    def coupling_pattern(self, l: int) -> sp.csr_matrix:
        """Parameter-independent coupling pattern of the level-l operator (the
        union over its Dirichlet-reduced affine pieces)."""
        lv = self.levels[l]
        return coupling_pattern([fem.dirichlet_reduce(lv, self.parts[l][k])
                                 for k in ("base", "AG", "AC", "Amu")])

    def rhs(self, fnodal: np.ndarray) -> np.ndarray:
        """Finest-level right-hand side for a nodal body force (Dirichlet-lifted)."""
        lv = self.finest
        w = None if self.w_finest is None else self.w_finest
        tau = self.parts[-1]["tau"]
        b_raw = fem.load_vector(lv, self.cfg, fnodal, w, tau)
        return fem.dirichlet_rhs(lv, self.A_full[-1], b_raw)

    # ------------------------------------------------------------------
    def _sweeps(self, l, b, x, n, transpose):
        A = self.Ac[l]
        S = self.smoothers[l]
        om = self.cfg["omega"]
        for s in range(n):
            if x is None:                      # first sweep from x = 0: r = b
                x = om * (S.apply_transpose(b) if transpose else S.apply(b))
            else:
                r = b - (A.T @ x if transpose else A @ x)
                x = x + om * (S.apply_transpose(r) if transpose else S.apply(r))
        return x

    def vcycle(self, b: np.ndarray, l: int | None = None, transpose: bool = False,
               x0: np.ndarray | None = None, kind: str | None = None):
        """z = M^{-1} b (or M^{-T} b) on level l (default finest) for the
        configured cycle (cfg["cycle"]: "V" default, "W" or "F"; Section 3.2
        allows any).  With an initial guess x0 the cycle returns
        x0 + M^{-1} (b - A x0) (pre-smoothing starts from x0).

        The coarse correction solves the restricted residual equation by
          V: one cycle on level l-1 from zero,
          W: two W-cycles, the second from the first one's result,
          F: an F-cycle then a V-cycle from its result.
        Transposed: pre and post smoothing swapped, every operator
        transposed; the coarse cycles of F run in the reverse order (V, then
        F), which is what transposing x1 = M_F b, x2 = x1 + M_V (b - A x1)
        gives."""
        if l is None:
            l = self.L - 1
        if kind is None:
            kind = self.cfg.get("cycle", "V")
        if l == 0:
            return la.lu_solve(self.coarse_lu, b, trans=1 if transpose else 0)
        cfg = self.cfg
        n1, n2 = cfg["nu_pre"], cfg["nu_post"]
        if transpose:
            n1, n2 = n2, n1
        x = self._sweeps(l, b, x0, n1, transpose)
        A = self.Ac[l]
        if x is None:
            x = np.zeros_like(b)
        r = b - (A.T @ x if transpose else A @ x)
        if transpose:
            bc = self.P[l].T @ r
        else:
            bc = self.Rc[l] @ r
        coarse = {"V": ["V"], "W": ["W", "W"], "F": ["F", "V"]}[kind]
        if transpose:
            coarse = coarse[::-1]
        xc = None
        for k in coarse:
            xc = self.vcycle(bc, l - 1, transpose, xc, k)
        x = x + (self.Rc[l].T @ xc if transpose else self.P[l] @ xc)
        x = self._sweeps(l, b, x, n2, transpose)
        return x

    def dense_preconditioner(self, transpose=False) -> np.ndarray:
        N = self.A[-1].shape[0]
        M = np.zeros((N, N))
        for i in range(N):
            e = np.zeros(N)
            e[i] = 1.0
            M[:, i] = self.vcycle(e, transpose=transpose)
        return M

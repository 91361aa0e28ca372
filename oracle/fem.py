"""Q2/Q1 assembly of the linearized monolithic FSI operator (oracle).

What is assembled (paper Section 2.2 and Section 3.1, linearized about the
stress-free state d = 0 with a frozen advecting velocity w; steady):

* S rows (momentum, test functions of solid-side nodes, eq. momentum_supg):
  over solid elements the linearized Mooney-Rivlin stress, which at the
  stress-free state is -p^s I + G (grad d + grad d^T) with C1 = G/3,
  C2 = C1/2 and E = 2G(1+nu) (eq. Mooney-Rivelin-cauchy);
  over fluid elements the Newtonian stress -p^f I + mu (grad u + grad u^T)
  (eq. newtonian), the convective term rho (w.grad) u and SUPG.
* F rows: the same fluid terms for test functions of fluid nodes.
* A rows (eq. kinfld): (k (grad d + grad d^T), grad phi) over fluid elements
  for test functions of fluid nodes (they vanish on the interface), with
  k = 1 / V_el (the choice after eq. newtonian).  V_el is the volume of the
  COARSEST-mesh element containing the point, so k is one function of the
  reference coordinate on every level (with per-level volumes the
  re-discretized coarse ALE operators would be 2^dim times weaker than the
  fine ones).  cfg['ale_k'] == 1 selects k = 1.
* K rows (eq. kinsld): lumped Q2 mass on u^s (cfg['k_mass'] == 0) or the
  consistent mass (== 1); with a backward-Euler step dt (cfg['dt'] finite)
  the time derivative of d adds K_ds = -K_us / dt.  Steady: dt = inf.
* inertia (eq. momentum_supg, backward Euler): rho M / dt on u in every
  momentum row, plus its SUPG counterpart on fluid elements.
* V rows (eq. cntsld linearized): -(div d, q) - (1/lambda_L) (p^s, q) with
  lambda_L = E nu / ((1+nu)(1-2nu)); the second term vanishes at nu = 1/2.
* W rows (eq. cntfld): -(div u, q).
* SUPG (eqs. tausupg, lambda_k): test function tau rho (w.grad) phi on fluid
  elements, tau = xi(Re) / (sqrt(lambda_k) |w|_2), Re = |w|/(4 sqrt(lambda_k) nu),
  lambda_k the largest eigenvalue of the generalized problem on the element's
  interior Q2 space, which is spanned by the element bubble times each unit
  vector, so the problem is dim x dim and is solved directly.

The operator is split affinely, A = A_base + G A_G + (1/lambda_L) A_C + mu A_mu
(tau held fixed), which is what parameter gradients differentiate.
Second derivatives of Q2 functions use the element Jacobian only (the map's
own curvature is neglected; exact on affine elements).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import Level, multi_index

_SQ = np.sqrt(0.6)
GAUSS_PTS = np.array([-_SQ, 0.0, _SQ])
GAUSS_W = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def q2_1d(xi):
    """1D quadratic Lagrange basis on nodes -1, 0, 1: values, 1st, 2nd derivatives."""
    xi = np.asarray(xi, dtype=np.float64)
    v = np.stack([0.5 * xi * (xi - 1.0), 1.0 - xi * xi, 0.5 * xi * (xi + 1.0)], -1)
    d = np.stack([xi - 0.5, -2.0 * xi, xi + 0.5], -1)
    dd = np.stack([np.ones_like(xi), -2.0 * np.ones_like(xi), np.ones_like(xi)], -1)
    return v, d, dd


def q1_1d(xi):
    xi = np.asarray(xi, dtype=np.float64)
    v = np.stack([0.5 * (1.0 - xi), 0.5 * (1.0 + xi)], -1)
    d = np.stack([-0.5 * np.ones_like(xi), 0.5 * np.ones_like(xi)], -1)
    return v, d


class RefElement:
    """Tensor-product Q2 / Q1 reference element with a 3-point Gauss rule per axis."""

    def __init__(self, D: int):
        self.D = D
        qidx = multi_index(3, D)
        self.nq = len(qidx)
        self.xi = GAUSS_PTS[qidx]
        self.wq = np.prod(GAUSS_W[qidx], axis=1)
        a2 = multi_index(3, D)
        a1 = multi_index(2, D)
        self.nb, self.np_ = len(a2), len(a1)
        L, dL, d2L = q2_1d(GAUSS_PTS)          # (3 pts, 3 nodes)
        N, dN = q1_1d(GAUSS_PTS)
        nq, nb = self.nq, self.nb
        self.phi = np.ones((nq, nb))
        self.dphi = np.ones((nq, nb, D))
        self.d2phi = np.ones((nq, nb, D, D))
        for k in range(D):
            Lk = L[qidx[:, k]][:, a2[:, k]]      # (nq, nb)
            dLk = dL[qidx[:, k]][:, a2[:, k]]
            d2Lk = d2L[qidx[:, k]][:, a2[:, k]]
            self.phi *= Lk
            for i in range(D):
                self.dphi[:, :, i] *= dLk if i == k else Lk
                for j in range(D):
                    if i == k and j == k:
                        f = d2Lk
                    elif i == k or j == k:
                        f = dLk
                    else:
                        f = Lk
                    self.d2phi[:, :, i, j] *= f
        self.psi = np.ones((nq, self.np_))
        self.dpsi = np.ones((nq, self.np_, D))
        for k in range(D):
            Nk = N[qidx[:, k]][:, a1[:, k]]
            dNk = dN[qidx[:, k]][:, a1[:, k]]
            self.psi *= Nk
            for i in range(D):
                self.dpsi[:, :, i] *= dNk if i == k else Nk
        self.bubble = int(sum(3 ** k for k in range(D)))   # local index of (1,..,1)


def geometry(ref: RefElement, Xe: np.ndarray):
    """Isoparametric geometry at Gauss points for elements with Q2 node coords Xe.

    Returns dV (nE,nq), physical Q2 gradients G (nE,nq,nb,D), Hessians
    H (nE,nq,nb,D,D) and Q1 gradients Gp (nE,nq,np,D)."""
    J = np.einsum("eai,qak->eqik", Xe, ref.dphi)          # dx_i / dxi_k
    det = np.linalg.det(J)
    if not np.all(det > 0):
        raise ValueError("non-positive Jacobian determinant")
    Jinv = np.linalg.inv(J)                               # dxi_k / dx_i  [k, i]
    G = np.einsum("qak,eqki->eqai", ref.dphi, Jinv)
    H = np.einsum("eqki,qakm,eqmj->eqaij", Jinv, ref.d2phi, Jinv)
    Gp = np.einsum("qmk,eqki->eqmi", ref.dpsi, Jinv)
    dV = det * ref.wq[None, :]
    return dV, G, H, Gp


def lame_constants(E: float, nu: float):
    """Shear modulus G = E/(2(1+nu)) and 1/lambda_L (0 for nu = 1/2)."""
    G = E / (2.0 * (1.0 + nu))
    inv_lam = 0.0 if nu >= 0.5 else (1.0 + nu) * (1.0 - 2.0 * nu) / (E * nu)
    return G, inv_lam


def coarse_element_volumes(cfg: dict) -> np.ndarray:
    """Volume of every level-0 element (isoparametric Q2 geometry, Gauss rule)."""
    lv0 = Level(cfg, 0)
    dV = geometry(RefElement(lv0.D), lv0.X[lv0.elem_nodes])[0]
    return dV.sum(axis=1)


def parent_coarse_element(lv: Level) -> np.ndarray:
    """Index of the level-0 element containing each element of level lv."""
    return Level._lin(lv.eidx >> lv.l, lv.cfg["nc"])


def supg_lambda(ref: RefElement, dV, G, H):
    """lambda_k of eq. (lambda_k) restricted to the element bubble space."""
    D = ref.D
    ab = ref.bubble
    lap = np.einsum("eqii->eq", H[:, :, ab])
    # div(grad w + grad w^T) for w = b e_a:  lap(b) e_a + grad(d_a b)
    v = np.einsum("ia,eq->eqai", np.eye(D), lap) + np.transpose(H[:, :, ab], (0, 1, 3, 2))
    Mb = np.einsum("eq,eqai,eqbi->eab", dV, v, v)
    Nb = np.einsum("eq,eqi,eqi->e", dV, G[:, :, ab], G[:, :, ab])
    return np.linalg.eigvalsh(Mb)[:, -1] / Nb


def supg_tau(lam, wnorm, mu, rho):
    """tau = xi(Re)/(sqrt(lambda)|w|) written as 1/max(4 lambda nu, sqrt(lambda)|w|)."""
    nu_k = mu / rho
    return 1.0 / np.maximum(4.0 * lam[:, None] * nu_k, np.sqrt(lam)[:, None] * wnorm)


class _COO:
    def __init__(self, N):
        self.N = N
        self.r, self.c, self.v = [], [], []

    def add(self, rows, cols, vals):
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        R = np.broadcast_to(rows[:, :, None], vals.shape)
        C = np.broadcast_to(cols[:, None, :], vals.shape)
        m = R >= 0
        self.r.append(R[m])
        self.c.append(C[m])
        self.v.append(vals[m])

    def csr(self):
        if not self.r:
            return sp.csr_matrix((self.N, self.N))
        A = sp.coo_matrix((np.concatenate(self.v),
                           (np.concatenate(self.r), np.concatenate(self.c))),
                          shape=(self.N, self.N)).tocsr()
        A.sum_duplicates()
        return A


def _sym_stiffness(dV, G):
    """K[e,a,c,b,f] = int (delta_cf grad phi_a . grad phi_b + d_f phi_a d_c phi_b)."""
    T = np.einsum("eq,eqai,eqbj->eabij", dV, G, G)
    nE, nb, _, D, _ = T.shape
    K = np.einsum("cf,eab->eacbf", np.eye(D), np.einsum("eabii->eab", T))
    K += np.transpose(T, (0, 1, 4, 2, 3))        # [e,a,b,f,c] -> [e,a,c,b,f]
    return K.reshape(nE, nb * D, nb * D)


def assemble_level(lv: Level, cfg: dict, w: np.ndarray | None = None,
                   tau: np.ndarray | None = None):
    """Assemble the unreduced level operator and its affine pieces.

    ``w``: advecting velocity at this level's Q2 nodes (N2, D) or None.
    ``tau``: optional frozen SUPG parameter per (fluid element, Gauss point).
    Returns dict(A, base, AG, AC, Amu, T, Tx, tau, G, inv_lam).  T is the
    time operator: the sum of the terms that carry 1/dt (a part of ``base``;
    zero when steady).  cfg["theta"] (default 1) weights the steady terms of
    the momentum rows (the rows of the momentum balance: solid-side d rows
    and fluid u rows), theta = 1/2 being Crank-Nicolson for the momentum
    balance while the other time derivatives stay backward differences;
    Tx = T - (1 - theta) M with M those steady momentum-row terms, so that
    one time step solves A x_n = load + Tx x_{n-1} (Tx = T for theta = 1)."""
    D, ref = lv.D, RefElement(lv.D)
    nb, npv = ref.nb, ref.np_
    rho, mu = cfg["rho"], cfg["mu"]
    Gmod, inv_lam = lame_constants(cfg["E"], cfg["nu"])
    inv_dt = 1.0 / cfg.get("dt", np.inf)
    theta = float(cfg.get("theta", 1.0))
    if not 0.0 < theta <= 1.0:
        raise ValueError("theta must lie in (0, 1]")
    base, AG, AC, Amu = _COO(lv.N), _COO(lv.N), _COO(lv.N), _COO(lv.N)
    Tt = _COO(lv.N)
    # the steady momentum-row terms, per affine piece (for Tx)
    Mb, MG, Mmu = _COO(lv.N), _COO(lv.N), _COO(lv.N)

    def add_time(rows, cols, vals):
        base.add(rows, cols, vals)
        Tt.add(rows, cols, vals)

    def add_mom(piece, mpiece, rows, cols, vals):
        """A steady term of a momentum row: weight theta in the operator."""
        piece.add(rows, cols, vals if theta == 1.0 else theta * vals)
        if inv_dt and theta != 1.0:
            mpiece.add(rows, cols, vals)
    comp = np.arange(D)

    Xe = lv.X[lv.elem_nodes]
    dV, G, H, Gp = geometry(ref, Xe)
    Bdiv = np.einsum("eq,qm,eqbf->embf", dV, ref.psi, G).reshape(lv.nE, npv, nb * D)
    Mq2 = np.einsum("eq,qa,qb->eab", dV, ref.phi, ref.phi)
    Mq1 = np.einsum("eq,qm,qn->emn", dV, ref.psi, ref.psi)
    Ksym = _sym_stiffness(dV, G)

    nodes = lv.elem_nodes
    dof_d = (D * nodes[:, :, None] + comp).reshape(lv.nE, nb * D)
    dof_u = lv.off_u + dof_d
    eyeD = np.eye(D)

    # ---------------- solid elements ----------------
    s = lv.region == 1
    if s.any():
        dps = lv.ps_of_vert[lv.elem_verts[s]]
        add_mom(AG, MG, dof_d[s], dof_d[s], Ksym[s])                     # S_ds
        add_mom(base, Mb, dof_d[s], dps, -np.transpose(Bdiv[s], (0, 2, 1)))   # S_ps
        base.add(dps, dof_d[s], -Bdiv[s])                                # V_ds
        AC.add(dps, dps, -Mq1[s])                                        # V_ps (compressible)
        if cfg.get("k_mass", 0) == 0:
            lump = Mq2[s].sum(axis=2)                                    # (nS, nb)
            vals = np.repeat(lump, D, axis=1)
            nS = vals.shape[0]
            diag = np.zeros((nS, nb * D, nb * D))
            idx = np.arange(nb * D)
            diag[:, idx, idx] = vals
            base.add(dof_u[s], dof_u[s], diag)                           # K_us lumped
            if inv_dt:
                add_time(dof_u[s], dof_d[s], -inv_dt * diag)             # K_ds
        else:
            Mc = np.einsum("eab,cf->eacbf", Mq2[s], eyeD).reshape(-1, nb * D, nb * D)
            base.add(dof_u[s], dof_u[s], Mc)
            if inv_dt:
                add_time(dof_u[s], dof_d[s], -inv_dt * Mc)
        if inv_dt:
            add_time(dof_d[s], dof_u[s], rho * inv_dt *
                     np.einsum("eab,cf->eacbf", Mq2[s], eyeD).reshape(-1, nb * D, nb * D))

    # ---------------- fluid elements ----------------
    f = lv.region == 0
    tau_out = None
    if f.any():
        nF = int(f.sum())
        ss = lv.solid_side[nodes[f]]                                     # (nF, nb)
        row_m = np.where(np.repeat(ss, D, axis=1), dof_d[f], dof_u[f])   # S or F rows
        dpf = lv.pf_of_vert[lv.elem_verts[f]]
        Kf = Ksym[f]
        add_mom(Amu, Mmu, row_m, dof_u[f], Kf)                           # viscous
        add_mom(base, Mb, row_m, dpf, -np.transpose(Bdiv[f], (0, 2, 1)))  # S_pf / F_pf
        base.add(dpf, dof_u[f], -Bdiv[f])                                # W_u
        # ALE rows, fluid-node test functions only
        if cfg.get("ale_k", 0) == 0:
            kel = 1.0 / coarse_element_volumes(cfg)[parent_coarse_element(lv)[f]]
        else:
            kel = np.ones(nF)
        rowA = np.where(np.repeat(ss, D, axis=1), -1, dof_d[f])
        base.add(rowA, dof_d[f], kel[:, None, None] * Kf)                # A_ds, A_df
        if inv_dt:
            add_time(row_m, dof_u[f], rho * inv_dt *
                     np.einsum("eab,cf->eacbf", Mq2[f], eyeD).reshape(nF, nb * D, nb * D))
        if w is not None and np.any(w != 0):
            we = w[nodes[f]]                                             # (nF, nb, D)
            wq = np.einsum("eai,qa->eqi", we, ref.phi)
            wg = np.einsum("eqi,eqai->eqa", wq, G[f])                    # w . grad phi_a
            Cm = np.einsum("eq,qa,eqb->eab", dV[f], ref.phi, wg)
            add_mom(base, Mb, row_m, dof_u[f],                           # convection
                    rho * np.einsum("eab,cf->eacbf", Cm, eyeD).reshape(nF, nb * D, nb * D))
            if cfg.get("supg", False):
                if tau is None:
                    lam = supg_lambda(ref, dV[f], G[f], H[f])
                    tau = supg_tau(lam, np.sqrt((wq ** 2).sum(axis=2)), mu, rho)
                tau_out = tau
                tw = dV[f] * tau * rho                                   # (nF, nq)
                S1 = rho * np.einsum("eq,eqa,eqb->eab", tw, wg, wg)
                if theta != 1.0 and inv_dt:     # only the steady part carries theta
                    Mb.add(row_m, dof_u[f],
                           np.einsum("eab,cf->eacbf", S1, eyeD).reshape(nF, nb * D, nb * D))
                    S1 = theta * S1
                if inv_dt:
                    S1 = S1 + rho * inv_dt * np.einsum("eq,eqa,qb->eab", tw, wg, ref.phi)
                base.add(row_m, dof_u[f],
                         np.einsum("eab,cf->eacbf", S1, eyeD).reshape(nF, nb * D, nb * D))
                if inv_dt:                    # the SUPG time term of S1, on its own
                    St = rho * inv_dt * np.einsum("eq,eqa,qb->eab", tw, wg, ref.phi)
                    Tt.add(row_m, dof_u[f],
                           np.einsum("eab,cf->eacbf", St, eyeD).reshape(nF, nb * D, nb * D))
                lap = np.einsum("eqbii->eqb", H[f])
                S2 = (np.einsum("eq,eqa,eqb,cf->eacbf", tw, wg, lap, eyeD)
                      + np.einsum("eq,eqa,eqbcf->eacbf", tw, wg, H[f]))
                add_mom(Amu, Mmu, row_m, dof_u[f], -S2.reshape(nF, nb * D, nb * D))
                Sp = np.einsum("eq,eqa,eqmc->eacm", tw, wg, Gp[f]).reshape(nF, nb * D, npv)
                add_mom(base, Mb, row_m, dpf, Sp)

    out = dict(base=base.csr(), AG=AG.csr(), AC=AC.csr(), Amu=Amu.csr(), T=Tt.csr(),
               tau=tau_out, G=Gmod, inv_lam=inv_lam, theta=theta)
    M = (Mb.csr() + Gmod * MG.csr() + mu * Mmu.csr()).tocsr()
    out["Tx"] = (out["T"] - (1.0 - theta) * M).tocsr() if theta != 1.0 else out["T"]
    out["A"] = (out["base"] + Gmod * out["AG"] + inv_lam * out["AC"]
                + mu * out["Amu"]).tocsr()
    return out


def load_vector(lv: Level, cfg: dict, fnodal: np.ndarray, w=None, tau=None):
    """Momentum right-hand side rho (f_h, phi) + SUPG rho (f_h, tau rho w.grad phi)
    for a nodal body force f (N2, D) on this level (unreduced)."""
    D, ref = lv.D, RefElement(lv.D)
    nb = ref.nb
    rho = cfg["rho"]
    Xe = lv.X[lv.elem_nodes]
    dV, G, H, Gp = geometry(ref, Xe)
    Mq2 = np.einsum("eq,qa,qb->eab", dV, ref.phi, ref.phi)
    nodes = lv.elem_nodes
    comp = np.arange(D)
    b = np.zeros(lv.N)
    fe = fnodal[nodes]                                               # (nE, nb, D)
    contrib = rho * np.einsum("eab,ebc->eac", Mq2, fe)               # (nE, nb, D)
    ss = lv.solid_side[nodes]
    solid_el = (lv.region == 1)[:, None]
    # momentum row: d-row for solid-side nodes, u-row for fluid nodes
    rows = np.where((ss | solid_el)[:, :, None], D * nodes[:, :, None] + comp,
                    lv.off_u + D * nodes[:, :, None] + comp)
    np.add.at(b, rows.ravel(), contrib.ravel())
    f = lv.region == 0
    if cfg.get("supg", False) and w is not None and np.any(w != 0) and f.any():
        we = w[nodes[f]]
        wq = np.einsum("eai,qa->eqi", we, ref.phi)
        wg = np.einsum("eqi,eqai->eqa", wq, G[f])
        if tau is None:
            lam = supg_lambda(ref, dV[f], G[f], H[f])
            tau = supg_tau(lam, np.sqrt((wq ** 2).sum(axis=2)), cfg["mu"], rho)
        fq = np.einsum("ebc,qb->eqc", fe[f], ref.phi)
        sc = rho * rho * np.einsum("eq,eq,eqa,eqc->eac", dV[f], tau, wg, fq)
        np.add.at(b, rows[f].ravel(), sc.ravel())
    return b


def dirichlet_reduce(lv: Level, A: sp.csr_matrix) -> sp.csr_matrix:
    """Symmetric elimination: Dirichlet rows and columns zeroed, unit diagonal."""
    Fm = sp.diags(lv.free.astype(np.float64))
    Dm = sp.diags(lv.dir_mask.astype(np.float64))
    Ared = (Fm @ A @ Fm + Dm).tocsr()
    Ared.eliminate_zeros()
    return Ared


def dirichlet_rhs(lv: Level, A: sp.csr_matrix, b_raw: np.ndarray) -> np.ndarray:
    """Lift: b_free - A_free,D g on free rows, g on Dirichlet rows."""
    g = np.where(lv.dir_mask, lv.dir_val, 0.0)
    b = b_raw - A @ g
    return np.where(lv.dir_mask, g, b)

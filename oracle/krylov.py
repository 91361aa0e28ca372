"""Restarted flexible GMRES, right-preconditioned, classical Gram-Schmidt twice.

The paper's outer solver is GMRES preconditioned by GMG (Section 3.2); it
fixes neither the orthogonalization nor the tolerance.  Reading used here:
FGMRES(m) (the preconditioned vectors z_j are stored, so the preconditioner
may change between applications), x0 = 0, Arnoldi by classical Gram-Schmidt
applied twice, the Hessenberg least-squares problem solved by Givens
rotations, and convergence declared when the TRUE residual
||b - A x||_2 <= rtol ||b||_2 after the Givens estimate has crossed rtol.
"""
from __future__ import annotations

import numpy as np


def fgmres(A_mv, M_apply, b, x0=None, restart=30, rtol=1e-10, max_restarts=20):
    """Return (x, info) with info = dict(converged, iters, restarts, history,
    rel_res_true).  history holds the Givens residual estimates / ||b||."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    info = dict(converged=False, iters=0, restarts=0, history=[], rel_res_true=np.nan)
    if bnorm == 0.0:
        info.update(converged=True, rel_res_true=0.0)
        return np.zeros_like(b), info
    m = int(restart)
    for cycle in range(max_restarts + 1):
        r = b - A_mv(x)
        beta = np.linalg.norm(r)
        if cycle == 0:
            info["history"].append(beta / bnorm)
        if beta <= rtol * bnorm:
            info.update(converged=True, rel_res_true=beta / bnorm)
            return x, info
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M_apply(V[j])
            w = A_mv(Z[j])
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["iters"] += 1
            k = j + 1
            est = abs(g[j + 1])
            info["history"].append(est / bnorm)
            if est <= rtol * bnorm or hn == 0.0:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        true = np.linalg.norm(b - A_mv(x)) / bnorm
        info["rel_res_true"] = true
        if true <= rtol:
            info["converged"] = True
            return x, info
        info["restarts"] += 1
    return x, info

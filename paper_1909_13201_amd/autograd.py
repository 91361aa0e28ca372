"""Differentiable solve: torch.autograd.Function around the C ABI.

    x = FSISolve.apply(f, E, mu, hierarchy, opts)

forward: b = assemble_load(f) (momentum load plus the Dirichlet lift, which
depends on mu through the fluid rows), blocks refactored when (E, mu)
changed (update_params + build_fs_as_blocks), x = gmres_solve(b).
backward, for an incoming gradient g = dL/dx:
    A^T lam = g                      (adjoint_solve: FGMRES with the
                                      transposed FS-AS V-cycle)
    dL/df  = (F L)^T lam             (load_adjoint)
    dL/dE  = -(F lam)^T dA/dE  x     (param_grad; includes the lift's
    dL/dmu = -(F lam)^T dA/dmu x      dependence, SUPG tau held fixed)
Argument marshalling only: every step runs in the library.
"""
from __future__ import annotations

import torch

from . import fsgmg


class FSISolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, E, mu, H, opts=None):
        opts = dict(opts or {})
        krylov = dict(restart=opts.pop("restart", 30), max_restarts=opts.pop("max_restarts", 20),
                      rtol=opts.pop("rtol", 1e-10))
        Ev, muv = float(E), float(mu)
        if (Ev, muv) != (float(H.cfg["E"]), float(H.cfg["mu"])) or not getattr(H, "_blocks_ok", False):
            if (Ev, muv) != (float(H.cfg["E"]), float(H.cfg["mu"])):
                H.update_params(Ev, muv)
            H.build_fs_as_blocks(**opts)
            H._blocks_ok = True
        b = torch.empty(H.N, dtype=torch.float64, device=f.device)
        H.assemble_load(f.detach().contiguous().view(-1), b)
        x = torch.empty_like(b)
        info = H.gmres_solve(b, x, **krylov)
        if not info["converged"]:
            raise RuntimeError("forward solve did not converge: %r" % info)
        ctx.H, ctx.krylov, ctx.fshape = H, krylov, f.shape
        ctx.save_for_backward(x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        H = ctx.H
        lam = torch.empty_like(x)
        info = H.adjoint_solve(gx.contiguous(), lam, **ctx.krylov)
        if not info["converged"]:
            raise RuntimeError("adjoint solve did not converge: %r" % info)
        gf = torch.empty(int(torch.tensor(ctx.fshape).prod()), dtype=torch.float64, device=x.device)
        H.load_adjoint(lam, gf)
        gE, gmu = H.param_grad(lam, x)
        dev = x.device
        return (gf.view(ctx.fshape), torch.tensor(gE, dtype=torch.float64, device=dev),
                torch.tensor(gmu, dtype=torch.float64, device=dev), None, None)

"""Differentiable solve: torch.autograd.Function around the C ABI.

    x = FSISolve.apply(f, E, mu, hierarchy, opts)

forward: the handle is brought to (E, mu) with blocks built for the smoother
options in opts (update_params and build_fs_as_blocks only when the handle
holds other parameters or blocks built with other options), b =
assemble_load(f) (momentum load plus the Dirichlet lift, which depends on mu
through the fluid rows), x = gmres_solve(b).
backward, for an incoming gradient g = dL/dx:
    A^T lam = g                      (adjoint_solve: FGMRES with the
                                      transposed FS-AS V-cycle)
    dL/df  = (F L)^T lam             (load_adjoint)
    dL/dE  = -(F lam)^T dA/dE  x     (param_grad; includes the lift's
    dL/dmu = -(F lam)^T dA/dmu x      dependence, SUPG tau held fixed)
The operator of the adjoint is the forward's: (E, mu) and the smoother
options are saved with the forward, and the handle is brought back to them
before the adjoint solve when other solves ran on it in between (several
forwards on one handle, then one backward of their summed loss).  A
re-assembly about another advecting velocity in between cannot be undone
that way: backward then raises.
Argument marshalling only: every step runs in the library.
"""
from __future__ import annotations

import torch


def _split(opts):
    opts = dict(opts or {})
    krylov = dict(restart=opts.pop("restart", 30), max_restarts=opts.pop("max_restarts", 20),
                  rtol=opts.pop("rtol", 1e-10))
    return opts, krylov


class FSISolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, E, mu, H, opts=None):
        sopts, krylov = _split(opts)
        Ev, muv = float(E), float(mu)
        H.ensure_blocks(Ev, muv, **sopts)
        b = torch.empty(H.N, dtype=torch.float64, device=f.device)
        H.assemble_load(f.detach().contiguous().view(-1), b)
        x = torch.empty_like(b)
        info = H.gmres_solve(b, x, **krylov)
        if not info["converged"]:
            raise RuntimeError("forward solve did not converge: %r" % info)
        ctx.H, ctx.krylov, ctx.fshape = H, krylov, f.shape
        ctx.params, ctx.sopts = (Ev, muv), sopts
        ctx.advection = H.advection
        ctx.save_for_backward(x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        H = ctx.H
        if H.advection != ctx.advection:
            # the operator was re-assembled about another advecting velocity
            # since the forward; the library keeps no copy of the old one
            raise RuntimeError("the hierarchy's advecting velocity changed between forward and "
                               "backward (update_advection / period_solve)")
        H.ensure_blocks(*ctx.params, **ctx.sopts)
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

"""Small hand-made problem descriptions for unit tests (same dict format as
paper_1909_13201_amd.inputs.config)."""
import numpy as np


def small(nc=(4, 4), solid_rows=(0,), levels=1, xb=None, yb=None, **kw):
    nx, ny = nc
    region = np.zeros((ny, nx), np.int8)
    for r in solid_rows:
        region[r, :] = 1
    cfg = dict(dim=2, n_levels=levels, nc=tuple(nc),
               breaks=(list(np.linspace(0, 1, nx + 1)) if xb is None else list(xb),
                       list(np.linspace(0, 1, ny + 1)) if yb is None else list(yb)),
               region=region.ravel(), mapping=0, map_params=[],
               bc_d=[[0, 0] for _ in range(6)], bc_u=[[0, 0] for _ in range(6)],
               inflow_peak=1.0, E=1e3, nu=0.3, mu=1e-2, rho=1.0, supg=False,
               w_amp=0.0, ale_k=0, k_mass=0, core=(2, 2), halo=1, nu_pre=2,
               nu_post=2, omega=1.0, restart=30, rtol=1e-10, seed=0, name="small")
    cfg.update(kw)
    return cfg


def channel3d(levels=2, nc=(2, 2, 2), **kw):
    """3D channel along x with a solid layer on y-min (hexahedral Q2/Q1):
    parabolic inflow on x-min, natural outflow on x-max, no-slip on the other
    fluid faces, solid clamped at both x ends, fluid mesh displacement fixed
    on every outer face.  E = 1e5, nu = 0.45, mu = 3.5e-3; w = 0."""
    nx, ny, nz = nc
    region = np.zeros((nz, ny, nx), np.int8)
    region[:, 0, :] = 1
    bc_d = [[1, 0] for _ in range(6)]
    bc_d[0][1] = bc_d[1][1] = 1
    bc_u = [[1, 0] for _ in range(6)]
    bc_u[0][0] = 2
    bc_u[1][0] = 0
    cfg = dict(dim=3, n_levels=levels, nc=tuple(nc),
               breaks=tuple(list(np.linspace(0, 1, n + 1)) for n in nc),
               region=region.ravel(), mapping=0, map_params=[],
               bc_d=bc_d, bc_u=bc_u, inflow_peak=1.0, E=1e5, nu=0.45, mu=3.5e-3,
               rho=1.0, supg=False, w_amp=0.0, ale_k=0, k_mass=0, core=(1, 1, 1),
               halo=1, nu_pre=2, nu_post=2, omega=0.8, restart=30, rtol=1e-10, seed=0,
               name="channel3d")
    cfg.update(kw)
    return cfg

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

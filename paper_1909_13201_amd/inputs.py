"""Seeded synthetic workloads for the FS-AS-GMG-GMRES solver.

This module only describes problems and draws random numbers: mesh shape,
material constants, boundary-condition tags, the seeded nodal body force and
the seeded advecting velocity of the Oseen linearization.  It holds none of
the solver's arithmetic (no assembly, no transfer, no smoother), so both the
CPU oracle and the GPU library can be fed from it without sharing code.

Configurations (stand-ins for the paper's aneurysm / valve meshes, which are
not public; Section 4 of the paper):

* ``c1``  2D unit square, coarse 4x4, 2 levels (finest 8x8).  Bottom coarse row
  is a linear-elastic solid (E=1e3, nu=0.3), Stokes fluid above (mu=1e-2),
  parabolic inflow, clamped bottom.  2x2-element subdomains with a one-element
  halo (the literal Vanka rule), 2 pre/post sweeps, FP64.
* ``c2``  2D straight channel, coarse 8x8 graded (walls of height 0.1 at top
  and bottom are solid, E=1e4, nu=0.45), 5 levels (finest 128x128), fluid
  mu=3.5e-3, Oseen about a seeded smooth field of amplitude 1, SUPG on,
  4x4-element subdomains.
* ``c3``  2D aneurysm-like channel with a bulge of height and half-width 0.3
  on the top wall (smooth cos^2 profile tangent to the wall), coarse 16x8,
  6 levels (finest 512x256), 2-element-thick walls, interface cores 4 x 12.
* ``c4``  3D tube along z with an elastic wall and a leaflet-like plate:
  reference box [0,1]^2 x [0,2], coarse 4x4x8, the square section mapped to
  a disc of radius 0.5, the outer coarse ring of the section solid (graded
  to 0.1 R), one thin coarse z-layer at z = 1 solid over x < 0.5 of the
  lumen (attached to the wall), 4 levels (finest 32x32x64), E=1e5,
  nu=0.45, mu=3.5e-3, Oseen about a seeded 3D field with SUPG, one-element
  cores with the one-element Vanka halo.
* ``c5``  c2 at 4 levels (finest 64x64), one backward-Euler step dt = 1/32,
  with 32 seeded (load, E, mu) samples.

``dt`` absent (or inf) means the steady problem.

Conventions shared by every consumer (a data format, not arithmetic):

* Element ``(ex, ey)`` is stored x-fastest; ``region`` is 1 for solid, 0 for
  fluid, given on the coarse mesh and inherited by refinement.
* Faces are numbered 0:x-min 1:x-max 2:y-min 3:y-max (4:z-min 5:z-max).
* ``bc_d[face][region]``: 0 natural, 1 homogeneous Dirichlet on displacement.
* ``bc_u[face][region]``: 0 natural, 1 no-slip (u=0), 2 parabolic inflow.
* The finest-level Q2 node grid has ``2*nc[a]*2**(L-1)+1`` nodes per axis,
  numbered x-fastest; nodal arrays are ``(N2, dim)`` row-major.
"""
from __future__ import annotations

import copy
import numpy as np

FACE_XMIN, FACE_XMAX, FACE_YMIN, FACE_YMAX, FACE_ZMIN, FACE_ZMAX = range(6)
MAP_IDENTITY, MAP_BULGE, MAP_SMOOTH_BULGE, MAP_DISC = 0, 1, 2, 3


def _uniform(n, lo=0.0, hi=1.0):
    return list(np.linspace(lo, hi, n + 1))


def _bc_tables():
    return [[0, 0] for _ in range(6)], [[0, 0] for _ in range(6)]


def _channel_bcs():
    """Straight channel: solid walls clamped at both ends, fluid inflow on x-min,
    natural outflow on x-max, mesh displacement fixed on fluid outer faces."""
    bc_d, bc_u = _bc_tables()
    for f in (FACE_XMIN, FACE_XMAX):
        bc_d[f][1] = 1          # solid clamped at inlet and outlet ends
        bc_d[f][0] = 1          # fluid mesh displacement fixed
    bc_u[FACE_XMIN][0] = 2      # parabolic inflow
    return bc_d, bc_u


def config(name: str) -> dict:
    """Return a fresh description of configuration ``name``."""
    if name == "c1":
        bc_d, bc_u = _bc_tables()
        bc_d[FACE_YMIN][1] = 1                      # bottom clamped
        bc_d[FACE_XMIN][0] = bc_d[FACE_XMAX][0] = bc_d[FACE_YMAX][0] = 1
        bc_u[FACE_XMIN][0] = 2                      # inflow
        bc_u[FACE_YMAX][0] = 1                      # top wall
        region = np.zeros((4, 4), np.int8)
        region[0, :] = 1
        cfg = dict(dim=2, n_levels=2, nc=(4, 4), breaks=(_uniform(4), _uniform(4)),
                   region=region.ravel(), mapping=MAP_IDENTITY, map_params=[],
                   bc_d=bc_d, bc_u=bc_u, inflow_peak=1.0,
                   E=1e3, nu=0.3, mu=1e-2, rho=1.0, supg=False, w_amp=0.0,
                   ale_k=0, k_mass=0,
                   core=(2, 2), halo=1, nu_pre=2, nu_post=2, omega=0.8,
                   restart=30, rtol=1e-10, seed=0)
    elif name in ("c2", "c5"):
        bc_d, bc_u = _channel_bcs()
        yb = [0.0] + list(np.linspace(0.1, 0.9, 7)) + [1.0]
        region = np.zeros((8, 8), np.int8)
        region[0, :] = 1
        region[7, :] = 1
        cfg = dict(dim=2, n_levels=5, nc=(8, 8), breaks=(_uniform(8), yb),
                   region=region.ravel(), mapping=MAP_IDENTITY, map_params=[],
                   bc_d=bc_d, bc_u=bc_u, inflow_peak=1.0,
                   E=1e4, nu=0.45, mu=3.5e-3, rho=1.0, supg=True, w_amp=1.0,
                   ale_k=0, k_mass=0,
                   core=(4, 4), halo=1, nu_pre=2, nu_post=2, omega=0.8,
                   restart=30, rtol=1e-10, seed=0)
        if name == "c5":
            cfg["n_levels"] = 4
            cfg["batch"] = 32
            # one backward-Euler step of the time-periodic problem (32 steps per
            # period, Section 4): makes u^s = dd/dt so the outlet flux depends on
            # the wall stiffness (the steady problem is one-way coupled)
            cfg["dt"] = 1.0 / 32.0
            # samples pair E = 1e5 with mu = 1e-3: ||A|| ||x|| / ||b|| reaches ~1e6,
            # so an FP64 iterate cannot push the relative residual much below
            # 1e-10 (rounding of x alone); 1e-9 is attainable for every sample
            cfg["rtol"] = 1e-9
    elif name == "c3":
        bc_d, bc_u = _channel_bcs()
        yb = [0.0, 0.05, 0.1, 0.3, 0.5, 0.7, 0.9, 0.95, 1.0]
        region = np.zeros((8, 16), np.int8)
        region[0:2, :] = 1
        region[6:8, :] = 1
        cfg = dict(dim=2, n_levels=6, nc=(16, 8), breaks=(_uniform(16, 0.0, 2.0), yb),
                   # bulge of height / half-width 0.3 with a profile tangent to
                   # the straight wall (the circular one, MAP_BULGE, meets the
                   # wall vertically and its elements shear without bound
                   # under refinement)
                   region=region.ravel(), mapping=MAP_SMOOTH_BULGE,
                   # bulge centre x, radius, blend start y, blend end y
                   map_params=[1.0, 0.3, 0.5, 0.9],
                   bc_d=bc_d, bc_u=bc_u, inflow_peak=1.0,
                   E=1e4, nu=0.45, mu=3.5e-3, rho=1.0, supg=True, w_amp=1.0,
                   ale_k=0, k_mass=0,
                   core=(4, 4), halo=1, nu_pre=2, nu_post=2, omega=0.8,
                   # interface cores 4 x 12 elements: uneven blocks, the
                   # enlarged ones about 2x the unknowns of the interior ones
                   iface_mult=3,
                   restart=30, rtol=1e-10, seed=0)
    elif name == "c4":
        # tube along z: solid ring clamped at both ends, fluid inflow on
        # z-min, natural outflow on z-max, fluid mesh displacement fixed on
        # the end faces; the outer surface of the ring is traction-free
        bc_d, bc_u = _bc_tables()
        for f in (FACE_ZMIN, FACE_ZMAX):
            bc_d[f][1] = 1
            bc_d[f][0] = 1
        bc_u[FACE_ZMIN][0] = 2
        sec = [0.0, 0.125, 0.5, 0.875, 1.0]        # wall ring a quarter of the radius
        zb = [0.0, 0.25, 0.5, 0.75, 0.975, 1.025, 1.35, 1.675, 2.0]
        region = np.zeros((8, 4, 4), np.int8)      # (z, y, x), x fastest
        region[:, 0, :] = region[:, 3, :] = 1
        region[:, :, 0] = region[:, :, 3] = 1
        region[4, 1:3, 1] = 1                      # leaflet: z in [0.975, 1.025], x < 0.5
        cfg = dict(dim=3, n_levels=4, nc=(4, 4, 8), breaks=(sec, list(sec), zb),
                   region=region.ravel(), mapping=MAP_DISC, map_params=[0.5, 0.5, 0.5],
                   bc_d=bc_d, bc_u=bc_u, inflow_peak=1.0,
                   E=1e5, nu=0.45, mu=3.5e-3, rho=1.0, supg=True, w_amp=1.0,
                   ale_k=0, k_mass=0,
                   # in 3D only the literal Vanka rule (one-element cores
                   # with the one-element halo) converges
                   core=(1, 1, 1), halo=1, nu_pre=2, nu_post=2, omega=0.8,
                   restart=30, rtol=1e-10, seed=0)
    else:
        raise KeyError(name)
    cfg["name"] = name
    return cfg


def with_levels(cfg: dict, n_levels: int) -> dict:
    """Copy of ``cfg`` with a different number of levels (same coarse mesh)."""
    out = copy.deepcopy(cfg)
    out["n_levels"] = int(n_levels)
    return out


# ----------------------------------------------------------------------------
# finest-grid index helpers (pure bookkeeping)
# ----------------------------------------------------------------------------

def finest_elems(cfg: dict) -> tuple:
    s = 2 ** (cfg["n_levels"] - 1)
    return tuple(int(n) * s for n in cfg["nc"])


def finest_nodes_shape(cfg: dict) -> tuple:
    return tuple(2 * n + 1 for n in finest_elems(cfg))


def n_finest_nodes(cfg: dict) -> int:
    return int(np.prod(finest_nodes_shape(cfg)))


def _refined_breaks(b, times):
    b = np.asarray(b, float)
    for _ in range(times):
        mid = 0.5 * (b[:-1] + b[1:])
        out = np.empty(2 * len(b) - 1)
        out[0::2] = b
        out[1::2] = mid
        b = out
    return b


def finest_node_reference_coords(cfg: dict) -> list:
    """Per-axis reference coordinates of the finest Q2 node lines."""
    return [_refined_breaks(cfg["breaks"][a], cfg["n_levels"])
            for a in range(cfg["dim"])]


# ----------------------------------------------------------------------------
# seeded random inputs
# ----------------------------------------------------------------------------

def body_force(cfg: dict, seed: int | None = None) -> np.ndarray:
    """Nodal body force f ~ U[-1,1]^dim at every finest Q2 node, shape (N2, dim)."""
    rng = np.random.default_rng(cfg["seed"] if seed is None else seed)
    return rng.uniform(-1.0, 1.0, size=(n_finest_nodes(cfg), cfg["dim"]))


def _fluid_box(cfg: dict):
    """Reference-coordinate bounding box of the fluid region, per axis."""
    nc = cfg["nc"]
    D = cfg["dim"]
    reg = np.asarray(cfg["region"]).reshape(tuple(nc[a] for a in reversed(range(D))))
    fluid = reg == 0
    box = []
    for a in range(D):
        ax = D - 1 - a                              # numpy axis of reference axis a
        other = tuple(i for i in range(D) if i != ax)
        idx = np.where(fluid.any(axis=other))[0]
        b = cfg["breaks"][a]
        box.append((b[idx.min()], b[idx.max() + 1]))
    return tuple(box)


def _nodes_touching_solid(cfg: dict) -> np.ndarray:
    """Finest Q2 nodes that belong to at least one solid element, (N2,) bool."""
    D = cfg["dim"]
    s = 2 ** (cfg["n_levels"] - 1)
    nc = cfg["nc"]
    reg = np.asarray(cfg["region"]).reshape(tuple(nc[a] for a in reversed(range(D))))
    fine = reg
    for ax in range(D):
        fine = np.repeat(fine, s, axis=ax)            # finest elements, (z,) y, x
    solid = fine == 1
    ne = solid.shape
    out = np.zeros(tuple(2 * n + 1 for n in ne), bool)
    for off in np.ndindex(*(3,) * D):
        sl = tuple(slice(o, o + 2 * n, 2) for o, n in zip(off, ne))
        out[sl] |= solid
    return out.ravel()


def advecting_field(cfg: dict, seed: int | None = None) -> np.ndarray | None:
    """Seeded smooth advecting velocity w at every finest Q2 node, shape (N2, dim).

    w = (d psi/dt, -d psi/ds) with psi = (t(1-t))^2 sum_{k,l<=3} a_kl sin(k pi s)
    sin(l pi t), a_kl ~ N(0,1), where (s, t) are the reference coordinates
    normalised to the fluid box.  w vanishes outside the open fluid box (so on
    the fluid-solid interface) and is scaled to max |w|_2 = w_amp.  Returns
    None when w_amp == 0.
    """
    if not cfg.get("w_amp", 0.0):
        return None
    if cfg["dim"] == 3:
        return _advecting_field_3d(cfg, seed)
    rng = np.random.default_rng(1000 + (cfg["seed"] if seed is None else seed))
    a = rng.standard_normal((3, 3))
    (x0, x1), (y0, y1) = _fluid_box(cfg)
    xr, yr = finest_node_reference_coords(cfg)
    X, Y = np.meshgrid(xr, yr, indexing="xy")          # (ny, nx): x fastest
    s = (X - x0) / (x1 - x0)
    t = (Y - y0) / (y1 - y0)
    inside = (s > 0) & (s < 1) & (t > 0) & (t < 1)
    B = (t * (1 - t)) ** 2
    dB = 2 * t * (1 - t) * (1 - 2 * t)
    S = np.zeros_like(s)
    dS_ds = np.zeros_like(s)
    dS_dt = np.zeros_like(s)
    for k in range(1, 4):
        for l in range(1, 4):
            sk, ck = np.sin(k * np.pi * s), np.cos(k * np.pi * s)
            sl, cl = np.sin(l * np.pi * t), np.cos(l * np.pi * t)
            S += a[k - 1, l - 1] * sk * sl
            dS_ds += a[k - 1, l - 1] * k * np.pi * ck * sl
            dS_dt += a[k - 1, l - 1] * l * np.pi * sk * cl
    wx = dB * S + B * dS_dt
    wy = -B * dS_ds
    wx = np.where(inside, wx, 0.0)
    wy = np.where(inside, wy, 0.0)
    w = np.stack([wx.ravel(), wy.ravel()], axis=1)
    mx = np.sqrt((w ** 2).sum(axis=1)).max()
    return w * (cfg["w_amp"] / mx)


def _advecting_field_3d(cfg: dict, seed: int | None = None) -> np.ndarray:
    """Seeded smooth 3D advecting velocity at every finest Q2 node, (N2, 3).

    With (s, t, q) the reference coordinates normalised to the fluid box,
    w = (d psi/dt, -d psi/ds, phi): a swirl from the stream function
    psi = (s(1-s))^2 (t(1-t))^2 (1 + sin(pi q)/2) sum_{k,l<=3} a_kl
    sin(k pi s) sin(l pi t), a_kl ~ N(0,1), plus the axial profile
    phi = 16 s(1-s) t(1-t); both are divergence-free in (s, t, q).  w is
    zero outside the open fluid box and at every node of a solid element
    (the wall and the leaflet), and scaled to max |w|_2 = w_amp."""
    rng = np.random.default_rng(1000 + (cfg["seed"] if seed is None else seed))
    a = rng.standard_normal((3, 3))
    (x0, x1), (y0, y1), (z0, z1) = _fluid_box(cfg)
    xr, yr, zr = finest_node_reference_coords(cfg)
    Z, Y, X = np.meshgrid(zr, yr, xr, indexing="ij")     # x fastest after ravel
    s = (X - x0) / (x1 - x0)
    t = (Y - y0) / (y1 - y0)
    q = (Z - z0) / (z1 - z0)
    inside = (s > 0) & (s < 1) & (t > 0) & (t < 1) & (q >= 0) & (q <= 1)
    Bs, dBs = (s * (1 - s)) ** 2, 2 * s * (1 - s) * (1 - 2 * s)
    Bt, dBt = (t * (1 - t)) ** 2, 2 * t * (1 - t) * (1 - 2 * t)
    g = 1.0 + 0.5 * np.sin(np.pi * q)
    S = np.zeros_like(s)
    dS_ds = np.zeros_like(s)
    dS_dt = np.zeros_like(s)
    for k in range(1, 4):
        for l in range(1, 4):
            sk, ck = np.sin(k * np.pi * s), np.cos(k * np.pi * s)
            sl, cl = np.sin(l * np.pi * t), np.cos(l * np.pi * t)
            S += a[k - 1, l - 1] * sk * sl
            dS_ds += a[k - 1, l - 1] * k * np.pi * ck * sl
            dS_dt += a[k - 1, l - 1] * l * np.pi * sk * cl
    w_s = g * Bs * (dBt * S + Bt * dS_dt)
    w_t = -g * Bt * (dBs * S + Bs * dS_ds)
    w_q = 16.0 * s * (1 - s) * t * (1 - t)
    w = np.stack([w_s.ravel(), w_t.ravel(), w_q.ravel()], axis=1)
    w[~inside.ravel()] = 0.0
    w[_nodes_touching_solid(cfg)] = 0.0
    mx = np.sqrt((w ** 2).sum(axis=1)).max()
    return w * (cfg["w_amp"] / mx)


def sample_parameters(cfg: dict, batch: int, seed: int | None = None):
    """Log-uniform (E, mu) pairs in [1e3,1e5] x [1e-3,1e-1], shape (batch, 2)."""
    rng = np.random.default_rng(2000 + (cfg["seed"] if seed is None else seed))
    logE = rng.uniform(3.0, 5.0, size=batch)
    logmu = rng.uniform(-3.0, -1.0, size=batch)
    return np.stack([10.0 ** logE, 10.0 ** logmu], axis=1)


def sample_loads(cfg: dict, batch: int, seed: int | None = None) -> np.ndarray:
    """Batch of nodal body forces, shape (batch, N2, dim)."""
    base = cfg["seed"] if seed is None else seed
    return np.stack([body_force(cfg, seed=base + 100 + i) for i in range(batch)])

"""Benchmark of the FS-AS-GMG-FGMRES solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]

A step is one full solve of A x = b to a true relative residual of 1e-10
(FGMRES(30) right-preconditioned by one V-cycle per iteration: finest-level
operator products, CGS2 dot products, Givens updates, and in the V-cycle the
residual products, the FS-AS smoother sweeps, restriction, the coarse FP64
solve and prolongation on every level), with the hierarchy and the block
factors built before the timed region and b resident on the GPU.  `value` is
solves/s of the mixed-precision path (FP32 smoother and level operators, FP64
Krylov, outer products and coarse solve); the FP64 path, V-cycles/s, the
setup times, one adjoint solve, the roofline of the dominant kernel (the
finest-level smoother sweep, timed with HIP events on the library's stream
in a separate pass of three solves, since the timed solves run as HIP graphs)
and the CPU oracle's time are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s to 1e-10 rel. residual, mixed vs FP64 FS-AS-GMG-GMRES; V-cycles/s"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c5": "differentiation: 2D channel of c2 at 4 levels (64x64 finest), one backward-Euler "
          "step dt=1/32, batch of 32 seeded loads and (E, mu) log-uniform in "
          "[1e3,1e5] x [1e-3,1e-1]",
    "c2": "2D straight channel, coarse 8x8 graded -> finest 128x128 Q2/Q1 (5 levels, "
          "281,095 unknowns), solid walls E=1e4 nu=0.45, fluid mu=3.5e-3, Oseen about a "
          "seeded field of amplitude 1 with SUPG, FS-AS on 4x4-element cores with the "
          "one-element Vanka halo, 2+2 sweeps",
    "c1": "2D unit square, coarse 4x4 -> 8x8 (2 levels), solid bottom row, Stokes fluid",
    "c3": "2D aneurysm-like channel with a smooth bulge of height 0.3 on the top wall, coarse 16x8 -> 512x256 (6 levels, 2,236,167 unknowns), 2-element walls, 4x4 interior and 4x12 interface cores",
    "c4": "3D tube along z, square section mapped to a disc of radius 0.5, elastic ring (E=1e5, "
          "nu=0.45) and a leaflet-like plate over half the lumen at z=1, fluid mu=3.5e-3, Oseen "
          "about a seeded 3D field with SUPG, hexahedral Q2/Q1, coarse 4x4x8, one-element cores "
          "with the one-element Vanka halo",
}
# workloads with the several-load, comparator and multiplicative legs (the
# 3D tube's monolithic blocks exceed one workgroup's LDS, and its extras
# would take minutes)
EXTRAS = ("c1", "c2", "c3")


def smoother_bytes(H, level, prec):
    """Algorithmic bytes of one FS-AS sweep on `level`: owned rows of every
    block inverse (n_j x m_j values), the gather / scatter index lists, and
    the residual read plus the correction read and write (one pass each)."""
    from paper_1909_13201_amd import fsgmg
    ptr, dofs, owner = fsgmg.export_blocks(H.h, level)
    n = np.diff(ptr)
    own = owner[owner >= 0]
    m = np.bincount(own, minlength=len(n))
    sW = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    sV = 8 if prec == "fp64" else 4
    N = H.info[level]["N"]
    return int((n * m).sum() * sW + 4 * (n.sum() + m.sum()) + 3 * N * sV), int(len(n))


MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 157.3}   # dense; BF16 inverses run FP32 MFMA


def mc_smoother_model(H, level, prec, K):
    """One K-column block apply on `level`: algorithmic bytes (owned rows of
    every inverse once, index lists, K columns of residual read and
    correction read + write) and matrix-core flops (2 n_j m_j K per block)."""
    from paper_1909_13201_amd import fsgmg
    ptr, dofs, owner = fsgmg.export_blocks(H.h, level)
    n = np.diff(ptr)
    m = np.bincount(owner[owner >= 0], minlength=len(n))
    sW = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    sV = 8 if prec == "fp64" else 4
    N = H.info[level]["N"]
    nbytes = int((n * m).sum() * sW + 4 * (n.sum() + m.sum()) + 3 * N * K * sV)
    flops = int(2 * (n * m).sum() * K)
    return nbytes, flops


def mrhs_solves(H, cfg, K, steps, rtol, dev):
    """FGMRES on K seeded loads at once (gmres_solve_batch): solves/s over all
    columns, iterations and the worst true relative residual."""
    import torch
    from paper_1909_13201_amd import inputs
    Bm = torch.zeros((H.N, K), dtype=torch.float64, device=dev)
    bc = torch.zeros(H.N, dtype=torch.float64, device=dev)
    for c in range(K):
        f = inputs.body_force(cfg, seed=1000 + c)
        H.assemble_load(torch.tensor(f.ravel(), dtype=torch.float64, device=dev), bc)
        Bm[:, c] = bc
    Xm = torch.zeros_like(Bm)
    H.gmres_solve_batch(Bm, Xm, rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = H.gmres_solve_batch(Bm, Xm, rtol=rtol)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    check_converged(infos, rtol, "%d-load batch" % K)
    return dict(solves_per_s=round(K * steps / t, 2), ms_per_call=round(1e3 * t / steps, 3),
                iters_max=max(i["iters"] for i in infos), iters_min=min(i["iters"] for i in infos),
                all_converged=all(i["converged"] for i in infos),
                worst_rel_res_true=max(i["rel_res_true"] for i in infos))


def mrhs_measure(H, K, calls, prec, dev):
    """K-column cycles: calls/s, column-cycles/s and the finest-level block
    apply (HIP events on the handle stream) against HBM and matrix-core peaks."""
    import torch
    R = torch.randn((H.N, K), dtype=torch.float64, device=dev)
    Z = torch.zeros_like(R)
    for _ in range(2):
        H.vcycle_apply_batch(R, Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        H.vcycle_apply_batch(R, Z)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    H.kernel_timing(True)
    for _ in range(3):
        H.vcycle_apply_batch(R, Z)
    torch.cuda.synchronize()
    kt = H.kernel_timing(False)
    n_l, ms_l = kt["smoother"]
    us = 1e3 * ms_l / max(n_l, 1)
    nbytes, flops = mc_smoother_model(H, H.L - 1, prec, K)
    gbs = nbytes / (us * 1e-6) / 1e9
    tfl = flops / (us * 1e-6) / 1e12
    return dict(calls_per_s=round(calls / t, 2), column_cycles_per_s=round(K * calls / t, 1),
                block_apply=dict(kernel="k_smooth_mc (finest level)", launches=n_l,
                                 avg_us=round(us, 2), bytes_per_launch=nbytes,
                                 flops_per_launch=flops, achieved_gbs=round(gbs, 1),
                                 hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                                 achieved_tflops=round(tfl, 2),
                                 mfma_frac=round(tfl / MFMA_PEAK_TFLOPS[prec], 4)))


def _units(info):
    """Node-block unit of every unknown: a Q2 node's dim components of d (or
    u) form one unit, each pressure is its own unit."""
    N, N2, Nps, D = info["N"], info["N2"], info["Nps"], info["dim"]
    i = np.arange(N)
    unit = np.empty(N, np.int64)
    d = i < info["off_ps"]
    ps = (i >= info["off_ps"]) & (i < info["off_u"])
    u = (i >= info["off_u"]) & (i < info["off_pf"])
    pf = i >= info["off_pf"]
    unit[d] = i[d] // D
    unit[ps] = N2 + i[ps] - info["off_ps"]
    unit[u] = N2 + Nps + (i[u] - info["off_u"]) // D
    unit[pf] = 2 * N2 + Nps + i[pf] - info["off_pf"]
    return unit, int(unit.max()) + 1


def _unit_pairs(M, urow, ucol, ncol):
    r = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    return int(np.unique(urow[r] * ncol + ucol[M.indices]).size)


def operator_bytes(H, level, sv, nvec):
    """Algorithmic bytes of one level-operator product: every stored value,
    one 4-byte column index per nonzero node block (dim x dim, dim x 1, 1 x dim
    or scalar), one row pointer per unit row, and nvec vector passes (x, b, y)."""
    A = H.csr(level, 0)
    unit, nu = _units(H.info[level])
    return int(A.nnz * sv + 4 * _unit_pairs(A, unit, unit, nu) + 4 * nu
               + nvec * H.info[level]["N"] * sv)


def transfer_bytes(H, level, sv):
    """Mean algorithmic bytes of the restriction to level-1 and the
    prolongation from it: the node-weight entries (shared by the dim
    components; 4-byte index + value), the pressure entries, the input read
    and the output write (read + write for the prolongation's update)."""
    uf, nf = _units(H.info[level])
    uc, nc = _units(H.info[level - 1])
    Nf, Nc = H.info[level]["N"], H.info[level - 1]["N"]
    R, P = H.csr(level, 2), H.csr(level, 1)
    br = _unit_pairs(R, uc, uf, nf) * (4 + sv) + Nf * sv + Nc * sv
    bp = _unit_pairs(P, uf, uc, nc) * (4 + sv) + Nc * sv + 2 * Nf * sv
    return int((br + bp) / 2)


def copy_ceiling(dev, nbytes=1 << 30, reps=5):
    """Streaming ceiling measured on the device: bytes read plus bytes written
    per second by torch's device-to-device copy of `nbytes` (median of
    `reps`, HIP events on torch's stream, which runs the copy)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / sorted(ts)[reps // 2] / 1e9


def read_ceiling(H, nbytes=1 << 30, reps=7):
    """Read-only streaming ceiling measured on the device by the library
    (stream_read_ceiling: 16-byte loads over `nbytes` by 2,048 workgroups,
    median of `reps`, HIP events).  The smoother sweep reads far more than it
    writes, so this, not a read-plus-write copy, is the ceiling it is held
    against."""
    return H.stream_read_ceiling(nbytes, reps)


def kernel_fracs(H, ktime, prec):
    """Per-kernel HBM rates of the finest level from a kernel_timing record:
    the smoother sweep, the V-cycle residual product, the outer FP64 product
    and the transfers, each against its algorithmic bytes."""
    sv = 8 if prec == "fp64" else 4
    fin = H.L - 1
    sm_bytes, nblk = smoother_bytes(H, fin, prec)
    model = dict(smoother=("k_smooth_fwd (finest level)", sm_bytes),
                 vspmv=("k_spmv residual, finest", operator_bytes(H, fin, sv, 3)),
                 outer_spmv=("k_spmv<double> outer product, finest", operator_bytes(H, fin, 8, 2)),
                 transfer=("k_transfer restriction / prolongation, finest",
                           transfer_bytes(H, fin, sv)))
    out = {}
    for k, (name, nbytes) in model.items():
        n, ms = ktime[k]
        us = ms * 1e3 / max(n, 1)
        gbs = nbytes / (us * 1e-6) / 1e9 if n else 0.0
        out[k] = dict(kernel=name, launches=n, avg_us=round(us, 2), bytes_per_launch=nbytes,
                      achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def c3_legs(args, dev):
    """The aneurysm-like workload (c3, 2.2 M unknowns, working set far beyond
    the 256 MB Infinity Cache): FP64, FP32 and BF16-factor solves/s and the
    finest-level kernels' HBM rates, GPU legs only (the oracle is timed on
    c2).  Returned as the `c3` object of the c2 line."""
    import torch
    from paper_1909_13201_amd import fsgmg, inputs
    cfg = inputs.config("c3")
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    rtol = cfg["rtol"]
    steps = max(3, args.steps // 2)
    t0 = time.perf_counter()
    H = fsgmg.Hierarchy(cfg, w, device=0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    b = torch.zeros(H.N, dtype=torch.float64, device=dev)
    H.assemble_load(torch.tensor(f.ravel(), dtype=torch.float64, device=dev), b)
    out = dict(workload=WORKLOADS["c3"], unknowns=H.N, levels=H.L, steps=steps,
               setup_hierarchy_s=round(t_setup, 3))
    sps = {}
    for prec in ("fp64", "fp32", "bf16"):
        H.build_fs_as_blocks(prec=prec)
        x = torch.zeros_like(b)
        t, infos = timed_solves(H, b, x, steps, 1, rtol, "c3 " + prec)
        sps[prec] = steps / t
        leg = dict(solves_per_s=round(sps[prec], 4), iters=infos[-1]["iters"],
                   rel_res_true=infos[-1]["rel_res_true"])
        if prec != "fp64":
            H.kernel_timing(True)
            H.gmres_solve(b, x, restart=30, rtol=rtol)
            torch.cuda.synchronize()
            leg["kernels"] = kernel_fracs(H, H.kernel_timing(False), prec)
        out[prec] = leg
    out["mixed_over_fp64"] = round(sps["fp32"] / sps["fp64"], 3)
    out["bf16_over_fp64"] = round(sps["bf16"] / sps["fp64"], 3)
    H.close()
    torch.cuda.empty_cache()
    return out


PICARD_MAX, PICARD_TOL = 6, 1e-5


def progress(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_loop_leg(args, dev):
    """The time-periodic outer loop (Sections 2.2 and 4): backward-Euler
    steps of the pulsatile problem (inflow factor 1 + 0.75 sin 2 pi t, dt =
    1/32: 32 steps a period) from rest on the differentiation workload's
    channel, each time step by Picard steps (re-assembly about the latest
    velocity, block refactorization, FGMRES with FP32 inverses) until the
    iterate changes by less than 1e-5 (at most 6).  Section 4's N, rho and
    s^max and the
    split of the wall time.  Returned as the `time_loop` object."""
    import torch
    from paper_1909_13201_amd import fsgmg, inputs
    cfg = inputs.config("c5")
    n2, dim = inputs.n_finest_nodes(cfg), cfg["dim"]
    f = inputs.body_force(cfg)
    H = fsgmg.Hierarchy(cfg, np.zeros((n2, dim)), device=0)
    try:
        H.build_fs_as_blocks(prec="fp32")
        x = torch.zeros(H.N, dtype=torch.float64, device=dev)
        fd = torch.tensor(f.ravel(), dtype=torch.float64, device=dev)
        res = H.period_solve(fd, x, steps=args.period_steps, picard_max=PICARD_MAX,
                             picard_tol=PICARD_TOL, rtol=1e-10)
        out = dict(workload="2D channel of c2 at 4 levels (64x64 finest Q2/Q1), E=1e4, nu=0.45, "
                            "mu=3.5e-3, backward-Euler dt=1/32 from rest, pulsatile inflow, Picard "
                            "re-linearization of convection and SUPG",
                   unknowns=H.N, levels=H.L, dt=cfg["dt"], steps=res["steps"],
                   picard_max=PICARD_MAX, picard_tol=PICARD_TOL, inflow_amp=0.75,
                   converged=res["converged"],
                   N=round(res["N"], 3), rho=round(res["rho"], 4), s_max=round(res["s_max"], 3),
                   solves=res["solves"], max_iters=res["max_iters"],
                   steps_per_s=round(res["steps"] / (1e-3 * res["t_total_ms"]), 3),
                   t_total_s=round(1e-3 * res["t_total_ms"], 3),
                   t_assemble_s=round(1e-3 * res["t_assemble_ms"], 3),
                   t_factor_s=round(1e-3 * res["t_factor_ms"], 3),
                   t_solve_s=round(1e-3 * res["t_solve_ms"], 3),
                   iters_per_step=[[int(v) for v in row if v >= 0] for row in res["iters"]])
    finally:
        H.close()
        torch.cuda.empty_cache()
    # the time-step study of Section 4 (t_step steps per period): the first
    # quarter period at other step sizes
    study = {}
    for t_step in (16, 64):
        c = dict(cfg, dt=1.0 / t_step)
        Hs = fsgmg.Hierarchy(c, np.zeros((n2, dim)), device=0)
        try:
            Hs.build_fs_as_blocks(prec="fp32")
            xs = torch.zeros(Hs.N, dtype=torch.float64, device=dev)
            r = Hs.period_solve(fd, xs, steps=t_step // 4, picard_max=PICARD_MAX,
                                picard_tol=PICARD_TOL, rtol=1e-10)
            study[str(t_step)] = dict(steps=r["steps"], N=round(r["N"], 3), rho=round(r["rho"], 4),
                                      s_max=round(r["s_max"], 3), max_iters=r["max_iters"],
                                      converged=r["converged"])
        finally:
            Hs.close()
            torch.cuda.empty_cache()
    out["dt_study"] = study
    # the paper's comparator inside the loop: the monolithic AS blocks
    # (Section 3.2), the first quarter period, against FS on the same steps
    cmp = {}
    for name, mono in (("fs", False), ("as", True)):
        Ha = fsgmg.Hierarchy(cfg, np.zeros((n2, dim)), device=0)
        try:
            Ha.build_fs_as_blocks(prec="fp32", monolithic=mono)
            xa = torch.zeros(Ha.N, dtype=torch.float64, device=dev)
            r = Ha.period_solve(fd, xa, steps=8, picard_max=PICARD_MAX, picard_tol=PICARD_TOL,
                                rtol=1e-10)
            cmp[name] = dict(N=round(r["N"], 3), rho=round(r["rho"], 4), s_max=round(r["s_max"], 3),
                             converged=r["converged"],
                             factor_s=round(1e-3 * r["t_factor_ms"], 3),
                             solve_s=round(1e-3 * r["t_solve_ms"], 3))
        finally:
            Ha.close()
            torch.cuda.empty_cache()
    out["fs_vs_as_quarter_period"] = cmp
    # Crank-Nicolson for the momentum balance (theta = 1/2), the paper's
    # scheme: the first quarter period
    c = dict(cfg, theta=0.5)
    Hc = fsgmg.Hierarchy(c, np.zeros((n2, dim)), device=0)
    try:
        Hc.build_fs_as_blocks(prec="fp32")
        xc = torch.zeros(Hc.N, dtype=torch.float64, device=dev)
        r = Hc.period_solve(fd, xc, steps=8, picard_max=PICARD_MAX, picard_tol=PICARD_TOL,
                            rtol=1e-10)
        out["crank_nicolson"] = dict(steps=r["steps"], N=round(r["N"], 3), rho=round(r["rho"], 4),
                                     s_max=round(r["s_max"], 3), max_iters=r["max_iters"],
                                     converged=r["converged"])
    finally:
        Hc.close()
        torch.cuda.empty_cache()
    return out


def measured_traffic():
    """HBM bytes per launch of the finest-level smoother from the committed
    rocprofv3 counter summary, or None when kernels.hip has changed since the
    counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "k_smooth_fwd_c2_traffic.md")
    src = os.path.join(ROOT, "paper_1909_13201_amd", "csrc", "kernels.hip")
    try:
        txt = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in txt.splitlines()
                if l.startswith(("kernels_hip_sha256:", "traffic_bytes_per_launch:")))
    if vals.get("kernels_hip_sha256", "").strip() != sha:
        return None
    return int(vals["traffic_bytes_per_launch"])


class SolveFailed(RuntimeError):
    """A timed solve did not reach the tolerance: no throughput is reported."""


def check_converged(infos, rtol, what):
    """Every timed solve must have converged with a true relative residual
    <= rtol, else the line would count solves that are not solves."""
    bad = [i for i in infos if not i["converged"] or not (i["rel_res_true"] <= rtol)]
    if bad:
        raise SolveFailed("%s: %d of %d timed solves missed rtol %.1e (first: %r)"
                          % (what, len(bad), len(infos), rtol,
                             {k: bad[0][k] for k in ("converged", "iters", "rel_res_true")}))


def timed_solves(H, b, x, steps, warmup, rtol, what="solve"):
    import torch
    infos = []
    for _ in range(warmup):
        H.gmres_solve(b, x, restart=30, rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(H.gmres_solve(b, x, restart=30, rtol=rtol))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    check_converged(infos, rtol, what)
    return t, infos


def cpu_baseline(cfg, w, f):
    """The oracle as it stands: one full FGMRES solve of the same workload on
    the host (hierarchy and LU factors built first, untimed), once with the
    BLAS pools held to one thread (the reported value) and once with the
    host's default pools (SciPy's sparse products stay single-threaded)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.krylov import fgmres
    from oracle.multigrid import Hierarchy as OracleHierarchy
    t0 = time.perf_counter()
    O = OracleHierarchy(cfg, w)
    t_setup = time.perf_counter() - t0
    b = O.rhs(f)
    A = O.A[-1]

    def solve():
        t0 = time.perf_counter()
        _, info = fgmres(lambda v: A @ v, O.vcycle, b, restart=30, rtol=cfg["rtol"])
        return time.perf_counter() - t0, info

    with threadpool_limits(limits=1):
        t, info = solve()
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    t_all, _ = solve()
    return dict(value=1.0 / t, unit="solves/s", cores=1, kind="oracle",
                sample="one full FGMRES(30) solve of the same %s workload to 1e-10 "
                       "(%d iterations, %.1f s; hierarchy and block LUs built "
                       "beforehand in %.1f s, untimed), NumPy/SciPy FP64, one thread"
                       % (cfg["name"], info["iters"], t, t_setup),
                default_threads=dict(value=round(1.0 / t_all, 4), blas_threads=threads))


def grad_bench(cfg, args):
    """Differentiation workload: the batch of seeded (f, E, mu) samples through
    FSISolve (forward: update_params + build_fs_as_blocks + assemble_load +
    gmres_solve; backward: adjoint_solve + load_adjoint + param_grad), once
    with FP64 block inverses and once with FP32 ones.  Accuracy against the
    oracle's gradients is checked by the GPU tests; here: throughput and the
    FP32 / FP64 agreement of every gradient.  J = sum of the outlet
    x-velocities (a linear functional of the solution)."""
    import torch
    from paper_1909_13201_amd import fsgmg, inputs
    from paper_1909_13201_amd.autograd import FSISolve
    batch = int(cfg.get("batch", 32))
    w = inputs.advecting_field(cfg)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    dev = torch.device("cuda:0")
    params = inputs.sample_parameters(cfg, batch)
    loads = inputs.sample_loads(cfg, batch)
    # J = sum of the x-velocities on the outlet face (x = max, node lines x-fastest)
    nx = inputs.finest_nodes_shape(cfg)[0]
    fin = H.info[-1]
    outlet = np.arange(nx - 1, fin["N2"], nx)
    cnp = np.zeros(H.N)
    cnp[fin["off_u"] + fin["dim"] * outlet] = 1.0
    c = torch.tensor(cnp, device=dev)
    rng = np.random.default_rng(7)
    probe = torch.tensor(rng.standard_normal(loads[0].size), device=dev)

    def one(i, prec):
        f = torch.tensor(loads[i].ravel(), dtype=torch.float64, device=dev, requires_grad=True)
        E = torch.tensor(float(params[i][0]), dtype=torch.float64, requires_grad=True)
        mu = torch.tensor(float(params[i][1]), dtype=torch.float64, requires_grad=True)
        x = FSISolve.apply(f, E, mu, H, dict(prec=prec, rtol=cfg["rtol"]))
        J = (c * x).sum()
        J.backward()
        return (float(J.detach()), float(E.grad), float(mu.grad), float((f.grad * probe).sum()))

    res, out = {}, {}
    for prec in ("fp64", "fp32"):
        one(0, prec)                                   # warm-up: plan, graphs, tuning
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res[prec] = [one(i, prec) for i in range(batch)]
        torch.cuda.synchronize()
        out[prec] = batch / (time.perf_counter() - t0)
    a, b = np.array(res["fp64"]), np.array(res["fp32"])
    rel = np.abs(a - b) / np.maximum(np.abs(a), 1e-300)

    # the same loads on one operator (E, mu of sample 0): one K-column forward
    # solve, one adjoint solve (J's gradient in x is c for every load, so one
    # lambda serves all), the shared load adjoint, and each load's parameter
    # gradients; sample 0 checked against its per-sample result above
    E0, mu0 = float(params[0][0]), float(params[0][1])
    Fm = torch.tensor(np.stack([l.ravel() for l in loads]), dtype=torch.float64, device=dev)

    def shared():
        H.update_params(E0, mu0)
        H.build_fs_as_blocks(prec="fp32")
        Bm = torch.empty((H.N, batch), dtype=torch.float64, device=dev)
        bc = torch.empty(H.N, dtype=torch.float64, device=dev)
        for i in range(batch):
            H.assemble_load(Fm[i].contiguous(), bc)
            Bm[:, i] = bc
        Xm = torch.zeros_like(Bm)
        infos = H.gmres_solve_batch(Bm, Xm, rtol=cfg["rtol"])
        lam = torch.empty(H.N, dtype=torch.float64, device=dev)
        ainfo = H.adjoint_solve(c, lam, rtol=cfg["rtol"])
        gf = torch.empty(Fm.shape[1], dtype=torch.float64, device=dev)
        H.load_adjoint(lam, gf)
        Js = (c[:, None] * Xm).sum(0)
        grads = [H.param_grad(lam, Xm[:, i].contiguous()) for i in range(batch)]
        torch.cuda.synchronize()
        ok = all(i_["converged"] for i_ in infos) and ainfo["converged"]
        return Js, grads, gf, ok

    shared()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Js, grads, gf, ok = shared()
    t_sh = time.perf_counter() - t0
    got0 = np.array([float(Js[0]), grads[0][0], grads[0][1], float((gf * probe).sum())])
    ref0 = np.array(res["fp32"][0])
    shared_line = dict(samples_per_s=round(batch / t_sh, 2),
                       over_per_sample=round((batch / t_sh) / out["fp32"], 2),
                       all_converged=bool(ok),
                       sample0_max_rel_diff=float((np.abs(got0 - ref0) /
                                                   np.maximum(np.abs(ref0), 1e-300)).max()))
    # the per-sample pipeline (the same library calls FSISolve makes) on a
    # pool of handles, one host thread and stream each, so that independent
    # samples overlap on the device; checked against the FSISolve results
    from paper_1909_13201_amd.pool import HandlePool

    def pipeline(Hk, i):
        Hk.update_params(float(params[i][0]), float(params[i][1]))
        Hk.build_fs_as_blocks(prec="fp32")
        fi = torch.tensor(loads[i].ravel(), dtype=torch.float64, device=dev)
        bi = torch.empty(Hk.N, dtype=torch.float64, device=dev)
        Hk.assemble_load(fi, bi)
        xi = torch.empty_like(bi)
        inf_f = Hk.gmres_solve(bi, xi, rtol=cfg["rtol"])
        lam = torch.empty_like(xi)
        inf_a = Hk.adjoint_solve(c, lam, rtol=cfg["rtol"])
        gf = torch.empty(fi.numel(), dtype=torch.float64, device=dev)
        Hk.load_adjoint(lam, gf)
        gE, gmu = Hk.param_grad(lam, xi)
        if not (inf_f["converged"] and inf_a["converged"]):
            raise RuntimeError("sample %d did not converge" % i)
        return (float((c * xi).sum()), gE, gmu, float((gf * probe).sum()))

    pools = {}
    ref32 = np.array(res["fp32"])
    hw_queues = os.environ.get("GPU_MAX_HW_QUEUES", "4")   # the runtime's hardware queues
    for n in (2, 4, 8):
        with HandlePool(cfg, w, n=n, device=0) as pool:
            torch.cuda.synchronize()
            pool.map(pipeline, range(n))               # warm-up: tuning and graphs per handle
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = np.array(pool.map(pipeline, range(batch)))
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
        pools[str(n)] = dict(samples_per_s=round(batch / tp, 2),
                             over_per_sample=round((batch / tp) / out["fp32"], 2),
                             max_rel_diff=float((np.abs(got - ref32) /
                                                 np.maximum(np.abs(ref32), 1e-300)).max()))
    line = dict(metric="differentiated solves/s (forward + adjoint + gradients, blocks refactored per sample)",
                value=round(out["fp32"], 3), unit="samples/s", n_gpus=1, steps=batch, warmup=1,
                ms_per_step=round(1e3 / out["fp32"], 3), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32 smoother + f64 Krylov", data="synthetic",
                config=dict(workload=WORKLOADS.get(cfg["name"], cfg["name"]), name=cfg["name"],
                            levels=int(cfg["n_levels"]), unknowns=H.N, batch=batch),
                fp64_samples_per_s=round(out["fp64"], 3),
                max_rel_diff_fp32_vs_fp64=dict(J=float(rel[:, 0].max()), dJ_dE=float(rel[:, 1].max()),
                                               dJ_dmu=float(rel[:, 2].max()),
                                               dJ_df_probe=float(rel[:, 3].max())),
                shared_operator=shared_line,
                handle_pool=dict(hw_queues=int(hw_queues), **pools))
    H.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--levels", type=int, default=0, help="override the number of levels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-stored block inverses")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the aneurysm-like c3 legs that the default c2 run adds")
    ap.add_argument("--period-steps", type=int, default=32,
                    help="time steps of the time-loop leg (32 = one period)")
    ap.add_argument("--no-time-loop", action="store_true", help="skip the time-loop leg")
    ap.add_argument("--cycle", default="V", choices=["V", "W", "F"], help="multigrid cycle")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run three plain 256 MiB device copies first (counter calibration)")
    ap.add_argument("--mrhs", type=int, default=0,
                    help="only time K-column cycles (vcycle_apply_batch) with this K, FP32")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1909_13201_amd import fsgmg, inputs

    cfg = inputs.config(args.config)
    if args.levels:
        cfg = inputs.with_levels(cfg, args.levels)
    cfg["cycle"] = args.cycle
    if cfg.get("batch"):
        grad_bench(cfg, args)
        return
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    rtol = cfg["rtol"]
    dev = torch.device("cuda:0")

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    H = fsgmg.Hierarchy(cfg, w, device=0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    b = torch.zeros(H.N, dtype=torch.float64, device=dev)
    H.assemble_load(torch.tensor(f.ravel(), dtype=torch.float64, device=dev), b)
    x64 = torch.zeros_like(b)
    x32 = torch.zeros_like(b)

    if args.mrhs:
        H.build_fs_as_blocks(prec="fp32")
        m = mrhs_measure(H, args.mrhs, max(5, args.steps), "fp32", dev)
        ba = m["block_apply"]
        line = dict(metric="K-column V-cycles (one operator, K right-hand sides)",
                    value=m["column_cycles_per_s"], unit="column-cycles/s", n_gpus=1,
                    steps=max(5, args.steps), warmup=2, ms_per_step=round(1e3 / m["calls_per_s"], 3),
                    higher_is_better=True, scaling="weak", vs_baseline=None,
                    dtype="f32 (FP32 matrix cores)", data="synthetic",
                    config=dict(workload=WORKLOADS.get(cfg["name"], cfg["name"]), name=cfg["name"],
                                levels=int(cfg["n_levels"]), unknowns=H.N, K=args.mrhs),
                    calls_per_s=m["calls_per_s"],
                    roofline=dict(bound="mfma", kernel=ba["kernel"], achieved=ba["achieved_tflops"],
                                  peak=MFMA_PEAK_TFLOPS["fp32"], unit="TFLOP/s",
                                  frac=ba["mfma_frac"], traffic=None,
                                  hbm_gbs=ba["achieved_gbs"], hbm_frac=ba["hbm_frac"],
                                  avg_launch_us=ba["avg_us"], launches=ba["launches"],
                                  bytes_per_launch=ba["bytes_per_launch"],
                                  flops_per_launch=ba["flops_per_launch"]))
        H.close()
        print(json.dumps(line), flush=True)
        return
    res = {}

    def refactor_s(prec):
        # the paper's regime refactors the blocks before every solve: a rebuild
        # with the same options and index sets is the refactorization alone
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H.build_fs_as_blocks(prec=prec)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[1]

    # ---- plain FP64 path ----
    t0 = time.perf_counter()
    H.build_fs_as_blocks(prec="fp64")
    torch.cuda.synchronize()
    t_blocks64 = time.perf_counter() - t0
    progress("%s: FP64 and mixed solves" % cfg["name"])
    t64, inf64 = timed_solves(H, b, x64, args.steps, args.warmup, rtol)
    t_ref64 = refactor_s("fp64")
    # ---- mixed FP32 path (the reported value) ----
    t0 = time.perf_counter()
    H.build_fs_as_blocks(prec="fp32")
    torch.cuda.synchronize()
    t_blocks32 = time.perf_counter() - t0
    t32, inf32 = timed_solves(H, b, x32, args.steps, args.warmup, rtol)
    t_ref32 = refactor_s("fp32")
    # kernel durations for the roofline: a separate pass with HIP events
    # around the launches (graphs are bypassed while events are recorded).
    # The autotuner may give the finest level the fused sweep form, whose
    # launch also forms the block residual rows; the roofline holds the
    # sweep kernel the byte model describes (the SpMV form's k_smooth_fwd),
    # so this pass forces that form and then restores the tuned one.
    H.build_fs_as_blocks(prec="fp32", sweep_form="spmv")
    tfin = H.tuning_info()[-1]      # launch shape of the timed finest sweep
    H.kernel_timing(True)
    for _ in range(3):
        H.gmres_solve(b, x32, restart=30, rtol=rtol)
    torch.cuda.synchronize()
    ktime = H.kernel_timing(False)
    H.build_fs_as_blocks(prec="fp32")
    # V-cycles/s (mixed)
    r = b / b.norm()
    z = torch.zeros_like(b)
    for _ in range(3):
        H.vcycle_apply(r, z)
    torch.cuda.synchronize()
    nv = max(20, 5 * args.steps)
    t0 = time.perf_counter()
    for _ in range(nv):
        H.vcycle_apply(r, z)
    torch.cuda.synchronize()
    tv = time.perf_counter() - t0
    # several right-hand sides on the same operator (vcycle_apply_batch):
    # K columns per call, column-cycles/s against the one-column cycles/s
    mrhs = {}
    for K in ((8, 32, 64) if cfg["name"] in EXTRAS else ()):
        mrhs[str(K)] = mrhs_measure(H, K, max(5, args.steps), "fp32", dev)
        mrhs[str(K)]["over_one_column"] = round(mrhs[str(K)]["column_cycles_per_s"] / (nv / tv), 2)
    # FGMRES on K loads at once against one-load solves
    msol = {}
    for K in ((8, 32) if cfg["name"] in EXTRAS else ()):
        msol[str(K)] = mrhs_solves(H, cfg, K, max(2, args.steps // 3), rtol, dev)
        msol[str(K)]["over_one_load"] = round(msol[str(K)]["solves_per_s"] / (args.steps / t32), 2)
    # adjoint solve (mixed)
    c = torch.zeros_like(b)
    fi = H.info[-1]
    c[fi["off_u"]:fi["off_u"] + fi["dim"] * fi["N2"]:fi["dim"]] = 1.0
    lam = torch.zeros_like(b)
    H.adjoint_solve(c, lam, rtol=rtol)      # first call builds the transposed operators
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ainfo = H.adjoint_solve(c, lam, rtol=rtol)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    bf = None
    if not args.no_bf16:
        H.build_fs_as_blocks(prec="bf16")
        xb = torch.zeros_like(b)
        try:
            tb, infb = timed_solves(H, b, xb, args.steps, 1, rtol, "bf16")
            bf = dict(solves_per_s=round(args.steps / tb, 4), iters=infb[-1]["iters"],
                      rel_res_true=infb[-1]["rel_res_true"],
                      over_fp64=round((args.steps / tb) / (args.steps / t64), 3))
        except SolveFailed as e:   # BF16 inverses too coarse for this workload
            bf = dict(not_converged=str(e))
        H.build_fs_as_blocks(prec="fp32")

    x64h = x64.double()
    rel_diff = float((x32 - x64h).norm() / x64h.norm())
    sm_bytes, nblk = smoother_bytes(H, H.L - 1, "fp32")
    # launch grid (threads) of the finest sweep, which names it in a kernel trace
    _, _, owner_f = fsgmg.export_blocks(H.h, H.L - 1)
    njac_f = int((owner_f < 0).sum())
    wg = abs(tfin["smooth_threads"]) or (1024 if nblk < 1024 else 256)
    grid_f = (nblk * max(1, tfin["split"]) + (njac_f + wg - 1) // wg) * wg
    n_sm, ms_sm = ktime["smoother"]
    avg_ms = ms_sm / max(n_sm, 1)
    achieved = sm_bytes / (avg_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", kernel="k_smooth_fwd<float,float> (finest level)",
                achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic() if cfg["name"] == "c2" and not args.levels else None,
                bytes_per_launch=sm_bytes, blocks_per_launch=nblk, grid_threads=grid_f,
                avg_launch_us=round(avg_ms * 1e3, 2), launches=n_sm)
    ceil = copy_ceiling(dev)
    roof["copy_ceiling_gbs"] = round(ceil, 1)
    roof["frac_of_copy"] = round(achieved / ceil, 4)
    rceil = read_ceiling(H)
    roof["read_ceiling_gbs"] = round(rceil, 1)
    roof["frac_of_read"] = round(achieved / rceil, 4)
    # the other HBM-bound kernels of the path, same live HIP-event timing
    fin = H.L - 1
    model = dict(vspmv=("k_spmv<float> residual, finest", operator_bytes(H, fin, 4, 3)),
                 outer_spmv=("k_spmv<double> outer product, finest", operator_bytes(H, fin, 8, 2)),
                 transfer=("k_transfer<float> restriction / prolongation, finest",
                           transfer_bytes(H, fin, 4)))
    other = {}
    for k in ("vspmv", "outer_spmv", "transfer"):
        n, ms = ktime[k]
        us = ms * 1e3 / max(n, 1)
        name, nbytes = model[k]
        gbs = nbytes / (us * 1e-6) / 1e9 if n else 0.0
        other[k] = dict(kernel=name, launches=n, avg_us=round(us, 2), bytes_per_launch=nbytes,
                        achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))

    sps32 = args.steps / t32
    sps64 = args.steps / t64
    out = dict(metric=METRIC, value=round(sps32, 4), unit="solves/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup,
               ms_per_step=round(1e3 * t32 / args.steps, 3), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32 smoother + f64 Krylov",
               data="synthetic",
               config=dict(workload=WORKLOADS.get(cfg["name"], cfg["name"]),
                           name=cfg["name"], levels=int(cfg["n_levels"]), unknowns=H.N,
                           core=list(cfg["core"]), halo=cfg["halo"], cycle=cfg["cycle"],
                           restart=30, rtol=rtol),
               fp64_solves_per_s=round(sps64, 4), mixed_over_fp64=round(sps32 / sps64, 3),
               vcycles_per_s=round(nv / tv, 2), multi_rhs_vcycles=mrhs, multi_rhs_solves=msol,
               iters_mixed=inf32[-1]["iters"],
               iters_fp64=inf64[-1]["iters"], rel_res_true_mixed=inf32[-1]["rel_res_true"],
               rel_res_true_fp64=inf64[-1]["rel_res_true"], rel_diff_mixed_vs_fp64=rel_diff,
               setup_hierarchy_s=round(t_setup, 3), build_blocks_fp64_s=round(t_blocks64, 3),
               build_blocks_fp32_s=round(t_blocks32, 3),
               with_refactor=dict(refactor_fp32_s=round(t_ref32, 4), refactor_fp64_s=round(t_ref64, 4),
                                  solves_per_s=round(1.0 / (t32 / args.steps + t_ref32), 3),
                                  fp64_solves_per_s=round(1.0 / (t64 / args.steps + t_ref64), 3)),
               adjoint=dict(seconds=round(t_adj, 4), iters=ainfo["iters"],
                            rel_res_true=ainfo["rel_res_true"]),
               kernels=other, tuning=H.tuning_info(), roofline=roof)
    if bf is not None:
        out["bf16_factors"] = bf
    # the paper's comparator: monolithic Vanka blocks over d, u, p (no field
    # split), everything else identical
    progress("comparator")
    comp = {}
    if cfg["name"] not in EXTRAS:
        comp = dict(not_run="not run for the 3D tube (monolithic blocks of several thousand unknowns)")
    else:
        # each precision on its own: FP64 monolithic blocks can exceed one
        # workgroup's LDS where FP32 ones still fit
        for prec in ("fp64", "fp32"):
            try:
                t0 = time.perf_counter()
                H.build_fs_as_blocks(prec=prec, monolithic=True)
                torch.cuda.synchronize()
                tb = time.perf_counter() - t0
                xa = torch.zeros_like(b)
                ta, infa = timed_solves(H, b, xa, args.steps, args.warmup, rtol)
                comp[prec] = dict(solves_per_s=round(args.steps / ta, 4), iters=infa[-1]["iters"],
                                  rel_res_true=infa[-1]["rel_res_true"],
                                  build_blocks_s=round(tb, 3))
                ptr, _, _ = fsgmg.export_blocks(H.h, H.L - 1)
                comp["max_block"] = int(np.diff(ptr).max())
            except (fsgmg.FsgmgError, SolveFailed) as e:
                comp[prec] = dict(not_run=str(e))
        for prec, t in (("fp32", t32), ("fp64", t64)):
            if "solves_per_s" in comp[prec]:
                comp["fs_over_as_" + prec] = round((args.steps / t) / comp[prec]["solves_per_s"], 3)

    out["comparator_as"] = comp
    # multicolour multiplicative Schwarz (the within-process variant of
    # Section 3.2): same blocks, colour by colour on the latest residual
    progress("multiplicative")
    mult = {}
    try:
        if cfg["name"] not in EXTRAS:
            raise SolveFailed("not run for the 3D tube")
        for prec in ("fp64", "fp32"):
            t0 = time.perf_counter()
            H.build_fs_as_blocks(prec=prec, schwarz="multiplicative")
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
            xm = torch.zeros_like(b)
            tm, infm = timed_solves(H, b, xm, args.steps, args.warmup, rtol)
            mult[prec] = dict(solves_per_s=round(args.steps / tm, 4), iters=infm[-1]["iters"],
                              rel_res_true=infm[-1]["rel_res_true"], build_blocks_s=round(tb, 3))
        mult["colours_per_level"] = [int(fsgmg.block_colours(H.h, l).size - 1)
                                     for l in range(1, H.L)]
        mult["mult_over_add_fp32"] = round(mult["fp32"]["solves_per_s"] / (args.steps / t32), 3)
        mult["mult_over_add_fp64"] = round(mult["fp64"]["solves_per_s"] / (args.steps / t64), 3)
    except (fsgmg.FsgmgError, SolveFailed) as e:
        mult = dict(not_run=str(e))
    out["multiplicative"] = mult
    # the interchanged cascade (the paper's future work: GMRES preconditioned
    # by the field split, each diagonal block by one GMG cycle on it)
    progress("interchange")
    inter = {}
    try:
        for prec in ("fp64", "fp32"):
            t0 = time.perf_counter()
            H.build_fs_as_blocks(prec=prec, interchange=True)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
            xi = torch.zeros_like(b)
            ti, infi = timed_solves(H, b, xi, args.steps, args.warmup, rtol)
            inter[prec] = dict(solves_per_s=round(args.steps / ti, 4), iters=infi[-1]["iters"],
                               rel_res_true=infi[-1]["rel_res_true"], build_blocks_s=round(tb, 3))
        inter["over_standard_fp32"] = round(inter["fp32"]["solves_per_s"] / (args.steps / t32), 3)
        inter["iters_standard"] = inf32[-1]["iters"]
        H.build_fs_as_blocks(prec="fp32")
    except (fsgmg.FsgmgError, SolveFailed) as e:
        inter = dict(not_run=str(e))
    out["interchange"] = inter
    if cfg["name"] == "c2" and not args.levels and not args.no_c3:
        H.close()
        torch.cuda.empty_cache()
        progress("c3 legs")
        out["c3"] = c3_legs(args, dev)
    if cfg["name"] == "c2" and not args.levels and not args.no_time_loop:
        progress("time loop")
        out["time_loop"] = time_loop_leg(args, dev)
    if not args.no_cpu_baseline and (cfg["name"] != "c4" or cfg["n_levels"] <= 2):
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(cfg, w, f)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    try:
        main()
    except SolveFailed as e:
        print(json.dumps(dict(metric=METRIC, value=None, unit="solves/s", n_gpus=1,
                              failed=str(e))), flush=True)
        sys.exit(1)

"""Thin ctypes binding of libfsgmg.so (argument marshalling only).

Module-level functions carry the C-ABI names (setup_hierarchy,
build_fs_as_blocks, vcycle_apply, gmres_solve, adjoint_solve, assemble_load,
apply_operator, param_grad, update_params, ...); ``Hierarchy`` wraps a handle.
Device vectors are torch CUDA (HIP) tensors of dtype float64; every compute
step runs inside the library.  The library is loaded from this directory and
the import fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsgmg.so")

FSGMG_OK, FSGMG_NOT_CONVERGED = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EHIP", -3: "ESINGULAR",
          -4: "ENOMEM", -5: "ESTATE"}
CYCLE = {"V": 0, "W": 1, "F": 2}
SCHWARZ = {"additive": 0, "multiplicative": 1}
SWEEP_FORM = {"auto": 0, "spmv": 1, "fused": 2}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}

EXPORTED = ["setup_hierarchy", "build_fs_as_blocks", "vcycle_apply", "vcycle_apply_batch",
            "gmres_solve", "gmres_solve_batch", "adjoint_solve_batch",
            "adjoint_solve", "assemble_load", "load_adjoint", "apply_operator", "param_grad",
            "param_grad_noalloc",
            "update_params", "update_advection", "time_rhs", "period_solve", "level_info", "dof_map", "debug_zero_block", "export_csr", "export_vector", "export_blocks", "block_colours",
            "kernel_timing", "stream_read_ceiling", "tuning_info", "last_error",
            "hierarchy_destroy"]


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_levels", C.c_int), ("nc", C.c_int * 3),
                ("breaks", C.POINTER(C.c_double) * 3), ("region", C.POINTER(C.c_int8)),
                ("mapping", C.c_int), ("map_params", C.c_double * 8),
                ("bc_d", (C.c_int8 * 2) * 6), ("bc_u", (C.c_int8 * 2) * 6),
                ("inflow_peak", C.c_double)]


class Physics(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("mu", C.c_double),
                ("rho", C.c_double), ("dt", C.c_double), ("supg", C.c_int),
                ("ale_k", C.c_int), ("k_mass", C.c_int), ("w", C.POINTER(C.c_double)),
                ("theta", C.c_double)]


class SmootherOpts(C.Structure):
    _fields_ = [("core", C.c_int * 3), ("halo", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("omega", C.c_double), ("prec", C.c_int),
                ("use_graph", C.c_int), ("iface_mult", C.c_int), ("monolithic", C.c_int),
                ("cycle", C.c_int), ("schwarz", C.c_int), ("sweep_form", C.c_int),
                ("interchange", C.c_int)]


class KrylovOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_restarts", C.c_int), ("rtol", C.c_double)]


class PeriodOpts(C.Structure):
    _fields_ = [("steps", C.c_int), ("t0", C.c_double), ("picard_max", C.c_int),
                ("picard_tol", C.c_double), ("inflow_amp", C.c_double)]


class PeriodInfo(C.Structure):
    _fields_ = [("steps", C.c_int), ("solves", C.c_int), ("max_iters", C.c_int),
                ("N", C.c_double), ("rho", C.c_double), ("s_max", C.c_double),
                ("t_assemble_ms", C.c_double), ("t_factor_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("t_total_ms", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("rel_res_true", C.c_double), ("history", C.POINTER(C.c_double)),
                ("history_cap", C.c_int), ("history_len", C.c_int),
                ("t_solve_ms", C.c_double), ("vcycles", C.c_int),
                ("t_setup_ms", C.c_double), ("t_blocks_ms", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """The handle's device memory from torch's caching allocator on `device`:
    every buffer the library allocates is a block of torch's pool on the
    handle's stream.  The ctypes callbacks live as long as this object, which
    the owning Hierarchy keeps; `allocs` / `frees` count the calls."""

    def __init__(self, device):
        import torch
        self.device = int(device)
        self.allocs = self.frees = 0
        self.live = {}

        def _alloc(nbytes, stream, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:   # noqa: BLE001 - out of memory: NULL tells the library
                return None
            self.allocs += 1
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, stream, user):
            try:
                self.live.pop(ptr, None)
                self.frees += 1
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:   # noqa: BLE001 - interpreter shutdown
                pass

        self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
        self.struct = Allocator(self._cb[0], self._cb[1], None)


_lib = None


def lib():
    """Load libfsgmg.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfsgmg.so is not built: run "
                               "`python -m paper_1909_13201_amd.build` first")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        P = C.c_void_p
        sig = {
            "setup_hierarchy": ([C.POINTER(MeshDesc), C.POINTER(Physics), C.POINTER(Allocator),
                                 C.c_int, P, C.POINTER(H)], C.c_int),
            "build_fs_as_blocks": ([H, C.POINTER(SmootherOpts)], C.c_int),
            "vcycle_apply": ([H, P, P, C.c_int], C.c_int),
            "vcycle_apply_batch": ([H, P, P, C.c_int, C.c_int], C.c_int),
            "gmres_solve_batch": ([H, P, P, C.c_int, C.POINTER(KrylovOpts), P], C.c_int),
            "adjoint_solve_batch": ([H, P, P, C.c_int, C.POINTER(KrylovOpts), P], C.c_int),
            "gmres_solve": ([H, P, P, C.POINTER(KrylovOpts), C.POINTER(SolveInfo)], C.c_int),
            "adjoint_solve": ([H, P, P, C.POINTER(KrylovOpts), C.POINTER(SolveInfo)], C.c_int),
            "assemble_load": ([H, P, P], C.c_int),
            "load_adjoint": ([H, P, P], C.c_int),
            "apply_operator": ([H, C.c_int, P, P, C.c_int], C.c_int),
            "param_grad": ([H, P, P, C.POINTER(C.c_double)], C.c_int),
            "param_grad_noalloc": ([H, P, P, C.POINTER(C.c_double)], C.c_int),
            "update_params": ([H, C.c_double, C.c_double], C.c_int),
            "update_advection": ([H, P], C.c_int),
            "time_rhs": ([H, P, C.c_double, P, P], C.c_int),
            "period_solve": ([H, C.POINTER(PeriodOpts), C.POINTER(KrylovOpts), P, P, P, P,
                              C.POINTER(PeriodInfo)], C.c_int),
            "level_info": ([H, C.c_int, C.POINTER(C.c_int64)], C.c_int),
            "dof_map": ([H, C.c_int, C.POINTER(C.c_int64), P, P, P, P], C.c_int),
            "debug_zero_block": ([H, C.c_int, C.c_int64], C.c_int),
            "export_csr": ([H, C.c_int, C.c_int, C.POINTER(C.c_int64), P, P, P], C.c_int),
            "export_vector": ([H, C.c_int, C.c_int, P], C.c_int),
            "export_blocks": ([H, C.c_int, C.POINTER(C.c_int64), P, P, P], C.c_int),
            "block_colours": ([H, C.c_int, C.POINTER(C.c_int64), P], C.c_int),
            "kernel_timing": ([H, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
                              C.c_int),
            "tuning_info": ([H, C.c_int, C.POINTER(C.c_int32)], C.c_int),
            "stream_read_ceiling": ([H, C.c_int64, C.c_int, C.POINTER(C.c_double)], C.c_int),
            "last_error": ([H], C.c_char_p),
            "hierarchy_destroy": ([H], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class FsgmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def _ptr(t):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _mesh_desc(cfg, keep):
    m = MeshDesc()
    m.dim = int(cfg["dim"])
    m.n_levels = int(cfg["n_levels"])
    for a in range(3):
        m.nc[a] = int(cfg["nc"][a]) if a < m.dim else 1
    for a in range(m.dim):
        arr = np.ascontiguousarray(np.asarray(cfg["breaks"][a], dtype=np.float64))
        keep.append(arr)
        m.breaks[a] = arr.ctypes.data_as(C.POINTER(C.c_double))
    reg = np.ascontiguousarray(np.asarray(cfg["region"], dtype=np.int8))
    keep.append(reg)
    m.region = reg.ctypes.data_as(C.POINTER(C.c_int8))
    m.mapping = int(cfg["mapping"])
    for i, v in enumerate(cfg.get("map_params", [])):
        m.map_params[i] = float(v)
    for f in range(6):
        for r in range(2):
            m.bc_d[f][r] = int(cfg["bc_d"][f][r])
            m.bc_u[f][r] = int(cfg["bc_u"][f][r])
    m.inflow_peak = float(cfg["inflow_peak"])
    return m


def _physics(cfg, w, keep):
    p = Physics()
    p.E, p.nu, p.mu, p.rho = float(cfg["E"]), float(cfg["nu"]), float(cfg["mu"]), float(cfg["rho"])
    p.dt = float(cfg.get("dt", float("inf")))
    p.supg = int(bool(cfg.get("supg", False)))
    p.ale_k = int(cfg.get("ale_k", 0))
    p.k_mass = int(cfg.get("k_mass", 0))
    p.theta = float(cfg.get("theta", 1.0))
    if w is not None:
        arr = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        keep.append(arr)
        p.w = arr.ctypes.data_as(C.POINTER(C.c_double))
    return p


def _check(h, st, allow_not_converged=False):
    if st == FSGMG_OK or (allow_not_converged and st == FSGMG_NOT_CONVERGED):
        return st
    msg = lib().last_error(h).decode() if h else ""
    raise FsgmgError(st, msg)


# ----------------------------------------------------------------------------
# C-ABI named wrappers
# ----------------------------------------------------------------------------

def setup_hierarchy(cfg, w=None, device=0, stream=None, allocator=None):
    """allocator: an Allocator structure (or an object with a `struct`
    attribute holding one) for the handle's device memory, None = hipMalloc.
    It must outlive the handle."""
    keep = []
    m = _mesh_desc(cfg, keep)
    p = _physics(cfg, w, keep)
    h = C.c_void_p()
    s = C.c_void_p(stream) if stream is not None else None
    a = getattr(allocator, "struct", allocator)
    st = lib().setup_hierarchy(C.byref(m), C.byref(p), C.byref(a) if a is not None else None,
                               int(device), s, C.byref(h))
    if st != FSGMG_OK:
        msg = lib().last_error(h).decode() if h else ""
        if h:
            lib().hierarchy_destroy(h)
        raise FsgmgError(st, msg)
    return h


def build_fs_as_blocks(h, core=(4, 4), halo=1, nu_pre=2, nu_post=2, omega=0.8, prec="fp64",
                       use_graph=True, iface_mult=1, monolithic=False, cycle="V",
                       schwarz="additive", sweep_form="auto", interchange=False):
    o = SmootherOpts()
    for a in range(3):
        o.core[a] = int(core[a]) if a < len(core) else 1
    o.halo, o.nu_pre, o.nu_post = int(halo), int(nu_pre), int(nu_post)
    o.omega = float(omega)
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.use_graph = int(bool(use_graph))
    o.iface_mult = int(iface_mult)
    o.monolithic = int(bool(monolithic))
    o.cycle = CYCLE[cycle] if isinstance(cycle, str) else int(cycle)
    o.schwarz = SCHWARZ[schwarz] if isinstance(schwarz, str) else int(schwarz)
    o.sweep_form = SWEEP_FORM[sweep_form] if isinstance(sweep_form, str) else int(sweep_form)
    o.interchange = int(bool(interchange))
    _check(h, lib().build_fs_as_blocks(h, C.byref(o)))


def vcycle_apply(h, r, z, transpose=False):
    _check(h, lib().vcycle_apply(h, _ptr(r), _ptr(z), int(bool(transpose))))


def vcycle_apply_batch(h, r, z, k, transpose=False):
    _check(h, lib().vcycle_apply_batch(h, _ptr(r), _ptr(z), int(k), int(bool(transpose))))


def _solve(fn, h, b, x, restart, max_restarts, rtol, history_cap):
    o = KrylovOpts(int(restart), int(max_restarts), float(rtol))
    info = SolveInfo()
    hist = np.zeros(max(1, history_cap))
    info.history = hist.ctypes.data_as(C.POINTER(C.c_double))
    info.history_cap = int(history_cap)
    st = fn(h, _ptr(b), _ptr(x), C.byref(o), C.byref(info))
    _check(h, st, allow_not_converged=True)
    n = min(info.history_len, history_cap)
    return dict(converged=bool(info.converged), iters=info.iters, restarts=info.restarts,
                rel_res_true=info.rel_res_true, history=hist[:n].copy(),
                t_solve_ms=info.t_solve_ms, vcycles=info.vcycles, t_setup_ms=info.t_setup_ms,
                t_blocks_ms=info.t_blocks_ms, status=STATUS[st])


def _solve_batch(fn, h, b, x, k, restart, max_restarts, rtol):
    o = KrylovOpts(int(restart), int(max_restarts), float(rtol))
    infos = (SolveInfo * int(k))()
    st = fn(h, _ptr(b), _ptr(x), int(k), C.byref(o), C.cast(infos, C.c_void_p))
    _check(h, st, allow_not_converged=True)
    return [dict(converged=bool(i.converged), iters=i.iters, restarts=i.restarts,
                 rel_res_true=i.rel_res_true, t_solve_ms=i.t_solve_ms, vcycles=i.vcycles)
            for i in infos]


def gmres_solve_batch(h, b, x, k, restart=30, max_restarts=20, rtol=1e-10):
    return _solve_batch(lib().gmres_solve_batch, h, b, x, k, restart, max_restarts, rtol)


def adjoint_solve_batch(h, c, lam, k, restart=30, max_restarts=20, rtol=1e-10):
    return _solve_batch(lib().adjoint_solve_batch, h, c, lam, k, restart, max_restarts, rtol)


def gmres_solve(h, b, x, restart=30, max_restarts=20, rtol=1e-10, history_cap=1024):
    return _solve(lib().gmres_solve, h, b, x, restart, max_restarts, rtol, history_cap)


def adjoint_solve(h, c, lam, restart=30, max_restarts=20, rtol=1e-10, history_cap=1024):
    return _solve(lib().adjoint_solve, h, c, lam, restart, max_restarts, rtol, history_cap)


def assemble_load(h, f, b):
    _check(h, lib().assemble_load(h, _ptr(f), _ptr(b)))


def load_adjoint(h, lam, gf):
    _check(h, lib().load_adjoint(h, _ptr(lam), _ptr(gf)))


def apply_operator(h, level, x, y, transpose=False):
    _check(h, lib().apply_operator(h, int(level), _ptr(x), _ptr(y), int(bool(transpose))))


def param_grad(h, lam, x):
    out = (C.c_double * 2)()
    _check(h, lib().param_grad(h, _ptr(lam), _ptr(x), out))
    return float(out[0]), float(out[1])


def update_params(h, E, mu):
    _check(h, lib().update_params(h, float(E), float(mu)))


def level_info(h, level):
    out = (C.c_int64 * 9)()
    _check(h, lib().level_info(h, int(level), out))
    keys = ["N", "N2", "Nps", "Npf", "off_ps", "off_u", "off_pf", "nnz", "dim"]
    return {k: int(v) for k, v in zip(keys, out)}


FIELDS = ("d", "ps", "u", "pf")


def debug_zero_block(h, level, block):
    """Test hook: the next build_fs_as_blocks zeroes that block's matrix
    (it then reports ESINGULAR); block < 0 clears the hook."""
    _check(h, lib().debug_zero_block(h, int(level), int(block)))


def dof_map(h, level):
    """Per unknown of `level`: field code (0 d, 1 p^s, 2 u, 3 p^f), component,
    Q2 node or Q1 vertex index, physical coordinates (N x 3)."""
    n = C.c_int64(0)
    _check(h, lib().dof_map(h, int(level), C.byref(n), None, None, None, None))
    N = n.value
    field = np.zeros(N, np.int32)
    comp = np.zeros(N, np.int32)
    node = np.zeros(N, np.int32)
    xyz = np.zeros((N, 3))
    _check(h, lib().dof_map(h, int(level), C.byref(n), field.ctypes.data_as(C.c_void_p),
                            comp.ctypes.data_as(C.c_void_p), node.ctypes.data_as(C.c_void_p),
                            xyz.ctypes.data_as(C.c_void_p)))
    return field, comp, node, xyz


def export_csr(h, level, which):
    """Host copy of a setup matrix as (rowptr, col, val, shape)."""
    dims = (C.c_int64 * 3)()
    _check(h, lib().export_csr(h, int(level), int(which), dims, None, None, None))
    nr, nc, nnz = int(dims[0]), int(dims[1]), int(dims[2])
    rp = np.zeros(nr + 1, np.int64)
    col = np.zeros(max(nnz, 1), np.int32)
    val = np.zeros(max(nnz, 1), np.float64)
    _check(h, lib().export_csr(h, int(level), int(which), dims, rp.ctypes.data_as(C.c_void_p),
                               col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p)))
    return rp, col[:nnz], val[:nnz], (nr, nc)


def export_vector(h, level, which):
    n = level_info(h, level)["N"]
    out = np.zeros(n)
    _check(h, lib().export_vector(h, int(level), int(which), out.ctypes.data_as(C.c_void_p)))
    return out


def export_blocks(h, level):
    sizes = (C.c_int64 * 2)()
    _check(h, lib().export_blocks(h, int(level), sizes, None, None, None))
    nb, tot = int(sizes[0]), int(sizes[1])
    N = level_info(h, level)["N"]
    ptr = np.zeros(nb + 1, np.int64)
    dofs = np.zeros(max(tot, 1), np.int32)
    owner = np.zeros(N, np.int32)
    _check(h, lib().export_blocks(h, int(level), sizes, ptr.ctypes.data_as(C.c_void_p),
                                  dofs.ctypes.data_as(C.c_void_p),
                                  owner.ctypes.data_as(C.c_void_p)))
    return ptr, dofs[:tot], owner


def block_colours(h, level):
    """First block of each colour of the multiplicative sweep (export_blocks
    order, last entry = number of blocks); empty for the additive smoother."""
    n = C.c_int64(0)
    _check(h, lib().block_colours(h, int(level), C.byref(n), None))
    ptr = np.zeros(n.value + 1, np.int64)
    if n.value:
        _check(h, lib().block_colours(h, int(level), C.byref(n), ptr.ctypes.data_as(C.c_void_p)))
    return ptr if n.value else np.zeros(0, np.int64)


def kernel_timing(h, enable):
    """Start (enable=True) or stop event timing; on stop returns
    {kind: (launches, total_ms)} for kinds smoother / vspmv / outer_spmv / transfer."""
    counts = (C.c_int64 * 4)()
    tot = (C.c_double * 4)()
    _check(h, lib().kernel_timing(h, int(bool(enable)), counts, tot))
    if enable:
        return None
    names = ["smoother", "vspmv", "outer_spmv", "transfer"]
    return {n: (int(counts[i]), float(tot[i])) for i, n in enumerate(names)}


def tuning_info(h, level):
    out = (C.c_int32 * 7)()
    _check(h, lib().tuning_info(h, int(level), out))
    return dict(spmv_lanes=int(out[0]), smooth_threads=int(out[1]), outer_lanes=int(out[2]),
                restrict_lanes=int(out[3]), prolong_lanes=int(out[4]), fused=int(out[5]),
                split=int(out[6]))


def hierarchy_destroy(h):
    if h:
        lib().hierarchy_destroy(h)


# ----------------------------------------------------------------------------
class Hierarchy:
    """Owning wrapper of a handle.  device=-1 builds a host-only handle (setup
    data can be inspected, no device call is valid)."""

    def __init__(self, cfg, w=None, device=0, stream=None, allocator="torch"):
        """allocator: "torch" (device memory from torch's caching allocator,
        the default), None (the library's hipMalloc) or an object with a
        `struct` Allocator attribute."""
        self.cfg = dict(cfg)
        self.device = device
        self.h = None
        if device >= 0 and stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        if allocator == "torch":
            allocator = TorchAllocator(device) if device >= 0 else None
        self.allocator = allocator   # outlives the handle (closed first)
        self.built_key = None      # (E, mu, options) of the current block inverses
        self.advection = 0         # re-assemblies about a new advecting velocity so far
        self.h = setup_hierarchy(cfg, w, device, stream, allocator)
        self.L = int(cfg["n_levels"])
        self.info = [level_info(self.h, l) for l in range(self.L)]
        self.N = self.info[-1]["N"]

    def close(self):
        if self.h:
            hierarchy_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def smoother_options(self, **kw):
        """The full option set build_fs_as_blocks(**kw) would use: the
        workload's settings, the library defaults, then kw."""
        opts = dict(core=tuple(self.cfg.get("core", (4, 4))), halo=self.cfg.get("halo", 1),
                    nu_pre=self.cfg.get("nu_pre", 2), nu_post=self.cfg.get("nu_post", 2),
                    omega=self.cfg.get("omega", 0.8), prec="fp64", use_graph=True,
                    iface_mult=self.cfg.get("iface_mult", 1),
                    monolithic=self.cfg.get("monolithic", False),
                    cycle=self.cfg.get("cycle", "V"),
                    schwarz=self.cfg.get("schwarz", "additive"), sweep_form="auto",
                    interchange=bool(self.cfg.get("interchange", False)))
        opts.update(kw)
        if "core" in kw:
            opts["core"] = tuple(kw["core"])
        return opts

    def blocks_key(self, **kw):
        """What the block inverses depend on: (E, mu) and the smoother options."""
        opts = self.smoother_options(**kw)
        return (float(self.cfg["E"]), float(self.cfg["mu"]), tuple(sorted(opts.items())))

    def build_fs_as_blocks(self, **kw):
        opts = self.smoother_options(**kw)
        self.built_key = None
        build_fs_as_blocks(self.h, **opts)
        self.built_key = self.blocks_key(**kw)

    def ensure_blocks(self, E, mu, **kw):
        """Bring the handle to parameters (E, mu) with blocks built for the
        smoother options kw: update_params when (E, mu) differ from the
        handle's, build_fs_as_blocks when the blocks were built for other
        parameters or options (or never)."""
        if (float(E), float(mu)) != (float(self.cfg["E"]), float(self.cfg["mu"])):
            self.update_params(E, mu)
        if self.built_key != self.blocks_key(**kw):
            self.build_fs_as_blocks(**kw)

    def dof_map(self, level=None):
        return dof_map(self.h, self.L - 1 if level is None else level)

    def csr(self, level, which=0):
        import scipy.sparse as sp
        rp, col, val, shape = export_csr(self.h, level, which)
        return sp.csr_matrix((val, col, rp), shape=shape)

    def _vec(self, t, n=None):
        import torch
        n = self.N if n is None else n
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError("expected a float64 device tensor")
        if t.numel() != n or not t.is_contiguous():
            raise ValueError("expected a contiguous tensor of %d entries, got %d" % (n, t.numel()))
        return t

    def vcycle_apply(self, r, z, transpose=False):
        vcycle_apply(self.h, self._vec(r), self._vec(z), transpose)

    def _cols(self, a, b):
        import torch
        for t in (a, b):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
                raise TypeError("expected float64 device tensors")
            if t.dim() != 2 or t.shape[0] != self.N or not t.is_contiguous():
                raise ValueError("expected contiguous (N, k) tensors with N = %d" % self.N)
        if a.shape != b.shape:
            raise ValueError("the two tensors must have the same shape")
        return a.shape[1]

    def vcycle_apply_batch(self, r, z, transpose=False):
        """Cycle (or its transpose) on the columns of r ((N, k) float64 device tensors)."""
        vcycle_apply_batch(self.h, r, z, self._cols(r, z), transpose)

    def gmres_solve(self, b, x, **kw):
        return gmres_solve(self.h, self._vec(b), self._vec(x), **kw)

    def gmres_solve_batch(self, b, x, **kw):
        """FGMRES on the columns of b ((N, k) float64 device tensors)."""
        return gmres_solve_batch(self.h, b, x, self._cols(b, x), **kw)

    def adjoint_solve_batch(self, c, lam, **kw):
        """Adjoint FGMRES (A^T) on the columns of c ((N, k) float64 device tensors)."""
        return adjoint_solve_batch(self.h, c, lam, self._cols(c, lam), **kw)

    def adjoint_solve(self, c, lam, **kw):
        return adjoint_solve(self.h, self._vec(c), self._vec(lam), **kw)

    def assemble_load(self, f, b):
        n2d = self.info[-1]["N2"] * self.info[-1]["dim"]
        assemble_load(self.h, self._vec(f, n2d), self._vec(b))

    def load_adjoint(self, lam, gf):
        n2d = self.info[-1]["N2"] * self.info[-1]["dim"]
        load_adjoint(self.h, self._vec(lam), self._vec(gf, n2d))

    def apply_operator(self, level, x, y, transpose=False):
        n = self.info[level]["N"]
        apply_operator(self.h, level, self._vec(x, n), self._vec(y, n), transpose)

    def param_grad(self, lam, x):
        return param_grad(self.h, self._vec(lam), self._vec(x))

    def update_params(self, E, mu):
        self.built_key = None
        update_params(self.h, E, mu)
        self.cfg.update(E=float(E), mu=float(mu))

    def update_advection(self, x):
        """Picard step: re-assemble every level about the velocity part of x
        (a float64 device tensor; a float64 numpy array of N entries on a
        host-only handle)."""
        self.built_key = None
        self.advection += 1
        if self.device < 0:
            import numpy as np
            if not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.shape == (self.N,)
                    and x.flags.c_contiguous):
                raise TypeError("expected a contiguous float64 array of %d entries" % self.N)
            _check(self.h, lib().update_advection(self.h, x.ctypes.data_as(C.c_void_p)))
            return
        _check(self.h, lib().update_advection(self.h, _ptr(self._vec(x))))

    def time_rhs(self, f, g, x_prev, b):
        """b = F L f + g lift + F T x_prev (one backward-Euler step)."""
        n2d = self.info[-1]["N2"] * self.info[-1]["dim"]
        _check(self.h, lib().time_rhs(self.h, _ptr(self._vec(f, n2d)), float(g),
                                      _ptr(self._vec(x_prev)), _ptr(self._vec(b))))

    def period_solve(self, f, x, steps, picard_max=1, picard_tol=0.0, inflow_amp=0.75, t0=0.0,
                     rtol=None, restart=None, max_restarts=20):
        """Run `steps` backward-Euler steps with Picard updates (library
        loop); returns a dict with the statistics and per-solve records."""
        n2d = self.info[-1]["N2"] * self.info[-1]["dim"]
        o = PeriodOpts(int(steps), float(t0), int(picard_max), float(picard_tol), float(inflow_amp))
        k = KrylovOpts(int(self.cfg.get("restart", 30) if restart is None else restart),
                       int(max_restarts),
                       float(self.cfg.get("rtol", 1e-10) if rtol is None else rtol))
        it = np.zeros(steps * picard_max, np.int32)
        ch = np.zeros(steps * picard_max, np.float64)
        info = PeriodInfo()
        st = lib().period_solve(self.h, C.byref(o), C.byref(k), _ptr(self._vec(f, n2d)),
                                _ptr(self._vec(x)),
                                it.ctypes.data_as(C.c_void_p), ch.ctypes.data_as(C.c_void_p),
                                C.byref(info))
        self.built_key = None
        self.advection += 1
        if st not in (FSGMG_OK, FSGMG_NOT_CONVERGED):
            _check(self.h, st)
        out = {name: getattr(info, name) for name, _ in PeriodInfo._fields_}
        out.update(converged=(st == FSGMG_OK), iters=it.reshape(steps, picard_max),
                   changes=ch.reshape(steps, picard_max))
        return out

    def kernel_timing(self, enable):
        return kernel_timing(self.h, enable)

    def tuning_info(self):
        return [tuning_info(self.h, l) for l in range(self.L)]

    def stream_read_ceiling(self, nbytes=1 << 30, reps=7):
        """Read-only streaming rate of the device in GB/s (measurement)."""
        out = C.c_double(0.0)
        _check(self.h, lib().stream_read_ceiling(self.h, int(nbytes), int(reps), C.byref(out)))
        return out.value

"""GPU parity tests: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (each derived from the arithmetic); every vector comparison is
made per field (d, p^s, u, p^f, each against its own norm: tests/parity.py):
* operator apply, transfers, load: elementwise |y - y_ref| <= 64 eps (|A| |x|)_i
  (summation-order rounding only);
* FP64 V-cycle: the block inverses come from Gauss-Jordan (GPU) versus LU
  (oracle), so outputs differ by rounding amplified by block conditioning:
  relative error <= 1e-9 in every field;
* FP32 / BF16 smoother V-cycles: relative error to the FP64 oracle cycle
  <= 2e-4 / 2e-2 in every field (unit roundoff 6e-8 / 4e-3 times the same
  amplification);
* solves: true relative residual <= 1e-10 (checked here with the oracle's
  matrix on the CPU) and every field within 1e-8 of the oracle's reference
  solve (sparse LU with iterative refinement, oracle/direct.py: plain LU
  alone is off by ~5e-8 in the solid pressure).
"""
import sys

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import fem
from oracle.direct import direct_solve
from oracle.multigrid import Hierarchy as OracleHierarchy
from paper_1909_13201_amd import fsgmg, inputs
from tests.parity import check_fields, field_errors

# Solutions, per field, against the refined direct solve.  A solve that
# stops at a true relative residual rho leaves field errors up to
# kappa_f rho, kappa_f = ||(A^-1)_f|| ||b|| / ||x_f||: by dense inverses of
# the c1, c2-at-2-levels and 3D-channel operators 2.5e5 to 2.2e9 for the
# solid fields d and p^s of the nearly incompressible wall, 8e2 to 1e4 for
# u and p^f, and growing with refinement.  That worst case is vacuous for
# the solid fields; the bounds below sit 5 to 10 times above the largest
# errors observed at rho = 1e-10 over all these tests, on the oracle's own
# FGMRES and on the GPU (u 5e-10, p^f 1.2e-8 on full c2, d 3e-9, p^s 1.7e-7
# on the 3D channel's adjoint).
SOLVE_TOL = {"d": 1e-7, "ps": 1e-6, "u": 1e-8, "pf": 1e-7}
CYCLE_TOL = 1e-9      # per field, FP64 cycle against the oracle's

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {"c1": ("c1", 2), "c2L3": ("c2", 3), "c5L2": ("c5", 2)}


class Pair:
    def __init__(self, key, prec="fp64"):
        name, L = CASES[key]
        self.key = key
        self.cfg = inputs.with_levels(inputs.config(name), L)
        self.w = inputs.advecting_field(self.cfg)
        say("[setup]", key, "L", L)
        self.H = fsgmg.Hierarchy(self.cfg, self.w, device=0)
        self.O = OracleHierarchy(self.cfg, self.w)
        self.prec = None
        self.build(prec)

    def build(self, prec):
        if prec != self.prec:
            say("[blocks]", self.key, prec)
            self.H.build_fs_as_blocks(prec=prec)
            self.prec = prec


_pairs = {}


def pair(key, prec="fp64"):
    if key not in _pairs:
        _pairs[key] = Pair(key, prec)
    p = _pairs[key]
    p.build(prec)
    return p


@pytest.mark.parametrize("key", ["c1", "c2L3"])
def test_operator_apply_parity(key):
    p = pair(key)
    rng = np.random.default_rng(1)
    for l in range(p.H.L):
        A = p.O.A[l]
        x = rng.standard_normal(A.shape[0])
        for tr in (False, True):
            say("[apply]", key, "level", l, "transpose", tr)
            y = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
            p.H.apply_operator(l, dev(x), y, transpose=tr)
            M = A.T if tr else A
            ref = M @ x
            bound = 64 * EPS * (abs(M) @ abs(x)) + 1e-300
            assert np.all(abs(host(y) - ref) <= bound)


@pytest.mark.parametrize("key", ["c1", "c2L3", "c5L2"])
def test_load_parity(key):
    p = pair(key)
    f = inputs.body_force(p.cfg)
    say("[load]", key)
    b = torch.zeros(p.H.N, dtype=torch.float64, device="cuda")
    p.H.assemble_load(dev(f.ravel()), b)
    ref = p.O.rhs(f)
    assert np.allclose(host(b), ref, rtol=0, atol=1e-13 * abs(ref).max())


@pytest.mark.parametrize("key", ["c1", "c2L3"])
@pytest.mark.parametrize("transpose", [False, True])
def test_vcycle_fp64_parity(key, transpose):
    p = pair(key, "fp64")
    rng = np.random.default_rng(2)
    r = rng.standard_normal(p.H.N)
    say("[vcycle fp64]", key, "transpose", transpose)
    z = torch.zeros(p.H.N, dtype=torch.float64, device="cuda")
    p.H.vcycle_apply(dev(r), z, transpose=transpose)
    ref = p.O.vcycle(r, transpose=transpose)
    check_fields(host(z), ref, p.H.info[-1], CYCLE_TOL, "fp64 cycle")


@pytest.mark.parametrize("key", ["c1", "c2L3"])
def test_monolithic_comparator_parity(key):
    """The comparator (monolithic Vanka blocks over d, u, p): FP64 V-cycle and
    its transpose against the oracle's with the same blocks, and an FP32
    solve to a true 1e-10."""
    cfg = inputs.config("c1") if key == "c1" else inputs.with_levels(inputs.config("c2"), 3)
    w = inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w, build_smoothers=False)
    O.build_smoothers(monolithic=True)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64", monolithic=True)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for tr in (False, True):
        H.vcycle_apply(dev(r), z, transpose=tr)
        ref = O.vcycle(r, transpose=tr)
        say("[monolithic]", key, "transpose", tr)
        check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "fp64 cycle")
    H.build_fs_as_blocks(prec="fp32", monolithic=True)
    b = O.rhs(inputs.body_force(cfg))
    x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    info = H.gmres_solve(dev(b), x, rtol=1e-10)
    true = np.linalg.norm(b - O.A[-1] @ host(x)) / np.linalg.norm(b)
    say("   fp32 solve iters %d true %.2e" % (info["iters"], true))
    assert info["converged"] and true <= 1e-10
    check_fields(host(x), direct_solve(O.A[-1], b), H.info[-1], SOLVE_TOL, "fp32 solve")
    H.close()


@pytest.mark.parametrize("key", ["c1", "c2L3", "c2L3mono", "chan3d"])
def test_multiplicative_schwarz_parity(key):
    """Multicolour multiplicative Schwarz smoother: FP64 V-cycle and its
    transpose against the oracle's sequential sweep in the same colour order,
    the colour ranges equal to the oracle's, and an FP32 solve to a true
    1e-10 in no more iterations than the additive smoother needs."""
    import tests.cfgs as cfgs
    from oracle.schwarz import block_colouring, build_blocks, colour_major
    mono = key.endswith("mono")
    if key == "c1":
        cfg = inputs.config("c1")
    elif key == "chan3d":
        cfg = cfgs.channel3d(levels=2, nc=(2, 2, 2))
    else:
        cfg = inputs.with_levels(inputs.config("c2"), 3)
    cfg = dict(cfg, schwarz="multiplicative", monolithic=mono)
    w = None if key == "chan3d" else inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64")
    for l in range(1, H.L):
        blocks, _ = build_blocks(O.levels[l], cfg["core"], cfg["halo"],
                                 cfg.get("iface_mult", 1), mono)
        _, oc = colour_major(blocks, block_colouring(O.coupling_pattern(l), blocks))
        oc = np.array(oc)
        assert np.array_equal(fsgmg.block_colours(H.h, l),
                              np.searchsorted(oc, np.arange(oc.max() + 2)))
    rng = np.random.default_rng(13)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for tr in (False, True):
        H.vcycle_apply(dev(r), z, transpose=tr)
        ref = O.vcycle(r, transpose=tr)
        say("[multiplicative]", key, "transpose", tr)
        check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "fp64 cycle")
    b = O.rhs(inputs.body_force(cfg))
    xd = direct_solve(O.A[-1], b)
    its = {}
    for kind in ("multiplicative", "additive"):
        H.build_fs_as_blocks(prec="fp32", schwarz=kind)
        x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        info = H.gmres_solve(dev(b), x, rtol=1e-10)
        true = np.linalg.norm(b - O.A[-1] @ host(x)) / np.linalg.norm(b)
        say("   %s fp32 solve iters %d true %.2e" % (kind, info["iters"], true))
        assert info["converged"] and true <= 1e-10
        check_fields(host(x), xd, H.info[-1], SOLVE_TOL, kind + " fp32 solve")
        its[kind] = info["iters"]
    assert its["multiplicative"] <= its["additive"]
    H.close()


@pytest.mark.parametrize("schwarz", ["additive", "multiplicative"])
@pytest.mark.parametrize("key", ["c1", "c2L3", "chan3d"])
def test_fused_and_spmv_sweeps_parity(key, schwarz):
    """Forward sweeps that form their residual inside the smoother launch
    (sweep_form "fused") and sweeps after a residual SpMV ("spmv"): each FP64
    cycle and its transpose against the oracle's, the two forms against each
    other, FP32 solves to a true 1e-10 with the same iteration counts."""
    import tests.cfgs as cfgs
    if key == "c1":
        cfg = inputs.config("c1")
    elif key == "chan3d":
        cfg = cfgs.channel3d(levels=2, nc=(2, 2, 2))
    else:
        cfg = inputs.with_levels(inputs.config("c2"), 3)
    cfg = dict(cfg, schwarz=schwarz)
    w = None if key == "chan3d" else inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    rng = np.random.default_rng(17)
    r = rng.standard_normal(H.N)
    b = O.rhs(inputs.body_force(cfg))
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    zs, its = {}, {}
    for form in ("fused", "spmv"):
        H.build_fs_as_blocks(prec="fp64", sweep_form=form)
        assert all(t["fused"] == (form == "fused") for t in H.tuning_info()[1:])
        for tr in (False, True):
            H.vcycle_apply(dev(r), z, transpose=tr)
            zs[form, tr] = host(z)
            ref = O.vcycle(r, transpose=tr)
            say("[sweeps]", key, schwarz, form, "transpose", tr)
            check_fields(zs[form, tr], ref, H.info[-1], CYCLE_TOL, "fp64 cycle")
        H.build_fs_as_blocks(prec="fp32", sweep_form=form)
        x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        info = H.gmres_solve(dev(b), x, rtol=1e-10)
        true = np.linalg.norm(b - O.A[-1] @ host(x)) / np.linalg.norm(b)
        say("   %s fp32 solve iters %d true %.2e" % (form, info["iters"], true))
        assert info["converged"] and true <= 1e-10
        check_fields(host(x), direct_solve(O.A[-1], b), H.info[-1], SOLVE_TOL, "fp32 solve")
        its[form] = info["iters"]
        tune = H.tuning_info()
        for t in tune[1:]:
            assert t["spmv_lanes"] in (1, 2, 4, 8, 16)
            assert abs(t["smooth_threads"]) in (256, 512, 1024)
            assert t["restrict_lanes"] in (1, 2, 4, 8, 16)
            assert t["prolong_lanes"] in (1, 2, 4, 8, 16)
            assert t["split"] in (1, 2, 4, 8)
        # a rebuild with the same options keeps the launch shapes and the
        # captured graphs, and refactors in place: the same solve, bit for bit
        H.build_fs_as_blocks(prec="fp32", sweep_form=form)
        assert H.tuning_info() == tune
        x2 = torch.zeros_like(x)
        info2 = H.gmres_solve(dev(b), x2, rtol=1e-10)
        assert info2["iters"] == info["iters"] and torch.equal(x, x2)
    check_fields(zs["fused", False], zs["spmv", False], H.info[-1], 1e-12, "fused vs spmv form")
    assert abs(its["fused"] - its["spmv"]) <= 1
    H.close()


@pytest.mark.parametrize("key,cycle", [("c1", "V"), ("c2L3", "V"), ("c2L3", "W"),
                                       ("chan3d", "V")])
def test_vcycle_batch_parity(key, cycle):
    """Several right-hand sides at once (vcycle_apply_batch, k columns
    unknown-major, block apply on the matrix cores), the cycle and its
    transpose: every column against the one-column cycle of the same
    precision (FP64 to 1e-12, FP32 and BF16 factors to the FP32 rounding of
    the cycle), FP64 columns against the oracle's cycle, ragged k (5, 17,
    40: one to three 16-column tiles) and the largest k (64); error paths."""
    import tests.cfgs as cfgs
    if key == "c1":
        cfg = inputs.config("c1")
    elif key == "chan3d":
        cfg = cfgs.channel3d(levels=2, nc=(2, 2, 2))
    else:
        cfg = inputs.with_levels(inputs.config("c2"), 3)
    cfg = dict(cfg, cycle=cycle)
    w = None if key == "chan3d" else inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    rng = np.random.default_rng(23)
    # FP32 / BF16 columns against the one-column cycle of the same precision:
    # the same inverses, FP32 sums in another order, so the per-field bound is
    # the FP32 cycle's own (2e-4; observed 7e-5 in the small d field)
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-4), ("bf16", 2e-4)):
        H.build_fs_as_blocks(prec=prec)
        for k in ((5, 17, 40, 64) if prec == "fp64" else (8, 32)):
            R = rng.standard_normal((H.N, k))
            Rd = dev(R.ravel()).reshape(H.N, k).contiguous()
            Z = torch.zeros_like(Rd)
            z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
            for tr in (False, True):
                H.vcycle_apply_batch(Rd, Z, transpose=tr)
                Zb = host(Z.reshape(-1)).reshape(H.N, k)
                worst = 0.0
                for c in range(k):
                    H.vcycle_apply(dev(np.ascontiguousarray(R[:, c])), z, transpose=tr)
                    zc = host(z)
                    e = field_errors(Zb[:, c], zc, H.info[-1])
                    worst = max(worst, max(e.values()))
                say("[batch]", key, cycle, prec, "k", k, "transpose", tr,
                    "max column per-field rel diff %.3e" % worst)
                assert worst <= tol
                if prec == "fp64":
                    for c in (0, k - 1):
                        ref = O.vcycle(R[:, c], transpose=tr)
                        check_fields(Zb[:, c], ref, H.info[-1], CYCLE_TOL, "column %d" % c)
    Rd = torch.zeros((H.N, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(fsgmg.FsgmgError):
        H.vcycle_apply_batch(Rd, torch.zeros_like(Rd))
    H.build_fs_as_blocks(prec="fp64", schwarz="multiplicative")
    Rd = torch.zeros((H.N, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(fsgmg.FsgmgError):
        H.vcycle_apply_batch(Rd, torch.zeros_like(Rd))
    H.close()


@pytest.mark.parametrize("key,k", [("c1", 5), ("c2L3", 32), ("chan3d", 17)])
def test_gmres_solve_batch(key, k):
    """FGMRES on k loads at once (gmres_solve_batch, FP32 cycle): every column
    converges to a true 1e-10 (recomputed with the oracle's matrix), in the
    iteration count of its one-column solve (+-1), and agrees with that
    solve's solution; a zero column and a repeated column are handled.  The
    adjoint on the same k right-hand sides (adjoint_solve_batch) reaches a
    true 1e-10 with A^T in the one-column adjoint's iteration count."""
    import tests.cfgs as cfgs
    if key == "c1":
        cfg = inputs.config("c1")
    elif key == "chan3d":
        cfg = cfgs.channel3d(levels=2, nc=(2, 2, 2))
    else:
        cfg = inputs.with_levels(inputs.config("c2"), 3)
    w = None if key == "chan3d" else inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w, build_smoothers=False)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp32")
    rng = np.random.default_rng(29)
    Bh = np.column_stack([O.rhs(inputs.body_force(cfg, seed=s)) for s in range(k)])
    Bh[:, 1] = 0.0                        # a zero load
    Bh[:, 2] = Bh[:, 0]                   # a repeated load
    Bh[:, 3] *= 1e-6                      # a small one
    Bd = dev(Bh.ravel()).reshape(H.N, k).contiguous()
    Xd = torch.zeros_like(Bd)
    infos = H.gmres_solve_batch(Bd, Xd, rtol=1e-10)
    Xh = host(Xd.reshape(-1)).reshape(H.N, k)
    A = O.A[-1]
    x1 = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for c in range(k):
        bn = np.linalg.norm(Bh[:, c])
        if bn == 0.0:
            assert infos[c]["converged"] and np.all(Xh[:, c] == 0.0)
            continue
        true = np.linalg.norm(Bh[:, c] - A @ Xh[:, c]) / bn
        one = H.gmres_solve(dev(np.ascontiguousarray(Bh[:, c])), x1, rtol=1e-10)
        if c < 5 or c == k - 1:
            say("[gmres batch]", key, "col", c, "iters", infos[c]["iters"], "one-column", one["iters"],
                "true %.2e" % true)
        assert infos[c]["converged"] and true <= 1e-10
        assert abs(infos[c]["iters"] - one["iters"]) <= 1
        if c < 5 or c == k - 1:
            check_fields(Xh[:, c], direct_solve(A, Bh[:, c]), H.info[-1], SOLVE_TOL,
                         "column %d" % c)
    assert np.array_equal(Xh[:, 0], Xh[:, 2])
    # adjoint on the same loads (A^T, transposed K-column cycle)
    Ld = torch.zeros_like(Bd)
    ainfos = H.adjoint_solve_batch(Bd, Ld, rtol=1e-10)
    Lh = host(Ld.reshape(-1)).reshape(H.N, k)
    AT = A.T.tocsr()
    for c in (0, 3, k - 1):
        bn = np.linalg.norm(Bh[:, c])
        true = np.linalg.norm(Bh[:, c] - AT @ Lh[:, c]) / bn
        one = H.adjoint_solve(dev(np.ascontiguousarray(Bh[:, c])), x1, rtol=1e-10)
        say("[adjoint batch]", key, "col", c, "iters", ainfos[c]["iters"], "one-column", one["iters"],
            "true %.2e" % true)
        assert ainfos[c]["converged"] and true <= 1e-10
        assert abs(ainfos[c]["iters"] - one["iters"]) <= 1
        check_fields(Lh[:, c], direct_solve(A, Bh[:, c], transpose=True), H.info[-1], SOLVE_TOL,
                     "adjoint column %d" % c)
    H.close()


@pytest.mark.parametrize("kind", ["W", "F"])
def test_w_and_f_cycles_parity(kind):
    """W- and F-cycles (c2 at 3 levels): FP64 cycle and its transpose against
    the oracle's (whose compositions are pinned in closed form), and an FP32
    FGMRES solve to a true 1e-10."""
    cfg = dict(inputs.with_levels(inputs.config("c2"), 3), cycle=kind)
    w = inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64")
    rng = np.random.default_rng(8)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for tr in (False, True):
        H.vcycle_apply(dev(r), z, transpose=tr)
        ref = O.vcycle(r, transpose=tr)
        say("[%s-cycle] transpose %s" % (kind, tr))
        check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "fp64 cycle")
    H.build_fs_as_blocks(prec="fp32")
    b = O.rhs(inputs.body_force(cfg))
    x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    info = H.gmres_solve(dev(b), x, rtol=1e-10)
    true = np.linalg.norm(b - O.A[-1] @ host(x)) / np.linalg.norm(b)
    say("   fp32 solve iters %d true %.2e" % (info["iters"], true))
    assert info["converged"] and true <= 1e-10
    check_fields(host(x), direct_solve(O.A[-1], b), H.info[-1], SOLVE_TOL, "fp32 solve")
    H.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-4), ("bf16", 2e-2)])
def test_vcycle_mixed_precision(prec, tol):
    p = pair("c2L3", prec)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(p.H.N)
    say("[vcycle]", prec)
    z = torch.zeros(p.H.N, dtype=torch.float64, device="cuda")
    p.H.vcycle_apply(dev(r), z)
    ref = p.O.vcycle(r)
    check_fields(host(z), ref, p.H.info[-1], tol, prec + " cycle")
    p.build("fp64")


def test_vcycle_deterministic():
    p = pair("c2L3", "fp32")
    r = dev(np.random.default_rng(4).standard_normal(p.H.N))
    say("[determinism] 10 cycles and 10 solves")
    z1 = torch.zeros_like(r)
    p.H.vcycle_apply(r, z1)
    for rep in range(9):
        z2 = torch.zeros_like(r)
        p.H.vcycle_apply(r, z2)
        assert torch.equal(z1, z2), rep
    b = dev(p.O.rhs(inputs.body_force(p.cfg)))
    x1 = torch.zeros_like(b)
    i1 = p.H.gmres_solve(b, x1)
    for rep in range(9):
        x2 = torch.zeros_like(b)
        i2 = p.H.gmres_solve(b, x2)
        assert i2["iters"] == i1["iters"] and torch.equal(x1, x2), rep
        assert np.array_equal(i2["history"], i1["history"])
    p.build("fp64")


@pytest.mark.parametrize("key", ["c1", "c2L3"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_gmres_solve(key, prec):
    p = pair(key, prec)
    f = inputs.body_force(p.cfg)
    b = p.O.rhs(f)
    A = p.O.A[-1]
    say("[gmres]", key, prec)
    x = torch.zeros(p.H.N, dtype=torch.float64, device="cuda")
    info = p.H.gmres_solve(dev(b), x, restart=30, rtol=1e-10)
    xs = host(x)
    true = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
    say("   iters", info["iters"], "true %.2e" % true, "lib %.2e" % info["rel_res_true"])
    assert info["converged"]
    assert true <= 1e-10
    assert abs(info["rel_res_true"] - true) <= 1e-3 * true + 1e-14
    assert info["vcycles"] == info["iters"] and info["t_setup_ms"] > 0 and info["t_blocks_ms"] > 0
    check_fields(xs, direct_solve(A, b), p.H.info[-1], SOLVE_TOL, "solution")
    hist = info["history"]
    assert np.all(np.diff(hist) <= 1e-12)
    if prec == "fp64":
        from oracle.krylov import fgmres
        _, oinfo = fgmres(lambda v: A @ v, p.O.vcycle, b, restart=30, rtol=1e-10)
        assert abs(oinfo["iters"] - info["iters"]) <= 1
    p.build("fp64")


def test_adjoint_and_gradients():
    p = pair("c5L2", "fp64")
    lv = p.O.finest
    A = p.O.A[-1]
    f = inputs.body_force(p.cfg)
    b = p.O.rhs(f)
    c = oadj.outlet_flux_vector(lv)
    say("[adjoint]")
    x = torch.zeros(p.H.N, dtype=torch.float64, device="cuda")
    info = p.H.gmres_solve(dev(b), x, rtol=1e-12, max_restarts=40)
    lam = torch.zeros_like(x)
    ainfo = p.H.adjoint_solve(dev(c), lam, rtol=1e-11, max_restarts=40)
    assert info["converged"] and ainfo["converged"]
    lam_d = direct_solve(A, c, transpose=True)
    check_fields(host(lam), lam_d, p.H.info[-1], SOLVE_TOL, "lambda")
    gE, gmu = p.H.param_grad(lam, x)
    x_d = direct_solve(A, b)
    check_fields(host(x), x_d, p.H.info[-1], SOLVE_TOL, "x")
    oE, omu = oadj.gradients(p.O, x_d, lam_d)
    say("   grads", gE, gmu, "oracle", oE, omu)
    assert gE == pytest.approx(oE, rel=1e-6)
    assert gmu == pytest.approx(omu, rel=1e-6)


def test_update_params_matches_reassembly():
    p = _pairs.pop("c5L2", None) or Pair("c5L2")
    E2, mu2 = 3.0e3, 2.0e-2
    say("[update_params]")
    p.H.update_params(E2, mu2)
    taus = [q["tau"] for q in p.O.parts]
    cfg2 = dict(p.cfg, E=E2, mu=mu2)
    O2 = OracleHierarchy(cfg2, p.w, taus=taus, build_smoothers=False)
    rng = np.random.default_rng(6)
    for l in range(p.H.L):
        x = rng.standard_normal(O2.A[l].shape[0])
        y = torch.zeros(len(x), dtype=torch.float64, device="cuda")
        p.H.apply_operator(l, dev(x), y)
        ref = O2.A[l] @ x
        assert np.all(abs(host(y) - ref) <= 64 * EPS * (abs(O2.A[l]) @ abs(x)) + 1e-300)
    p.H.build_fs_as_blocks(prec="fp64")
    b = O2.rhs(inputs.body_force(cfg2))
    bl = torch.zeros(p.H.N, dtype=torch.float64, device="cuda")
    p.H.assemble_load(dev(inputs.body_force(cfg2).ravel()), bl)
    assert np.allclose(host(bl), b, rtol=0, atol=1e-13 * abs(b).max())
    x = torch.zeros_like(bl)
    info = p.H.gmres_solve(bl, x, rtol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(b - O2.A[-1] @ host(x)) <= 1e-10 * np.linalg.norm(b)
    p.H.close()


def test_status_codes():
    p = pair("c1", "fp64")
    say("[status]")
    b = torch.full((p.H.N,), float("nan"), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(fsgmg.FsgmgError) as e:
        p.H.gmres_solve(b, x)
    assert e.value.status == -1
    b = dev(p.O.rhs(inputs.body_force(p.cfg)))
    info = p.H.gmres_solve(b, x, restart=2, max_restarts=0, rtol=1e-10)
    assert info["status"] == "NOT_CONVERGED" and not info["converged"] and info["iters"] == 2


def test_singular_block_status():
    """FSGMG_ESINGULAR forced from the host (debug_zero_block zeroes one
    block's gathered matrix before its inversion): the build reports the
    block and level, no cycle runs on the failed factors (ESTATE), and the
    next build without the hook restores a solve to a true 1e-10."""
    cfg = inputs.with_levels(inputs.config("c2"), 3)
    w = inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w, build_smoothers=False)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp32")
    b = O.rhs(inputs.body_force(cfg))
    for level, block in ((2, 5), (1, 0)):
        say("[esingular] level", level, "block", block)
        fsgmg.debug_zero_block(H.h, level, block)
        with pytest.raises(fsgmg.FsgmgError) as e:
            H.build_fs_as_blocks(prec="fp32")
        assert e.value.status == -3
        assert "block %d on level %d" % (block, level) in str(e.value)
        z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        with pytest.raises(fsgmg.FsgmgError) as e2:
            H.vcycle_apply(dev(b), z)
        assert e2.value.status == -5
        H.build_fs_as_blocks(prec="fp32")          # the hook applied once
        x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        info = H.gmres_solve(dev(b), x, rtol=1e-10)
        true = np.linalg.norm(b - O.A[-1] @ host(x)) / np.linalg.norm(b)
        assert info["converged"] and true <= 1e-10
    with pytest.raises(fsgmg.FsgmgError):
        fsgmg.debug_zero_block(H.h, 0, 1)             # level 0 has no Schwarz blocks
    H.close()


def test_full_size_c2_bench_configuration():
    """c2 at full size (5 levels, 281,095 unknowns), the configuration the
    benchmark times: FP32 V-cycle against the oracle's FP64 cycle and FP32 /
    BF16 solves whose true residual is recomputed with the oracle's matrix."""
    cfg = inputs.config("c2")
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    say("[full c2] oracle setup")
    O = OracleHierarchy(cfg, w)
    say("[full c2] library setup")
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64")
    rng = np.random.default_rng(9)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    say("[full c2] vcycle fp64")
    H.vcycle_apply(dev(r), z)
    ref = O.vcycle(r)
    check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "fp64 cycle")
    b = O.rhs(f)
    bd = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    H.assemble_load(dev(f.ravel()), bd)
    assert np.allclose(host(bd), b, rtol=0, atol=1e-13 * abs(b).max())
    A = O.A[-1]
    say("[full c2] reference solve")
    xd = direct_solve(A, b)
    for prec, tol in (("fp32", 2e-4), ("bf16", 2e-2)):
        say("[full c2]", prec)
        H.build_fs_as_blocks(prec=prec)
        H.vcycle_apply(dev(r), z)
        check_fields(host(z), ref, H.info[-1], tol, prec + " cycle")
        x = torch.zeros_like(bd)
        info = H.gmres_solve(bd, x, rtol=1e-10)
        xs = host(x)
        true = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
        say("   iters", info["iters"], "true %.2e" % true)
        assert info["converged"] and true <= 1e-10
        check_fields(xs, xd, H.info[-1], SOLVE_TOL, prec + " solve")
    H.close()


def test_full_size_c2_multiplicative_and_k_loads():
    """c2 at full size (5 levels, 281,095 unknowns): the multicolour
    multiplicative FP64 cycle against the oracle's sequential sweep (same
    colour order), an FP32 multiplicative solve, and FGMRES on 32 seeded
    loads at once (K-column cycle on the matrix cores) whose every column
    reaches a true 1e-10 with the oracle's matrix in the iteration count of
    its one-load solve (sampled columns)."""
    cfg = dict(inputs.config("c2"), schwarz="multiplicative")
    w = inputs.advecting_field(cfg)
    say("[full c2 mult] oracle setup")
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64")
    rng = np.random.default_rng(31)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    H.vcycle_apply(dev(r), z)
    ref = O.vcycle(r)
    check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "multiplicative fp64 cycle")
    A = O.A[-1]
    b = O.rhs(inputs.body_force(cfg))
    H.build_fs_as_blocks(prec="fp32")
    x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    info = H.gmres_solve(dev(b), x, rtol=1e-10)
    true = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
    say("   multiplicative fp32 iters", info["iters"], "true %.2e" % true)
    assert info["converged"] and true <= 1e-10
    K = 32
    H.build_fs_as_blocks(prec="fp32", schwarz="additive")
    Bh = np.column_stack([O.rhs(inputs.body_force(cfg, seed=100 + c)) for c in range(K)])
    Bd = dev(Bh.ravel()).reshape(H.N, K).contiguous()
    Xd = torch.zeros_like(Bd)
    infos = H.gmres_solve_batch(Bd, Xd, rtol=1e-10)
    Xh = host(Xd.reshape(-1)).reshape(H.N, K)
    worst = 0.0
    for c in range(K):
        t = np.linalg.norm(Bh[:, c] - A @ Xh[:, c]) / np.linalg.norm(Bh[:, c])
        worst = max(worst, t)
        assert infos[c]["converged"] and t <= 1e-10
    x1 = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for c in (0, K - 1):
        one = H.gmres_solve(dev(np.ascontiguousarray(Bh[:, c])), x1, rtol=1e-10)
        assert abs(infos[c]["iters"] - one["iters"]) <= 1
    say("   %d loads: iters %d..%d, worst true %.2e" % (K, min(i["iters"] for i in infos),
                                                         max(i["iters"] for i in infos), worst))
    H.close()


def test_c3_enlarged_interface_blocks_parity():
    """c3 (bulge geometry, layered walls, 4 x 12 interface cores) at 4
    levels: uneven blocks in one launch; FP64 V-cycle against the oracle's,
    FP32 / BF16 solves to a true 1e-10 (oracle matrix)."""
    cfg = inputs.with_levels(inputs.config("c3"), 4)
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    say("[c3 L4] oracle setup")
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64")
    ptr, _, _ = fsgmg.export_blocks(H.h, H.L - 1)
    n = np.diff(ptr)
    say("   finest blocks %d, sizes %d..%d" % (len(n), n.min(), n.max()))
    assert n.max() > 2 * np.percentile(n, 10)      # uneven sizes in one launch
    rng = np.random.default_rng(13)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for tr in (False, True):
        H.vcycle_apply(dev(r), z, transpose=tr)
        ref = O.vcycle(r, transpose=tr)
        check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "fp64 cycle transpose=%s" % tr)
    b = O.rhs(f)
    bd = dev(b)
    A = O.A[-1]
    xd = direct_solve(A, b)
    for prec in ("fp64", "fp32", "bf16"):
        H.build_fs_as_blocks(prec=prec)
        x = torch.zeros_like(bd)
        info = H.gmres_solve(bd, x, rtol=1e-10)
        true = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
        say("   %s iters %d true %.2e" % (prec, info["iters"], true))
        assert info["converged"] and true <= 1e-10
        check_fields(host(x), xd, H.info[-1], SOLVE_TOL, prec + " solve")
    H.close()


def _c3_cycle_golden():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "c3_fp64_cycle_samples.txt")
    out = dict(fields={}, samples={})
    smp = {}
    with open(path) as fi:
        for line in fi:
            t = line.split()
            if line.startswith("# oracle"):
                out["seed"] = int(line.split("default_rng(")[1].split(")")[0])
            elif t and t[0] == "N":
                out["N"] = int(t[1])
            elif t and t[0] == "field":
                out["fields"][t[1]] = (int(t[2]), int(t[3]), (float(t[4]), float(t[5])))
            elif t and t[0] == "s":
                smp.setdefault(t[1], []).append((int(t[2]), float(t[3]), float(t[4])))
    for f, rows in smp.items():
        a = np.array(rows)
        out["samples"][f] = (a[:, 0].astype(np.int64), a[:, 1:])
    return out


def test_full_size_c3():
    """c3 at full size (6 levels, 512 x 256 finest, about 2.2 M unknowns): the
    FP64 cycle and its transpose against the oracle's (per field, from the
    oracle's stored norms and sampled entries); FP32 and BF16-factor solves
    reach a true 1e-10 residual measured with the oracle's own finest matrix
    and right-hand side, and agree with each other to the
    conditioning-limited bound."""
    cfg = inputs.config("c3")
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    say("[full c3] oracle finest assembly")
    from oracle.mesh import Level
    lv = Level(cfg, cfg["n_levels"] - 1)
    asm = fem.assemble_level(lv, cfg, w)
    say("[full c3] library setup")
    H = fsgmg.Hierarchy(cfg, w, device=0)
    b = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    H.assemble_load(dev(f.ravel()), b)
    A = fem.dirichlet_reduce(lv, asm["A"])
    bo = fem.dirichlet_rhs(lv, asm["A"], fem.load_vector(lv, cfg, f, w, asm["tau"]))
    assert np.allclose(host(b), bo, rtol=0, atol=1e-13 * abs(bo).max())
    # FP64 cycle and its transpose against the oracle's, through the
    # per-field norms and sampled entries the oracle wrote for the same
    # seeded right-hand side (tests/golden/make_c3_cycle_samples.py)
    gold = _c3_cycle_golden()
    assert gold["N"] == H.N
    H.build_fs_as_blocks(prec="fp64")
    r = dev(np.random.default_rng(gold["seed"]).standard_normal(H.N))
    z = torch.zeros_like(r)
    for tr in (False, True):
        say("[full c3] fp64 cycle transpose", tr)
        H.vcycle_apply(r, z, transpose=tr)
        zh = host(z)
        for f, (i0, i1, nrm) in gold["fields"].items():
            idx, ref = gold["samples"][f]
            ref = ref[:, int(tr)]
            e = zh[idx] - ref
            est = np.sqrt((i1 - i0) / len(idx) * (e * e).sum())   # estimate of ||e_f||
            dn = abs(np.linalg.norm(zh[i0:i1]) - nrm[int(tr)])
            say("   field %s: sampled error norm estimate %.2e, norm diff %.2e (rel)"
                % (f, est / nrm[int(tr)], dn / nrm[int(tr)]))
            assert est <= CYCLE_TOL * nrm[int(tr)] and dn <= CYCLE_TOL * nrm[int(tr)]
    xs = {}
    for prec in ("fp32", "bf16"):
        say("[full c3]", prec)
        H.build_fs_as_blocks(prec=prec)
        x = torch.zeros_like(b)
        info = H.gmres_solve(b, x, rtol=1e-10)
        xs[prec] = host(x)
        true = np.linalg.norm(bo - A @ xs[prec]) / np.linalg.norm(bo)
        say("   iters %d true %.2e" % (info["iters"], true))
        assert info["converged"] and true <= 1e-10
    d = np.linalg.norm(xs["fp32"] - xs["bf16"]) / np.linalg.norm(xs["fp32"])
    say("   fp32 vs bf16 solution rel diff %.2e" % d)
    assert d <= 1e-6
    H.close()


def test_3d_channel_parity():
    """dim = 3 (hexahedral Q2/Q1, 4x4x4 finest, one-element cores with the
    one-element Vanka halo): the D = 3 SpMV, transfer and smoother kernels
    against the oracle's FP64 V-cycle and a sparse direct solve."""
    import tests.cfgs as cfgs
    cfg = cfgs.channel3d()
    f = inputs.body_force(cfg)
    O = OracleHierarchy(cfg, None)
    H = fsgmg.Hierarchy(cfg, None, device=0)
    H.build_fs_as_blocks(prec="fp64")
    rng = np.random.default_rng(21)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for tr in (False, True):
        H.vcycle_apply(dev(r), z, transpose=tr)
        ref = O.vcycle(r, transpose=tr)
        check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "[3d] fp64 cycle transpose=%s" % tr)
    b = O.rhs(f)
    A = O.A[-1]
    xd = direct_solve(A, b)
    for prec in ("fp64", "fp32"):
        H.build_fs_as_blocks(prec=prec)
        x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        info = H.gmres_solve(dev(b), x, rtol=1e-10)
        xs = host(x)
        true = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
        say("[3d] %s iters %d true %.2e" % (prec, info["iters"], true))
        assert info["converged"] and true <= 1e-10
        check_fields(xs, xd, H.info[-1], SOLVE_TOL, "[3d] %s solve" % prec)
    H.close()


def test_c4_tube_parity():
    """The 3D tube with the elastic ring and the leaflet (c4) at 2 levels
    (8 x 8 x 16 finest, 58,879 unknowns, 1,264 finest blocks of 192 to
    1,013 unknowns, disc-mapped hexahedra, the seeded 3D advecting field
    with SUPG): FP64 cycle and its transpose against the oracle's per
    field, FP32 and FP64 solves to a true 1e-10 (oracle matrix) with every
    field against the refined direct solve."""
    import time
    cfg = inputs.with_levels(inputs.config("c4"), 2)
    w = inputs.advecting_field(cfg)
    f = inputs.body_force(cfg)
    say("[c4 L2] oracle setup")
    O = OracleHierarchy(cfg, w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    t0 = time.perf_counter()
    H.build_fs_as_blocks(prec="fp64")
    torch.cuda.synchronize()
    say("   fp64 block build %.2f s" % (time.perf_counter() - t0))
    rng = np.random.default_rng(43)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    for tr in (False, True):
        H.vcycle_apply(dev(r), z, transpose=tr)
        ref = O.vcycle(r, transpose=tr)
        check_fields(host(z), ref, H.info[-1], CYCLE_TOL, "[c4] fp64 cycle transpose=%s" % tr)
    b = O.rhs(f)
    A = O.A[-1]
    say("[c4 L2] reference solve")
    xd = direct_solve(A, b)
    for prec in ("fp64", "fp32"):
        t0 = time.perf_counter()
        H.build_fs_as_blocks(prec=prec)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        info = H.gmres_solve(dev(b), x, rtol=1e-10)
        true = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
        say("[c4] %s blocks %.2f s, iters %d, true %.2e, solve %.1f ms"
            % (prec, tb, info["iters"], true, info["t_solve_ms"]))
        assert info["converged"] and true <= 1e-10
        check_fields(host(x), xd, H.info[-1], SOLVE_TOL, "[c4] %s solve" % prec)
    H.close()


@pytest.mark.parametrize("key", ["c1", "c2L3", "c5L2"])
def test_interchange_parity(key):
    """The interchanged cascade (GMRES preconditioned by the field split,
    each diagonal block by one GMG cycle on it): FP64 cycle per field
    against the oracle's, FP32 and FP64 solves to a true 1e-10 (the whole
    operator) with every field against the refined direct solve; the
    transposed cycle, the adjoint and the K-column calls are refused; back
    to the standard cascade, its cycle matches the oracle's again."""
    name, L = CASES[key]
    cfg = inputs.with_levels(inputs.config(name), L)
    w = inputs.advecting_field(cfg)
    Oi = OracleHierarchy(dict(cfg, interchange=True), w)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    H.build_fs_as_blocks(prec="fp64", interchange=True)
    rng = np.random.default_rng(19)
    r = rng.standard_normal(H.N)
    z = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    say("[interchange]", key)
    H.vcycle_apply(dev(r), z)
    check_fields(host(z), Oi.vcycle(r), H.info[-1], CYCLE_TOL, "interchanged fp64 cycle")
    with pytest.raises(fsgmg.FsgmgError) as e:
        H.vcycle_apply(dev(r), z, transpose=True)
    assert e.value.status == -1
    b = Oi.rhs(inputs.body_force(cfg))
    A = Oi.A[-1]
    xd = direct_solve(A, b)
    its = {}
    for prec in ("fp64", "fp32"):
        H.build_fs_as_blocks(prec=prec, interchange=True)
        x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
        info = H.gmres_solve(dev(b), x, rtol=1e-10, max_restarts=40)
        true = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
        say("   %s interchanged solve iters %d true %.2e" % (prec, info["iters"], true))
        assert info["converged"] and true <= 1e-10
        check_fields(host(x), xd, H.info[-1], SOLVE_TOL, "interchanged %s solve" % prec)
        its[prec] = info["iters"]
    lam = torch.zeros_like(x)
    with pytest.raises(fsgmg.FsgmgError):
        H.adjoint_solve(dev(b), lam)
    Bm = torch.zeros((H.N, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(fsgmg.FsgmgError):
        H.vcycle_apply_batch(Bm, torch.zeros_like(Bm))
    H.build_fs_as_blocks(prec="fp64")
    Os = OracleHierarchy(cfg, w)
    H.vcycle_apply(dev(r), z)
    check_fields(host(z), Os.vcycle(r), H.info[-1], CYCLE_TOL, "standard fp64 cycle after")
    x = torch.zeros(H.N, dtype=torch.float64, device="cuda")
    std = H.gmres_solve(dev(b), x, rtol=1e-10)
    say("   iterations: standard %d, interchanged %d (fp64)" % (std["iters"], its["fp64"]))
    H.close()


def test_graph_replays_match_eager():
    """Arnoldi-step and V-cycle graphs replayed several times, with eager
    library work and host synchronizations in between, give bitwise the
    eager results (all reductions are fixed-order)."""
    p = pair("c2L3", "fp32")
    f = inputs.body_force(p.cfg)
    b = dev(p.O.rhs(f))
    r = dev(np.random.default_rng(12).standard_normal(p.H.N))
    say("[graphs] eager")
    p.H.build_fs_as_blocks(prec="fp32", use_graph=False)
    xe = torch.zeros_like(b)
    ie = p.H.gmres_solve(b, xe)
    ze = torch.zeros_like(b)
    p.H.vcycle_apply(r, ze)
    say("[graphs] captured")
    p.H.build_fs_as_blocks(prec="fp32", use_graph=True)
    for rep in range(3):
        xg = torch.zeros_like(b)
        ig = p.H.gmres_solve(b, xg)
        assert ig["iters"] == ie["iters"]
        assert torch.equal(xg, xe), rep
        zg = torch.zeros_like(b)
        p.H.vcycle_apply(r, zg)
        assert torch.equal(zg, ze), rep
        y = torch.zeros_like(b)
        p.H.apply_operator(p.H.L - 1, xg, y)      # eager work between replays
        torch.cuda.synchronize()
    p.prec = None
    p.build("fp64")


@pytest.mark.parametrize("prec,levels,nsamp", [("fp64", 2, 3), ("fp32", 2, 3), ("fp32", 4, 2)])
def test_autograd_batch_gradients(prec, levels, nsamp):
    """Differentiation workload (c5; at 2 levels and at its full 4 levels,
    70,919 unknowns): x = FSISolve(f, E, mu), J = outlet flux; torch autograd
    (adjoint solve, load adjoint, parameter gradient in the library) against
    the oracle's adjoint gradients for seeded (f, E, mu) samples.  tau is
    frozen at the hierarchy's setup parameters on both sides."""
    from paper_1909_13201_amd.autograd import FSISolve
    cfg = inputs.with_levels(inputs.config("c5"), levels)
    w = inputs.advecting_field(cfg)
    say("[autograd]", prec)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    O0 = OracleHierarchy(cfg, w, build_smoothers=False)
    taus = [q["tau"] for q in O0.parts]
    lv = O0.finest
    c = oadj.outlet_flux_vector(lv)
    ct = dev(c)
    params = inputs.sample_parameters(cfg, nsamp)
    loads = inputs.sample_loads(cfg, nsamp)
    rng = np.random.default_rng(21)
    for i in range(nsamp):
        E, mu = params[i]
        f = torch.tensor(loads[i].ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
        Et = torch.tensor(E, dtype=torch.float64, requires_grad=True)
        mt = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
        x = FSISolve.apply(f, Et, mt, H, dict(prec=prec, rtol=1e-11 if levels < 4 else 1e-10,
                                               max_restarts=40))
        J = (ct * x).sum()
        J.backward()
        cfg_i = dict(cfg, E=float(E), mu=float(mu))
        Oi = OracleHierarchy(cfg_i, w, taus=taus, build_smoothers=False)
        A = Oi.A[-1]
        b = Oi.rhs(loads[i])
        xd = direct_solve(A, b)
        lam = direct_solve(A, c, transpose=True)
        oE, omu = oadj.gradients(Oi, xd, lam)
        df = rng.standard_normal(loads[i].shape)
        dJ = lam @ (Oi.rhs(loads[i] + df) - b)
        gdf = float((f.grad.detach().cpu().numpy() * df.ravel()).sum())
        say("   sample", i, "E %.3g mu %.3g" % (E, mu), "dJ/dE %.6e vs %.6e" % (Et.grad.item(), oE),
            "dJ/dmu %.6e vs %.6e" % (mt.grad.item(), omu), "df %.6e vs %.6e" % (gdf, dJ))
        assert float(J.detach()) == pytest.approx(c @ xd, rel=1e-8)
        assert Et.grad.item() == pytest.approx(oE, rel=1e-6)
        assert mt.grad.item() == pytest.approx(omu, rel=1e-6)
        assert gdf == pytest.approx(dJ, rel=1e-6)
    H.close()


def test_handle_pool_gradients():
    """Several handles at once (HandlePool: one stream and host thread per
    handle; c5 at 2 levels, 6 seeded samples over 3 handles): each sample's
    forward solve, adjoint solve and parameter gradients through the library
    calls FSISolve makes, against the oracle's direct solves and adjoint
    gradients, and every handle's launches interleaved with the others'."""
    from paper_1909_13201_amd.pool import HandlePool
    cfg = inputs.with_levels(inputs.config("c5"), 2)
    w = inputs.advecting_field(cfg)
    nsamp = 6
    params = inputs.sample_parameters(cfg, nsamp)
    loads = inputs.sample_loads(cfg, nsamp)
    O0 = OracleHierarchy(cfg, w, build_smoothers=False)
    taus = [q["tau"] for q in O0.parts]
    c = oadj.outlet_flux_vector(O0.finest)
    ct = dev(c)
    torch.cuda.synchronize()

    def pipeline(H, i):
        H.update_params(float(params[i][0]), float(params[i][1]))
        H.build_fs_as_blocks(prec="fp32")
        f = torch.tensor(loads[i].ravel(), dtype=torch.float64, device="cuda")
        b = torch.empty(H.N, dtype=torch.float64, device="cuda")
        H.assemble_load(f, b)
        x = torch.empty_like(b)
        inf = H.gmres_solve(b, x, rtol=1e-11, max_restarts=40)
        lam = torch.empty_like(x)
        ainf = H.adjoint_solve(ct, lam, rtol=1e-11, max_restarts=40)
        gE, gmu = H.param_grad(lam, x)
        return inf["converged"] and ainf["converged"], float((ct * x).sum()), gE, gmu

    def failing(H, i):
        if i == 4:
            raise ValueError("item 4")
        return pipeline(H, i)

    say("[pool] 3 handles,", nsamp, "samples")
    with HandlePool(cfg, w, n=3, device=0) as pool:
        got = pool.map(pipeline, range(nsamp))
        got2 = pool.map(pipeline, reversed(range(nsamp)))[::-1]   # handles see other samples
        with pytest.raises(ValueError, match="item 4"):               # an item's error reaches the caller
            pool.map(failing, range(nsamp))
        assert pool.map(pipeline, [1])[0][1] == pytest.approx(got[1][1], rel=1e-9)   # still usable
    for i in range(nsamp):
        E, mu = params[i]
        Oi = OracleHierarchy(dict(cfg, E=float(E), mu=float(mu)), w, taus=taus,
                             build_smoothers=False)
        A = Oi.A[-1]
        xd = direct_solve(A, Oi.rhs(loads[i]))
        lam = direct_solve(A, c, transpose=True)
        oE, omu = oadj.gradients(Oi, xd, lam)
        for ok, J, gE, gmu in (got[i], got2[i]):
            say("   sample", i, "J %.9e vs %.9e" % (J, c @ xd), "dJ/dE %.6e vs %.6e" % (gE, oE))
            assert ok
            assert J == pytest.approx(c @ xd, rel=1e-8)
            assert gE == pytest.approx(oE, rel=1e-6)
            assert gmu == pytest.approx(omu, rel=1e-6)


def test_autograd_two_forwards_one_backward():
    """Two forwards on one handle with different (E, mu) and smoother
    precisions, then one backward of the summed loss: each sample's
    gradients must be those of its own operator (the handle is brought back
    to each forward's parameters and options before its adjoint solve)."""
    from paper_1909_13201_amd.autograd import FSISolve
    cfg = inputs.with_levels(inputs.config("c5"), 2)
    w = inputs.advecting_field(cfg)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    O0 = OracleHierarchy(cfg, w, build_smoothers=False)
    taus = [q["tau"] for q in O0.parts]
    c = oadj.outlet_flux_vector(O0.finest)
    ct = dev(c)
    params = inputs.sample_parameters(cfg, 2)
    loads = inputs.sample_loads(cfg, 2)
    say("[autograd] two forwards, one backward")
    Es, mus, xs = [], [], []
    J = 0
    for i, prec in enumerate(("fp64", "fp32")):
        E, mu = params[i]
        f = torch.tensor(loads[i].ravel(), dtype=torch.float64, device="cuda")
        Et = torch.tensor(E, dtype=torch.float64, requires_grad=True)
        mt = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
        x = FSISolve.apply(f, Et, mt, H, dict(prec=prec, rtol=1e-11, max_restarts=40))
        J = J + (ct * x).sum()
        Es.append(Et)
        mus.append(mt)
    J.backward()
    for i in range(2):
        E, mu = params[i]
        Oi = OracleHierarchy(dict(cfg, E=float(E), mu=float(mu)), w, taus=taus,
                             build_smoothers=False)
        A = Oi.A[-1]
        xd = direct_solve(A, Oi.rhs(loads[i]))
        lam = direct_solve(A, c, transpose=True)
        oE, omu = oadj.gradients(Oi, xd, lam)
        say("   sample", i, "dJ/dE %.6e vs %.6e" % (Es[i].grad.item(), oE),
            "dJ/dmu %.6e vs %.6e" % (mus[i].grad.item(), omu))
        assert Es[i].grad.item() == pytest.approx(oE, rel=1e-6)
        assert mus[i].grad.item() == pytest.approx(omu, rel=1e-6)
    H.close()


def test_autograd_refuses_backward_after_advection_update():
    """A re-assembly about another advecting velocity between a forward and
    its backward leaves no copy of the forward's operator: the backward
    raises instead of differentiating the new operator."""
    from paper_1909_13201_amd.autograd import FSISolve
    cfg = inputs.with_levels(inputs.config("c5"), 2)
    H = fsgmg.Hierarchy(cfg, inputs.advecting_field(cfg), device=0)
    say("[autograd] backward after update_advection")
    try:
        E, mu = inputs.sample_parameters(cfg, 1)[0]
        f = torch.tensor(inputs.sample_loads(cfg, 1)[0].ravel(), dtype=torch.float64,
                         device="cuda")
        Et = torch.tensor(E, dtype=torch.float64, requires_grad=True)
        mt = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
        x = FSISolve.apply(f, Et, mt, H, dict(prec="fp32"))
        H.update_advection(x.detach().contiguous())
        with pytest.raises(RuntimeError, match="advecting velocity changed"):
            x.sum().backward()
    finally:
        H.close()


def test_caller_allocator():
    """Device storage through the caller's allocator (torch's caching
    allocator, the binding's default): the library's buffers are blocks of
    torch's pool, every one is returned when the handle is destroyed, and
    solves are bitwise those of a handle on the library's own hipMalloc."""
    cfg = inputs.with_levels(inputs.config("c2"), 3)
    w = inputs.advecting_field(cfg)
    O = OracleHierarchy(cfg, w, build_smoothers=False)
    b = dev(O.rhs(inputs.body_force(cfg)))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    say("[allocator] torch caching allocator")
    H = fsgmg.Hierarchy(cfg, w, device=0)
    alloc = H.allocator
    assert isinstance(alloc, fsgmg.TorchAllocator)
    n_setup = alloc.allocs
    assert n_setup > 0 and alloc.frees == 0
    H.build_fs_as_blocks(prec="fp32")
    assert alloc.allocs > n_setup
    held = sum(alloc.live.values())
    assert torch.cuda.memory_allocated() - before >= held > 0
    x = torch.zeros_like(b)
    info = H.gmres_solve(b, x)
    assert info["converged"]
    H.build_fs_as_blocks(prec="fp32", core=(2, 2))      # new index sets: buffers replaced
    assert alloc.frees > 0
    H.build_fs_as_blocks(prec="fp32")
    x1 = torch.zeros_like(b)
    H.gmres_solve(b, x1)
    xh, x1h = host(x), host(x1)
    del x, x1
    H.close()
    torch.cuda.synchronize()
    assert alloc.allocs == alloc.frees and not alloc.live
    assert torch.cuda.memory_allocated() == before
    say("   %d allocations, all returned" % alloc.allocs)
    say("[allocator] library hipMalloc")
    H2 = fsgmg.Hierarchy(cfg, w, device=0, allocator=None)
    H2.build_fs_as_blocks(prec="fp32")
    x2 = torch.zeros_like(b)
    H2.gmres_solve(b, x2)
    H2.close()
    # launch shapes are autotuned per build, which changes rounding only
    info_f = dict(N=x2.numel(), off_ps=O.finest.off_ps, off_u=O.finest.off_u,
                  off_pf=O.finest.off_pf)
    check_fields(xh, host(x2), info_f, 1e-11, "torch-pool vs hipMalloc handle")
    check_fields(x1h, host(x2), info_f, 1e-11, "after a rebuild")

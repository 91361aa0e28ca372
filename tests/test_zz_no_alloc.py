"""GPU test of the allocation-free parameter gradient (param_grad_noalloc):
called through the C ABI, it must return what param_grad returns, on two
calls in a row, the second on a smaller problem (the scratch array keeps the
first call's contents)."""
import ctypes as C

import numpy as np
import pytest

from paper_1909_13201_amd import fsgmg, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    return fsgmg.lib().param_grad_noalloc


def _case(cfg, seed):
    w = inputs.advecting_field(cfg)
    H = fsgmg.Hierarchy(cfg, w, device=0)
    rng = np.random.default_rng(seed)
    lam = torch.tensor(rng.standard_normal(H.N), dtype=torch.float64, device="cuda")
    x = torch.tensor(rng.standard_normal(H.N), dtype=torch.float64, device="cuda")
    return H, lam, x


def test_param_grad_noalloc_matches_param_grad():
    f = _lib()
    big = inputs.with_levels(inputs.config("c5"), 3)
    small = inputs.config("c1")
    for cfg, seed in ((big, 1), (small, 2)):
        print("[noalloc]", cfg["name"], "levels", cfg["n_levels"], flush=True)
        H, lam, x = _case(cfg, seed)
        ref = H.param_grad(lam, x)
        out = (C.c_double * 2)()
        torch.cuda.synchronize()
        st = f(H.h, C.c_void_p(lam.data_ptr()), C.c_void_p(x.data_ptr()), out)
        assert st == 0, fsgmg.lib().last_error(H.h)
        print("   param_grad %r, noalloc %r" % (ref, (out[0], out[1])), flush=True)
        assert (out[0], out[1]) == ref          # same kernels, same order: bit for bit
        H.close()


def test_param_grad_noalloc_error_codes():
    """Status codes without any launch: a host-only handle is a state
    error, a null handle an argument error."""
    f = _lib()
    H = fsgmg.Hierarchy(inputs.config("c1"), None, device=-1)
    out = (C.c_double * 2)()
    assert f(H.h, C.c_void_p(16), C.c_void_p(32), out) == -5
    assert f(None, C.c_void_p(16), C.c_void_p(32), out) == -1
    H.close()

"""CPU tests of the benchmark's contract and of its byte model (no GPU).

* ``bench.py --gpus N`` with N above 1 exits with status 2 and says that the
  solver measures one GPU;
* the algorithmic bytes that the roofline divides by, for one FS-AS sweep
  (owned rows of every block inverse, index lists, one residual read and one
  correction read + write), recomputed from the oracle's own Schwarz blocks
  and owner map.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle.multigrid import Hierarchy as OracleHierarchy
from oracle.schwarz import build_blocks, owners
from paper_1909_13201_amd import fsgmg, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("prec,sw,sv", [("fp64", 8, 8), ("fp32", 4, 4), ("bf16", 2, 4)])
def test_smoother_bytes_from_oracle_blocks(prec, sw, sv):
    import bench
    cfg = inputs.with_levels(inputs.config("c2"), 3)
    w = inputs.advecting_field(cfg)
    H = fsgmg.Hierarchy(cfg, w, device=-1)
    fsgmg.build_fs_as_blocks(H.h, core=cfg["core"], halo=cfg["halo"])
    O = OracleHierarchy(cfg, w, build_smoothers=False)
    for l in range(1, H.L):
        got, nblk = bench.smoother_bytes(H, l, prec)
        blocks, _ = build_blocks(O.levels[l], cfg["core"], cfg["halo"])
        own = owners(O.levels[l].N, blocks)
        total = 0
        for j, I in enumerate(blocks):
            m = int((own[I] == j).sum())      # rows of block j's inverse that are kept
            total += len(I) * m * sw + 4 * (len(I) + m)
        total += 3 * O.levels[l].N * sv
        assert nblk == len(blocks)
        assert got == total
    H.close()


@pytest.mark.parametrize("K", [1, 32])
def test_k_column_model_from_oracle_blocks(K):
    import bench
    cfg = inputs.with_levels(inputs.config("c2"), 3)
    w = inputs.advecting_field(cfg)
    H = fsgmg.Hierarchy(cfg, w, device=-1)
    fsgmg.build_fs_as_blocks(H.h, core=cfg["core"], halo=cfg["halo"])
    O = OracleHierarchy(cfg, w, build_smoothers=False)
    l = H.L - 1
    nbytes, flops = bench.mc_smoother_model(H, l, "fp32", K)
    blocks, _ = build_blocks(O.levels[l], cfg["core"], cfg["halo"])
    own = owners(O.levels[l].N, blocks)
    b = f = 0
    for j, I in enumerate(blocks):
        m = int((own[I] == j).sum())
        b += len(I) * m * 4 + 4 * (len(I) + m)
        f += 2 * len(I) * m * K        # one multiply-add per kept inverse entry and column
    b += 3 * O.levels[l].N * K * 4
    assert (nbytes, flops) == (b, f)
    # one column: the model reduces to the one-column sweep's bytes
    if K == 1:
        assert nbytes == bench.smoother_bytes(H, l, "fp32")[0]
    H.close()

"""Write tests/golden/c3_fp64_cycle_samples.txt: the oracle's FP64 V-cycle
(and its transpose) on the full-size aneurysm-like workload (6 levels,
512 x 256 finest, 2.2 M unknowns) for a seeded right-hand side, as per-field
norms and sampled entries.  The oracle needs about five minutes and 23 GB
for this on eight cores, too long to run inside the GPU tests, which
compare the library's cycle with these values.

    python tests/golden/make_c3_cycle_samples.py

Calls only oracle/ and the seeded input generators.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.multigrid import Hierarchy  # noqa: E402
from paper_1909_13201_amd import inputs  # noqa: E402

SEED = 41            # right-hand side: default_rng(SEED).standard_normal(N)
NSAMP = 512          # sampled entries per field: default_rng(SEED + 1)
OUT = os.path.join(HERE, "c3_fp64_cycle_samples.txt")


def main():
    cfg = inputs.config("c3")
    w = inputs.advecting_field(cfg)
    O = Hierarchy(cfg, w)
    lv = O.finest
    N = lv.N
    r = np.random.default_rng(SEED).standard_normal(N)
    z = {tr: O.vcycle(r, transpose=tr) for tr in (False, True)}
    fields = {"d": (0, lv.off_ps), "ps": (lv.off_ps, lv.off_u), "u": (lv.off_u, lv.off_pf),
              "pf": (lv.off_pf, N)}
    rng = np.random.default_rng(SEED + 1)
    with open(OUT, "w") as fo:
        fo.write("# oracle FP64 V-cycle on c3 (full size), r = default_rng(%d).standard_normal(N)\n"
                 % SEED)
        fo.write("# written by tests/golden/make_c3_cycle_samples.py (oracle only)\n")
        fo.write("N %d\n" % N)
        for f, (a, b) in fields.items():
            fo.write("field %s %d %d %r %r\n" % (f, a, b, float(np.linalg.norm(z[False][a:b])),
                                                  float(np.linalg.norm(z[True][a:b]))))
        for f, (a, b) in fields.items():
            idx = np.sort(rng.choice(np.arange(a, b), size=min(NSAMP, b - a), replace=False))
            for i in idx:
                fo.write("s %s %d %r %r\n" % (f, i, float(z[False][i]), float(z[True][i])))
    print("wrote", OUT)


if __name__ == "__main__":
    main()

"""Per-field comparison of level vectors for the parity tests.

A level vector holds four fields of very different magnitudes (mesh
displacement d, solid pressure p^s, velocity u, fluid pressure p^f; in a
cycle's output on the channel workloads ||d|| is ~1e-6 of ||p^s||), so one
global 2-norm hardly sees the small fields.  Every comparison here reports
and bounds the relative error of each field against that field's own norm.
"""
from __future__ import annotations

import sys

import numpy as np

FIELDS = ("d", "ps", "u", "pf")


def field_slices(info):
    """Slices of the four fields in a level vector (info: level_info dict or
    an oracle Level, both carry off_ps / off_u / off_pf / N)."""
    g = (lambda k: info[k]) if isinstance(info, dict) else (lambda k: getattr(info, k))
    return {"d": slice(0, g("off_ps")), "ps": slice(g("off_ps"), g("off_u")),
            "u": slice(g("off_u"), g("off_pf")), "pf": slice(g("off_pf"), g("N"))}


def field_errors(x, ref, info):
    """{field: ||x_f - ref_f|| / ||ref_f||} (absolute when ref_f is zero)."""
    out = {}
    for k, sl in field_slices(info).items():
        nr = np.linalg.norm(ref[sl])
        nd = np.linalg.norm(np.asarray(x[sl]) - ref[sl])
        out[k] = nd / nr if nr > 0 else nd
    return out


def check_fields(x, ref, info, tol, label=""):
    """Assert every field's relative error <= tol (a number or a dict per
    field); print the four errors and the global one; return the errors."""
    e = field_errors(x, ref, info)
    glob = np.linalg.norm(np.asarray(x) - ref) / max(np.linalg.norm(ref), 1e-300)
    print("   %s per-field rel err: %s (global %.2e)"
          % (label, " ".join("%s %.2e" % (k, e[k]) for k in FIELDS), glob), flush=True)
    sys.stdout.flush()
    for k in FIELDS:
        t = tol[k] if isinstance(tol, dict) else tol
        assert e[k] <= t, "%s: field %s rel err %.3e > %.1e" % (label, k, e[k], t)
    return e

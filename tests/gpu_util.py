"""Shared helpers of the GPU tests: run a decode through the C ABI and
compare it with the oracle under the tiered parity criteria."""
from __future__ import annotations

import sys

import numpy as np

from paper_2004_09084_amd import qcmet as Q

APP_TOL = 1e-3   # |a - o| <= APP_TOL * max(|o|, 1)
# Binary16 message storage: the GPU rounds a float32 message and the oracle
# an FP64 one, so near a rounding boundary the stored messages can differ by
# one binary16 step, 2^-10 relative, i.e. at most 2^-10 * 32 = 0.03125 for
# |r| <= 30.  Allow two such steps on top of the FP32 tolerance.
FP16_EXTRA = 2.0 * 2.0 ** -10 * 32.0


def precision_bound(case: str) -> dict:
    """Allowances of a reduced-precision message mode (binary16, e4m3) for
    `case`, written by tests/golden/make_precision_bounds.py from an
    oracle-only perturbation study: bound_mean_frac / bound_max_frac (APPs
    outside the float32 tolerance, mean over frames / worst frame, as
    fractions of n) and bound_max_rel (largest |a - o| / max(|o|, 1))."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision_bounds.json")
    return json.load(open(path))["cases"][case]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).reshape(-1))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_decode(H, Z, L, S, T, flags=0, tuning=None, want_app=True):
    """Decode frames (frame-major numpy) with one code; numpy outputs."""
    import torch
    code = Q.Code(H, Z)
    F = L.shape[0]
    dec = Q.Decoder([code], [F], flags=flags, tuning=tuning)
    hard, app, fl = dec.decode(to_dev(L), to_dev(S), T, want_app=want_app)
    torch.cuda.synchronize()
    out = (hard.cpu().numpy().reshape(F, -1), None if app is None else app.cpu().numpy().reshape(F, -1),
           fl.cpu().numpy())
    return out


def compare(app_g, hard_g, fl_g, app_o, hard_o, fl_o, tol=APP_TOL, extra=0.0):
    """Per-frame parity statistics.  app_viol counts |a - o| > tol*max(|o|,1)
    + extra; strict_viol counts the same without `extra`."""
    F = app_o.shape[0]
    rows = []
    for f in range(F):
        o = app_o[f]
        g = app_g[f].astype(np.float64)
        lim = tol * np.maximum(np.abs(o), 1.0)
        bad_app = np.abs(g - o) > lim + extra
        rows.append(dict(frame=f, flag_o=int(fl_o[f]), flag_g=int(fl_g[f]),
                         bits_diff=int((hard_g[f] != hard_o[f]).sum()),
                         bits_diff_confident=int(((hard_g[f] != hard_o[f]) & (np.abs(o) > tol + extra)).sum()),
                         app_viol=int(bad_app.sum()),
                         strict_viol=int((np.abs(g - o) > lim).sum()),
                         max_rel=float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)))))
    return rows


def assert_tiered(rows, strict_all=False):
    """T1: flags identical on every frame.  T2: hard decisions identical and
    APP within tolerance on every frame the oracle flags as converged.
    strict_all: also require it on every other frame."""
    for r in rows:
        assert r["flag_o"] == r["flag_g"], r
        if r["flag_o"] or strict_all:
            assert r["bits_diff"] == 0, r
            assert r["app_viol"] == 0, r

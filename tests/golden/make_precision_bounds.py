"""Writes tests/golden/precision_bounds.json: how far the reduced-precision
message modes (binary16, e4m3) of the FP64 oracle move when their inputs
change by float32-sized amounts.  The GPU parity tests of those modes take
their allowances from this file.

Why a study: the GPU forms each message in float32 (Phi's fit has 1.4e-6
relative error, plus a few float32 roundings) and then rounds it to the
storage format, while the oracle forms it in FP64.  Whenever the two values
lie on different sides of a rounding boundary of the storage format (one
binary16 step is 2^-10 relative, one e4m3 step 1/16 to 1/8), the stored
messages differ by one step, and the difference spreads through the rest of
the sweep.  The rate of such straddles is about (relative error) / (step),
so the float32 result is not expected to match the rounded oracle exactly;
how many APPs leave the float32 tolerance follows from the decoder's
dynamics, which only a decode can show.

Method (oracle only): decode the test's frames in the oracle's reduced mode,
then again with every channel LLR multiplied by (1 + eps u), u uniform in
[-1, 1], eps = 2e-6 (the float32 path's relative error), and compare the
two FP64 decodes with the float32 parity criterion |a - o| <= 1e-3 max(|o|, 1).
Several perturbation draws over more frames than the tests use; the stored
bounds are twice the worst figure seen (rounded up): the worst frame, the
worst mean over batches of as many frames as the GPU test decodes, and the
largest relative deviation.  Converged frames must keep identical flags and
hard decisions.

    python tests/golden/make_precision_bounds.py      (about a minute)
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_09084_amd import workload as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_bounds.json")
EPS = 2e-6
TOL = 1e-3
SPEC = W.RATE01_SMALL

# (case, decoder, message mode, SNR, frames in the study, sweeps, frames per
# GPU test batch: the mean fraction is the worst mean over batches of that
# many frames, as the GPU test takes it)
CASES = [
    ("fp16_layered", "layered", "fp16", 0.161, 64, (1, 2), 4),
    ("fp16_flooding", "flooding", "fp16", 0.161, 64, (1, 2), 4),
    ("fp8_layered", "layered", "fp8", 0.161, 64, (1, 2), 16),
]


def decode(kind, mode, H, L, S, T):
    kw = {"fp16_messages": mode == "fp16", "fp8_messages": mode == "fp8"}
    if kind == "flooding":
        return oracle.decode_flood(H, SPEC.Z, L, S, T, **kw)
    return oracle.decode_sp(H, SPEC.Z, L, S, T, **kw)


def study(kind, mode, snr, F, T, batch, trials=6, seed=0):
    H = W.make_code(SPEC, 0)
    _, L, S = W.make_frames(H, SPEC.Z, snr, F, seed=100 + seed)
    app0, hard0, fl0, _ = decode(kind, mode, H, L, S, T)
    fracs, rels, flag_diff = [], [], 0
    for t in range(trials):
        u = np.random.default_rng(1000 * seed + t).uniform(-1.0, 1.0, L.shape)
        Lp = (L.astype(np.float64) * (1.0 + EPS * u)).astype(np.float32)
        app1, hard1, fl1, _ = decode(kind, mode, H, Lp, S, T)
        lim = TOL * np.maximum(np.abs(app0), 1.0)
        out = np.abs(app1 - app0) > lim
        fracs.append(out.mean(axis=1))
        rels.append(float(np.max(np.abs(app1 - app0) / np.maximum(np.abs(app0), 1.0))))
        flag_diff += int((fl1 != fl0).sum())
        for f in np.nonzero(fl0 & fl1)[0]:
            assert np.array_equal(hard0[f], hard1[f]), (kind, mode, T, f)
    fr = np.concatenate(fracs)
    batch_means = fr[:len(fr) // batch * batch].reshape(-1, batch).mean(axis=1)
    return dict(mean_frac=float(batch_means.max()), max_frac=float(fr.max()), max_rel=float(np.max(rels)),
                flag_diff=flag_diff, frames=F * trials, batch=batch)


def up(x, digits=2):
    """Twice x, rounded up at `digits` significant digits (at least 1e-4)."""
    v = max(2.0 * x, 1e-4)
    e = math.floor(math.log10(v)) - digits + 1
    return float(f"{math.ceil(v / 10 ** e)}e{e}")


def main():
    out = {"eps": EPS, "tol": TOL, "code": SPEC.name, "cases": {}}
    for name, kind, mode, snr, F, Ts, batch in CASES:
        for T in Ts:
            r = study(kind, mode, snr, F, T, batch)
            key = f"{name}_T{T}"
            out["cases"][key] = {"measured": r,
                                 "bound_mean_frac": up(r["mean_frac"]), "bound_max_frac": up(r["max_frac"]),
                                 "bound_max_rel": up(r["max_rel"])}
            print(key, out["cases"][key], flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()

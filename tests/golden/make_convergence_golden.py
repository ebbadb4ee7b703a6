"""Writes tests/golden/convergence_oracle.json: per-frame convergence of
the oracle's layered sum-product decode (200 sweeps, no early stop) on the
128-frame rate-0.1 workload at two waterfall SNRs, for the paired
comparison of the GPU's FP32 and binary16 forms with it (the precision
form's shift of the syndrome-fail rate and FER on the same frames).

Calls only the oracle and the seeded workload generator (graph seed 0,
frame seed 0, frames 0-127).  Modes, each stored per SNR as the flag
(H c = s) and whether the hard decisions equal the transmitted word, per
frame:

  fp64       the FP64 oracle
  fp16       the oracle's binary16-message mode (messages rounded to
             binary16 where they are stored, as the GPU's FP16 form does)
  fp64_pert  fp64 with every LLR scaled by (1 + 2e-6 u), u uniform in
             [-1, 1] (seeded): how many frames change their outcome under
             a perturbation of the size of the FP32 path's relative error
  fp16_pert  the same perturbation in binary16 mode

The perturbed modes bound how many frames may legitimately differ between
two decodes whose arithmetic differs at that level; the GPU test takes
its allowance from them.

    python tests/golden/make_convergence_golden.py [mode ...]
        (default: all four; about 30 minutes per mode and SNR on 8 cores;
        the file is rewritten after every mode and SNR, keeping the others)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_09084_amd import workload as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "convergence_oracle.json")
SPEC = W.RATE01
F, T = 128, 200
SNRS = (0.5, 0.6)
CHUNK = 16
MODES = ("fp64", "fp16", "fp64_pert", "fp16_pert")
PERT_EPS = 2e-6
PERT_SEED = 7


def _load():
    if not os.path.exists(OUT):
        return {"code": SPEC.name, "frames": F, "sweeps": T, "graph_seed": 0, "frame_seed": 0,
                "pert_eps": PERT_EPS, "pert_seed": PERT_SEED, "snr": {}}
    with open(OUT) as fh:
        out = json.load(fh)
    out.setdefault("pert_eps", PERT_EPS)
    out.setdefault("pert_seed", PERT_SEED)
    for key, rec in out["snr"].items():
        if "flag" in rec:  # a file of the FP64 mode alone
            out["snr"][key] = {"fp64": rec}
    return out


def _save(out):
    with open(OUT, "w") as fh:
        json.dump(out, fh)
        fh.write("\n")


def run_mode(H, snr, mode):
    fp16 = mode.startswith("fp16")
    rng = np.random.default_rng([PERT_SEED, int(round(snr * 1000))])
    flags, correct = [], []
    t0 = time.time()
    for f0 in range(0, F, CHUNK):
        X, L, S = W.make_frames(H, SPEC.Z, snr, CHUNK, seed=0, first=f0)
        if mode.endswith("_pert"):
            u = rng.uniform(-1.0, 1.0, L.shape)
            L = (L.astype(np.float64) * (1.0 + PERT_EPS * u)).astype(np.float32)
        _, hard, fl, _ = oracle.decode_sp(H, SPEC.Z, L, S, T, fp16_messages=fp16, threads=8)
        flags += [int(v) for v in fl]
        correct += [int(np.array_equal(hard[i], X[i])) for i in range(CHUNK)]
        print(f"{mode} SNR {snr}: frames {f0}-{f0 + CHUNK - 1} done, {time.time() - t0:.0f} s", flush=True)
    return {"flag": flags, "correct": correct,
            "syndrome_fail": 1.0 - sum(flags) / F, "fer": 1.0 - sum(correct) / F}


def main(modes):
    H = W.make_code(SPEC, 0)
    out = _load()
    for mode in modes:
        for snr in SNRS:
            rec = out["snr"].setdefault(str(snr), {})
            if mode in rec:
                continue
            rec[mode] = run_mode(H, snr, mode)
            _save(out)
            print("wrote", OUT, mode, snr, flush=True)


if __name__ == "__main__":
    bad = [m for m in sys.argv[1:] if m not in MODES]
    if bad:
        raise SystemExit(f"unknown mode(s) {bad}; modes: {MODES}")
    main(sys.argv[1:] or MODES)

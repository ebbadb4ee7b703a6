"""Writes tests/golden/convergence_oracle.json: per-frame convergence of
the FP64 oracle's layered sum-product decode (200 sweeps, no early stop)
on the 128-frame rate-0.1 workload at two waterfall SNRs, for the paired
comparison of the GPU's FP32 and binary16 forms with it (the
precision form's shift of the syndrome-fail rate and FER).

Calls only the oracle and the seeded workload generator (graph seed 0,
frame seed 0, frames 0-127).  Stored per SNR: the flag (H c = s) and
whether the hard decisions equal the transmitted word, per frame.

    python tests/golden/make_convergence_golden.py   (about 40 minutes on 8 cores)
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


def main():
    H = W.make_code(SPEC, 0)
    out = {"code": SPEC.name, "frames": F, "sweeps": T, "graph_seed": 0, "frame_seed": 0, "snr": {}}
    for snr in SNRS:
        flags, correct = [], []
        t0 = time.time()
        for f0 in range(0, F, CHUNK):
            X, L, S = W.make_frames(H, SPEC.Z, snr, CHUNK, seed=0, first=f0)
            _, hard, fl, _ = oracle.decode_sp(H, SPEC.Z, L, S, T, threads=8)
            flags += [int(v) for v in fl]
            correct += [int(np.array_equal(hard[i], X[i])) for i in range(CHUNK)]
            print(f"SNR {snr}: frames {f0}-{f0 + CHUNK - 1} done, {time.time() - t0:.0f} s", flush=True)
        out["snr"][str(snr)] = {"flag": flags, "correct": correct,
                                "syndrome_fail": 1.0 - sum(flags) / F, "fer": 1.0 - sum(correct) / F}
    with open(OUT, "w") as fh:
        json.dump(out, fh)
        fh.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()

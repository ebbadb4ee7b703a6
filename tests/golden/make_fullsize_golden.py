"""Writes tests/golden/fullsize_oracle.npz: FP64 oracle results for sampled
frames of the full-size workloads (n = 10^6, graph seed 0, frame seed 0),
decoded alone (frames are independent), for the GPU parity test that decodes
the whole 128-frame batch.

Calls only the oracle and the seeded workload generator.  Stored per case:
flag, hard-decision errors against the truth, a SHA-256 of the hard
decisions, and the hard bits and APP values at 4096 sampled positions.

    python tests/golden/make_fullsize_golden.py            (all cases; about 25 minutes on 8 cores)
    python tests/golden/make_fullsize_golden.py CASE ...   (only these; the others are kept)

A case whose name ends in _fp16 decodes in the oracle's binary16-message
mode.  The SNRs of the converging cases sit on each code's waterfall, where
some frames reach a valid word and others do not.
"""
import concurrent.futures as cf
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_09084_amd import workload as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_oracle.npz")
SAMPLE = 4096

# (case name, spec, SNR or None for the spec's own, frames, iterations)
CASES = [
    ("r0.1_T200", W.RATE01, None, (0, 77), 200),
    ("r0.05_T200", W.RATE005, None, (0, 77), 200),
    ("r0.02_T200", W.RATE002, None, (0, 77), 200),
    ("r0.1_snr0.5_T60", W.RATE01, 0.5, (3, 100), 60),
    ("r0.05_snr0.2_T200", W.RATE005, 0.2, (0, 4), 200),
    ("r0.02_snr0.12_T200", W.RATE002, 0.12, (0, 2), 200),
    ("r0.1_snr0.5_T60_fp16", W.RATE01, 0.5, (1, 2), 60),
]


def positions(n, seed=123):
    return np.sort(np.random.default_rng(seed).choice(n, SAMPLE, replace=False)).astype(np.int64)


def run_case(case):
    name, spec, snr, frames, T = case
    H = W.make_code(spec, 0)
    snr_v = spec.snr if snr is None else snr
    X, L, S = [], [], []
    for f in frames:
        x, l, s = W.make_frame(H, spec.Z, snr_v, 0, f)
        X.append(x); L.append(l); S.append(s)
    X, L, S = np.array(X), np.array(L), np.array(S)
    t0 = time.time()
    app, hard, flags, _ = oracle.decode_sp(H, spec.Z, L, S, T, threads=len(frames),
                                           fp16_messages=name.endswith("_fp16"))
    pos = positions(spec.n)
    res = {}
    for i, f in enumerate(frames):
        p = f"{name}/f{f}/"
        res[p + "flag"] = np.array(flags[i])
        res[p + "errors"] = np.array(int((hard[i] != X[i]).sum()))
        res[p + "hard_sha256"] = np.frombuffer(hashlib.sha256(hard[i].tobytes()).digest(), dtype=np.uint8)
        res[p + "pos"] = pos
        res[p + "hard_at"] = hard[i][pos]
        res[p + "app_at"] = app[i][pos]
    res[f"{name}/meta"] = np.array([snr_v, T, spec.Z] + list(frames), dtype=np.float64)
    print(f"{name}: {time.time() - t0:.0f} s, flags {flags.tolist()}", flush=True)
    return res


def main():
    only = set(sys.argv[1:])
    unknown = only - {c[0] for c in CASES}
    if unknown:
        raise SystemExit(f"unknown cases: {sorted(unknown)}")
    cases = [c for c in CASES if not only or c[0] in only]
    out = {}
    if only and os.path.exists(OUT):
        old = np.load(OUT)
        out = {k: old[k] for k in old.files if k.split("/")[0] not in only}
    with cf.ThreadPoolExecutor(max_workers=len(cases)) as ex:
        for r in ex.map(run_case, cases):
            out.update(r)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()

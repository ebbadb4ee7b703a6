"""Seeded synthetic workloads: QC-MET-LDPC base matrices and BIAWGN frames.

This module only draws inputs. It holds none of the decoder's arithmetic and
is shared by the decoder tests, the benchmark and the CPU oracle's tests, so
that both sides are fed identical arrays.

Conventions (paper, Results, the base-matrix example around Eq. (m)):
a base entry a >= 0 stands for the Z x Z identity cyclically shifted right by
a, so check row k of block row i meets variable (k + a) mod Z of block column
j; a = -1 is an all-zero block.

Code construction (a multi-edge-type structure like the paper's codes, whose
own base matrices are not published):
  * block columns 0 .. ncol1-1 carry the "type-1" edges: each (row, column)
    entry is present with probability p; a row is redrawn until it holds at
    least ``min_type1`` type-1 entries;
  * block column ncol1 + i is a degree-1 column attached to block row i only;
  * every shift is uniform in [0, Z).

Frames (Methods, step 1): x is uniform random bits, BPSK maps bit b to
1 - 2b, y = 1 - 2x + N(0, sigma^2) with sigma^2 = 1/SNR, and the channel LLR
is 2 y / sigma^2 (stored as float32); the syndrome is s = H x mod 2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class CodeSpec:
    name: str
    mb: int          # base rows
    nb: int          # base columns
    Z: int           # lifting (expansion) factor
    ncol1: int       # number of type-1 block columns (0 .. ncol1-1)
    p: float         # presence probability of a type-1 entry
    snr: float       # operating SNR of the workload
    min_type1: int = 2  # a row is redrawn until it has this many type-1 entries

    @property
    def n(self) -> int:
        return self.nb * self.Z

    @property
    def m(self) -> int:
        return self.mb * self.Z

    @property
    def rate(self) -> float:
        return 1.0 - self.mb / self.nb

    def with_Z(self, Z: int) -> "CodeSpec":
        return CodeSpec(self.name + f"_Z{Z}", self.mb, self.nb, Z, self.ncol1,
                        self.p, self.snr, self.min_type1)


# The workloads: rate 0.1 / 0.05 / 0.02 codes of length 10^6 and the small
# rate-0.1 case (Z = 64, n = 3200) that the CPU oracle decodes in seconds.
RATE01_SMALL = CodeSpec("r0.1_Z64", 45, 50, 64, 5, 0.5, 0.161)
RATE01 = CodeSpec("r0.1_Z20000", 45, 50, 20000, 5, 0.5, 0.161)
RATE005 = CodeSpec("r0.05_Z10000", 95, 100, 10000, 5, 0.5, 0.076)
RATE002 = CodeSpec("r0.02_Z10000", 98, 100, 10000, 2, 0.9, 0.03)

SPECS = {s.name: s for s in (RATE01_SMALL, RATE01, RATE005, RATE002)}


def _graph_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(0,))))


def _frame_rng(seed: int, frame: int) -> np.random.Generator:
    # one independent stream per frame, so any frame can be drawn on its own
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(1, frame))))


def make_code(spec: CodeSpec, seed: int = 0) -> np.ndarray:
    """Base matrix of shifts, int32 [mb, nb] with -1 for an all-zero block."""
    if spec.ncol1 + spec.mb != spec.nb:
        raise ValueError("need nb == ncol1 + mb (one degree-1 column per row)")
    rng = _graph_rng(seed)
    present = np.zeros((spec.mb, spec.ncol1), dtype=bool)
    for i in range(spec.mb):
        while True:
            row = rng.random(spec.ncol1) < spec.p
            if row.sum() >= spec.min_type1:
                break
        present[i] = row
    H = np.full((spec.mb, spec.nb), -1, dtype=np.int32)
    for i in range(spec.mb):
        for j in range(spec.ncol1):
            if present[i, j]:
                H[i, j] = rng.integers(0, spec.Z)
    for i in range(spec.mb):
        H[i, spec.ncol1 + i] = rng.integers(0, spec.Z)
    return H


def syndrome(shifts: np.ndarray, Z: int, x: np.ndarray) -> np.ndarray:
    """s = H x mod 2 for bits x [..., nb*Z] (uint8); returns uint8 [..., mb*Z]."""
    mb, nb = shifts.shape
    x = np.asarray(x, dtype=np.uint8)
    lead = x.shape[:-1]
    xb = x.reshape(lead + (nb, Z))
    s = np.zeros(lead + (mb, Z), dtype=np.uint8)
    k = np.arange(Z)
    for i in range(mb):
        for j in range(nb):
            a = int(shifts[i, j])
            if a >= 0:
                s[..., i, :] ^= xb[..., j, (k + a) % Z]
    return s.reshape(lead + (mb * Z,))


def make_frame(shifts: np.ndarray, Z: int, snr: float, seed: int, frame: int,
               zero_noise: bool = False):
    """One frame: (x uint8 [n], llr float32 [n], s uint8 [m])."""
    mb, nb = shifts.shape
    n = nb * Z
    rng = _frame_rng(seed, frame)
    x = rng.integers(0, 2, n).astype(np.uint8)
    sigma2 = 1.0 / snr
    noise = rng.normal(0.0, np.sqrt(sigma2), n)
    y = 1.0 - 2.0 * x.astype(np.float64)
    if not zero_noise:
        y = y + noise
    llr = (2.0 * y / sigma2).astype(np.float32)
    s = syndrome(shifts, Z, x)
    return x, llr, s


def make_frames(shifts: np.ndarray, Z: int, snr: float, F: int, seed: int,
                first: int = 0, zero_noise: bool = False):
    """F frames (frame-major): x uint8 [F, n], llr float32 [F, n], s uint8 [F, m]."""
    mb, nb = shifts.shape
    n, m = nb * Z, mb * Z
    X = np.empty((F, n), dtype=np.uint8)
    L = np.empty((F, n), dtype=np.float32)
    S = np.empty((F, m), dtype=np.uint8)
    for f in range(F):
        X[f], L[f], S[f] = make_frame(shifts, Z, snr, seed, first + f, zero_noise)
    return X, L, S


@dataclass
class Workload:
    spec: CodeSpec
    shifts: np.ndarray
    x: np.ndarray
    llr: np.ndarray
    s: np.ndarray
    meta: dict = field(default_factory=dict)


def build(spec: CodeSpec, F: int, graph_seed: int = 0, frame_seed: int = 0,
          snr: float | None = None, first: int = 0) -> Workload:
    H = make_code(spec, graph_seed)
    snr = spec.snr if snr is None else snr
    X, L, S = make_frames(H, spec.Z, snr, F, frame_seed, first=first)
    return Workload(spec, H, X, L, S, dict(graph_seed=graph_seed, frame_seed=frame_seed,
                                          snr=snr, F=F, first=first))

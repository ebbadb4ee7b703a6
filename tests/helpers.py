"""Independent helpers for the tests: dense parity-check matrices, brute-force
MAP / ML decoding over a coset, small hand-built codes.  None of this calls
the oracle or the GPU library."""
from __future__ import annotations

import itertools

import numpy as np


def dense_H(shifts: np.ndarray, Z: int) -> np.ndarray:
    """Explicit H (uint8 [mb*Z, nb*Z]): block (i, j) with shift a >= 0 is the
    identity shifted right by a, i.e. row k has its 1 in column (k + a) mod Z."""
    mb, nb = shifts.shape
    H = np.zeros((mb * Z, nb * Z), dtype=np.uint8)
    for i in range(mb):
        for j in range(nb):
            a = int(shifts[i, j])
            if a < 0:
                continue
            for k in range(Z):
                H[i * Z + k, j * Z + (k + a) % Z] = 1
    return H


def coset(H: np.ndarray, s: np.ndarray) -> np.ndarray:
    """All x in {0,1}^n with H x = s (brute force; n <= ~20)."""
    n = H.shape[1]
    X = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.uint8)
    ok = ((X.astype(np.int64) @ H.T.astype(np.int64)) % 2 == s[None, :]).all(axis=1)
    return X[ok]


def map_llr(H, s, llr):
    """Exact bitwise a-posteriori LLRs ln P(x_n=0 | y, s) / P(x_n=1 | y, s)
    with P(y_n | x_n) proportional to exp(llr_n (1 - 2 x_n) / 2)."""
    C = coset(H, s)
    logw = 0.5 * ((1.0 - 2.0 * C) @ llr.astype(np.float64))
    mx = logw.max()
    w = np.exp(logw - mx)
    out = np.empty(H.shape[1])
    for v in range(H.shape[1]):
        p0 = w[C[:, v] == 0].sum()
        p1 = w[C[:, v] == 1].sum()
        out[v] = np.log(p0) - np.log(p1)
    return out


def ml_word(H, s, llr):
    """Block maximum-likelihood word in the coset {x : H x = s}."""
    C = coset(H, s)
    logw = (1.0 - 2.0 * C) @ llr.astype(np.float64)
    return C[int(np.argmax(logw))]


def random_tree_base(rng, n_rows: int, max_new: int = 2):
    """A base matrix whose row/column bipartite graph is a tree: every new
    row attaches to one existing column and opens 1..max_new new columns."""
    cols = 1
    rows = []
    for _ in range(n_rows):
        anchor = int(rng.integers(0, cols))
        new = int(rng.integers(1, max_new + 1))
        members = [anchor] + list(range(cols, cols + new))
        cols += new
        rows.append(members)
    H = np.full((n_rows, cols), -1, dtype=np.int32)
    for i, mem in enumerate(rows):
        for j in mem:
            H[i, j] = 0
    return H


def lift(base01: np.ndarray, Z: int, rng) -> np.ndarray:
    """Give every present entry of a 0/-1 pattern a random shift in [0, Z)."""
    H = np.where(base01 >= 0, rng.integers(0, Z, base01.shape), -1).astype(np.int32)
    return H


def frame_for(H_dense, x, snr, rng):
    sigma2 = 1.0 / snr
    y = 1.0 - 2.0 * x + rng.normal(0, np.sqrt(sigma2), x.shape)
    llr = (2.0 * y / sigma2).astype(np.float32)
    s = (H_dense.astype(np.int64) @ x.astype(np.int64) % 2).astype(np.uint8)
    return llr, s

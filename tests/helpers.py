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


# Philox4x32-10 (Salmon et al., SC 2011), vectorised over counters.
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    mask = np.uint64(0xFFFFFFFF)
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & mask for v in (c0, c1, c2, c3))
    k0, k1 = np.uint64(k0), np.uint64(k1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(_W0)) & mask
            k1 = (k1 + np.uint64(_W1)) & mask
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & mask, lo1, (hi0 ^ c3 ^ k1) & mask, lo0
    return c0, c1, c2, c3


def philox_frame(n, seed, frame, snr):
    """The GPU frame generator's definition in FP64: (x bits, standard normals)."""
    p = np.arange((n + 1) // 2, dtype=np.uint64)
    r0, r1, r2, r3 = philox4x32_10(p, frame & 0xFFFFFFFF, frame >> 32, 0, seed & 0xFFFFFFFF, seed >> 32)
    u1 = (r0.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (r1.astype(np.float64) + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    x = np.empty(2 * len(p), dtype=np.uint8)
    x[0::2] = (r2 >> np.uint64(31)).astype(np.uint8)
    x[1::2] = (r3 >> np.uint64(31)).astype(np.uint8)
    nrm = np.empty(2 * len(p))
    nrm[0::2] = rad * np.cos(2 * np.pi * u2)
    nrm[1::2] = rad * np.sin(2 * np.pi * u2)
    return x[:n], nrm[:n]

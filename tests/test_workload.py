"""The seeded input generator: determinism, code structure, s = H x."""
import numpy as np

from paper_2004_09084_amd import workload as W
from tests.helpers import dense_H


def test_code_structure_and_determinism():
    for spec in (W.RATE01_SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)):
        H = W.make_code(spec, 0)
        assert H.shape == (spec.mb, spec.nb)
        assert np.array_equal(H, W.make_code(spec, 0))
        assert not np.array_equal(H, W.make_code(spec, 1))
        t1 = H[:, :spec.ncol1] >= 0
        assert (t1.sum(1) >= spec.min_type1).all()
        d1 = H[:, spec.ncol1:]
        assert np.array_equal(d1 >= 0, np.eye(spec.mb, dtype=bool))
        assert ((H[H >= 0] >= 0) & (H[H >= 0] < spec.Z)).all()


def test_rate_and_sizes():
    assert W.RATE01.n == 10**6 and abs(W.RATE01.rate - 0.1) < 1e-12
    assert W.RATE005.n == 10**6 and abs(W.RATE005.rate - 0.05) < 1e-12
    assert W.RATE002.n == 10**6 and abs(W.RATE002.rate - 0.02) < 1e-12
    assert W.RATE01_SMALL.n == 3200


def test_syndrome_matches_dense_product():
    spec = W.RATE01_SMALL.with_Z(6)
    H = W.make_code(spec, 3)
    Hd = dense_H(H, spec.Z)
    rng = np.random.default_rng(0)
    x = rng.integers(0, 2, (3, spec.n)).astype(np.uint8)
    s = W.syndrome(H, spec.Z, x)
    ref = (x.astype(np.int64) @ Hd.T.astype(np.int64)) % 2
    assert np.array_equal(s, ref.astype(np.uint8))


def test_frames_deterministic_and_independent_of_batch():
    H = W.make_code(W.RATE01_SMALL, 0)
    X, L, S = W.make_frames(H, 64, 0.161, 4, seed=0)
    x2, l2, s2 = W.make_frame(H, 64, 0.161, 0, 2)
    assert np.array_equal(X[2], x2) and np.array_equal(L[2], l2) and np.array_equal(S[2], s2)
    Xb, Lb, Sb = W.make_frames(H, 64, 0.161, 2, seed=0, first=2)
    assert np.array_equal(Lb[0], L[2])
    assert L.dtype == np.float32 and X.dtype == np.uint8 and S.dtype == np.uint8


def test_llr_scale():
    # LLR = 2 y / sigma^2 = 2 SNR y; zero noise gives +-2 SNR exactly (in float32)
    H = W.make_code(W.RATE01_SMALL, 0)
    X, L, S = W.make_frames(H, 64, 0.25, 1, seed=0, zero_noise=True)
    assert np.array_equal(L[0], np.where(X[0] == 1, -0.5, 0.5).astype(np.float32))

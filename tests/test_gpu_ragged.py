"""Ragged and degenerate shapes against the FP64 oracle in every decoder
form: a frame count that fills two 16-frame tiles and part of a third, a
single frame, a lift of Z = 1 (every block a single edge) and a code of two
rows."""
import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.gpu_util import FP16_EXTRA, assert_tiered, compare, gpu_decode, say, to_dev

pytestmark = pytest.mark.gpu

SMALL = W.RATE01_SMALL


def _first_sweeps_ok(rows):
    for r in rows:
        assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0 and r["flag_o"] == r["flag_g"], r


@pytest.mark.parametrize("F", [37, 1])
def test_ragged_frame_counts_in_every_form(F):
    import torch
    wl = W.build(SMALL, F, snr=0.8, frame_seed=12)
    for T in (1, 2):
        say(f"F={F} T={T}")
        h, a, f = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T)
        appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, T)
        _first_sweeps_ok(compare(a, h, f, appo, hardo, flo))
        h, a, f = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T, flags=Q.QM_MSG_FP16)
        appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, T, fp16_messages=True)
        _first_sweeps_ok(compare(a, h, f, appo, hardo, flo, extra=FP16_EXTRA))
        h, a, f = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T, flags=Q.QM_FLOODING)
        appo, hardo, flo, _ = oracle.decode_flood(wl.shifts, SMALL.Z, wl.llr, wl.s, T)
        _first_sweeps_ok(compare(a, h, f, appo, hardo, flo))
    # fixed sweeps, converged frames bit-identical
    h, a, f = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 30)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, 30)
    assert_tiered(compare(a, h, f, appo, hardo, flo))
    assert flo.sum() >= 1
    # early termination
    code = Q.Code(wl.shifts, SMALL.Z)
    dec = Q.Decoder([code], [F], flags=Q.QM_EARLY_STOP)
    h, a, f, it = dec.decode_early(to_dev(wl.llr), to_dev(wl.s), 30)
    torch.cuda.synchronize()
    appo, hardo, flo, ito = oracle.decode_sp_early(wl.shifts, SMALL.Z, wl.llr, wl.s, 30)
    assert np.array_equal(it.cpu().numpy(), ito)
    assert_tiered(compare(a.cpu().numpy().reshape(F, -1), h.cpu().numpy().reshape(F, -1), f.cpu().numpy(),
                          appo, hardo, flo))
    # min-sum
    T = 3
    rng = np.random.default_rng(3)
    w = np.stack([rng.uniform(0.6, 1.0, (T, SMALL.mb, 2)), rng.uniform(0.0, 0.3, (T, SMALL.mb, 2))],
                 axis=-1).astype(np.float32)
    dec = Q.Decoder([code], [F])
    dec.nms_bind(T, False)
    h, a, f, _ = dec.nms_decode(to_dev(w), to_dev(wl.llr), to_dev(wl.s), T)
    torch.cuda.synchronize()
    appo, hardo, flo, _ = oracle.nms_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T, w[..., 0].astype(np.float64),
                                            w[..., 1].astype(np.float64))
    _first_sweeps_ok(compare(a.cpu().numpy().reshape(F, -1), h.cpu().numpy().reshape(F, -1), f.cpu().numpy(),
                             appo, hardo, flo))


def _frames(H, Z, F, snr, seed):
    from tests.helpers import dense_H, frame_for
    Hd = dense_H(H, Z)
    rng = np.random.default_rng(seed)
    L, S = [], []
    for _ in range(F):
        x = rng.integers(0, 2, Hd.shape[1]).astype(np.uint8)
        l, s = frame_for(Hd, x, snr, rng)
        L.append(l); S.append(s)
    return np.array(L, dtype=np.float32), np.array(S, dtype=np.uint8)


@pytest.mark.parametrize("which", ["lift_1", "two_rows"])
def test_degenerate_codes(which):
    if which == "lift_1":
        # the small code's base matrix itself (Z = 1): every block one edge
        H, Z = W.make_code(SMALL.with_Z(1), 0), 1
    else:
        # two rows sharing two columns, each with its own degree-1 column
        H, Z = np.array([[0, 3, 1, -1], [2, 5, -1, 4]], dtype=np.int32), 8
    L, S = _frames(H, Z, 20, 1.0, 4)
    for T in (1, 2, 10):
        h, a, f = gpu_decode(H, Z, L, S, T)
        appo, hardo, flo, _ = oracle.decode_sp(H, Z, L, S, T)
        rows = compare(a, h, f, appo, hardo, flo)
        if T <= 2:
            _first_sweeps_ok(rows)
        else:
            assert_tiered(rows)
        h, a, f = gpu_decode(H, Z, L, S, T, flags=Q.QM_FLOODING)
        appo, hardo, flo, _ = oracle.decode_flood(H, Z, L, S, T)
        rows = compare(a, h, f, appo, hardo, flo)
        if T <= 2:
            _first_sweeps_ok(rows)
        else:
            assert_tiered(rows)

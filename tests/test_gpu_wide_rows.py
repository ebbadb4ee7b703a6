"""Rows with 9 to 16 degree>=2 entries (the widest rows a code may have) on
the GPU against the FP64 oracle, in every layer-kernel mode: layered sweeps
with 1 and 2 frames per lane, binary16 messages, early termination,
flooding, a mixed batch, and the min-sum forward and gradient.  Such rows
take the kernels' 16-entry body, which must cover every lane the host
launches for the chosen frames per lane."""
import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import qcmet as Q
from tests.gpu_util import FP16_EXTRA, assert_tiered, compare, gpu_decode, say, to_dev

pytestmark = pytest.mark.gpu

Z = 24
NCOL1 = 16
ROW_DEGREES = (16, 9, 12, 3, 2, 5)   # degree>=2 entries per row


def _code(seed=0, with_degree1=True):
    # every one of the NCOL1 columns sits in row 0 and in row 1 or row 2, so
    # each has degree >= 2 and the only degree-1 columns are the diagonal ones
    rng = np.random.default_rng(seed)
    mb = len(ROW_DEGREES)
    nb = NCOL1 + (mb if with_degree1 else 0)
    H = np.full((mb, nb), -1, dtype=np.int32)
    row2 = rng.choice(NCOL1, ROW_DEGREES[2], replace=False)
    rest = np.setdiff1d(np.arange(NCOL1), row2)
    others = rng.choice(row2, ROW_DEGREES[1] - len(rest), replace=False)
    picks = {0: np.arange(NCOL1), 1: np.concatenate([rest, others]), 2: row2}
    for i, d in enumerate(ROW_DEGREES):
        cols = np.sort(picks[i] if i in picks else rng.choice(NCOL1, d, replace=False))
        assert len(cols) == d
        H[i, cols] = rng.integers(0, Z, d)
        if with_degree1:
            H[i, NCOL1 + i] = rng.integers(0, Z)
    assert ((H[:, :NCOL1] >= 0).sum(axis=0) >= 2).all()
    return H


def _frames(H, F, snr, seed):
    from tests.helpers import dense_H, frame_for
    Hd = dense_H(H, Z)
    rng = np.random.default_rng(seed)
    X, L, S = [], [], []
    for _ in range(F):
        x = rng.integers(0, 2, Hd.shape[1]).astype(np.uint8)
        l, s = frame_for(Hd, x, snr, rng)
        X.append(x); L.append(l); S.append(s)
    return np.array(X), np.array(L, dtype=np.float32), np.array(S, dtype=np.uint8)


def _first_sweeps_ok(rows):
    for r in rows:
        assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0 and r["flag_o"] == r["flag_g"], r


@pytest.mark.parametrize("with_degree1", [True, False])
@pytest.mark.parametrize("tun", [dict(frames_per_lane=2), dict(frames_per_lane=1),
                                 dict(frames_per_tile=4, block=64, frames_per_lane=2),
                                 dict(frames_per_tile=64, frames_per_lane=2)])
def test_wide_rows_layered_match_oracle(tun, with_degree1):
    H = _code(1, with_degree1)
    X, L, S = _frames(H, 20, 3.0, 2)
    for T in (1, 2, 3):
        say(f"wide rows {tun} degree1={with_degree1} T={T}")
        hard, app, fl = gpu_decode(H, Z, L, S, T, tuning=tun)
        appo, hardo, flo, _ = oracle.decode_sp(H, Z, L, S, T)
        _first_sweeps_ok(compare(app, hard, fl, appo, hardo, flo))
    hard, app, fl = gpu_decode(H, Z, L, S, 30, tuning=tun)
    appo, hardo, flo, _ = oracle.decode_sp(H, Z, L, S, 30)
    say(f"converged {int(flo.sum())}/20")
    assert_tiered(compare(app, hard, fl, appo, hardo, flo))


def test_wide_rows_fp16_messages():
    H = _code(2)
    X, L, S = _frames(H, 20, 0.9, 3)
    for T in (1, 2):
        hard, app, fl = gpu_decode(H, Z, L, S, T, flags=Q.QM_MSG_FP16)
        appo, hardo, flo, _ = oracle.decode_sp(H, Z, L, S, T, fp16_messages=True)
        for r in compare(app, hard, fl, appo, hardo, flo, extra=FP16_EXTRA):
            assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0 and r["flag_o"] == r["flag_g"], r


def test_wide_rows_early_termination_and_flooding():
    import torch
    H = _code(3)
    X, L, S = _frames(H, 20, 3.0, 4)
    code = Q.Code(H, Z)
    dec = Q.Decoder([code], [20], flags=Q.QM_EARLY_STOP)
    h, a, f, it = dec.decode_early(to_dev(L), to_dev(S), 25)
    torch.cuda.synchronize()
    appo, hardo, flo, ito = oracle.decode_sp_early(H, Z, L, S, 25)
    say("early stop iters", it.cpu().numpy().tolist(), ito.tolist())
    assert np.array_equal(it.cpu().numpy(), ito)
    assert_tiered(compare(a.cpu().numpy().reshape(20, -1), h.cpu().numpy().reshape(20, -1), f.cpu().numpy(),
                          appo, hardo, flo))
    assert flo.sum() >= 1
    for T in (1, 2):
        hard, app, fl = gpu_decode(H, Z, L, S, T, flags=Q.QM_FLOODING)
        appo, hardo, flo, _ = oracle.decode_flood(H, Z, L, S, T)
        _first_sweeps_ok(compare(app, hard, fl, appo, hardo, flo))


def test_wide_rows_in_a_mixed_batch():
    import torch
    Hs = [_code(4), _code(5, with_degree1=False)]
    Fs = [18, 7]
    data = [_frames(H, F, 0.9, 5 + i) for i, (H, F) in enumerate(zip(Hs, Fs))]
    codes = [Q.Code(H, Z) for H in Hs]
    L = to_dev(np.concatenate([d[1].reshape(-1) for d in data]))
    S = to_dev(np.concatenate([d[2].reshape(-1) for d in data]))
    for tun in (dict(fuse_codes=1), dict(fuse_codes=2), dict(fuse_codes=1, frames_per_lane=1)):
        dec = Q.Decoder(codes, Fs, tuning=tun)
        h, a, f = dec.decode(L, S, 2)
        torch.cuda.synchronize()
        h, a, f = h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()
        on = of = 0
        for H, F, d in zip(Hs, Fs, data):
            n = H.shape[1] * Z
            appo, hardo, flo, _ = oracle.decode_sp(H, Z, d[1], d[2], 2)
            _first_sweeps_ok(compare(a[on:on + F * n].reshape(F, -1), h[on:on + F * n].reshape(F, -1),
                                     f[of:of + F], appo, hardo, flo))
            on += F * n
            of += F


@pytest.mark.parametrize("fpl", [1, 2])
def test_wide_rows_min_sum_forward_and_gradient(fpl):
    import torch
    H = _code(6)
    mb = H.shape[0]
    F, T = 20, 3
    X, L, S = _frames(H, F, 3.0, 7)
    rng = np.random.default_rng(8)
    w = np.stack([rng.uniform(0.6, 1.0, (T, mb, 2)), rng.uniform(0.0, 0.3, (T, mb, 2))], axis=-1).astype(np.float32)
    a, b = w[..., 0].astype(np.float64), w[..., 1].astype(np.float64)
    code = Q.Code(H, Z)
    dec = Q.Decoder([code], [F], tuning=dict(frames_per_lane=fpl))
    dec.nms_bind(T, True)
    hard, app, fl, it = dec.nms_decode(to_dev(w), to_dev(L), to_dev(S), T)
    torch.cuda.synchronize()
    appo, hardo, flo, _ = oracle.nms_decode(H, Z, L, S, T, a, b)
    _first_sweeps_ok(compare(app.cpu().numpy().reshape(F, -1), hard.cpu().numpy().reshape(F, -1), fl.cpu().numpy(),
                             appo, hardo, flo))
    loss, grad = dec.nms_loss_grad(to_dev(w), to_dev(L), to_dev(S), to_dev(X), T)
    torch.cuda.synchronize()
    lo, ga, gb, _ = oracle.nms_loss_grad(H, Z, L, S, X, T, a, b)
    assert abs(float(loss.cpu()) - lo) <= 1e-5 * abs(lo)
    g = grad.cpu().numpy().reshape(T, mb, 2, 2).astype(np.float64)
    for comp, ref in ((0, ga), (1, gb)):
        err = np.abs(g[..., comp] - ref)
        lim = 1e-3 * np.abs(ref) + 2e-4 * np.abs(ref).max()
        assert np.all(err <= lim), (comp, fpl, np.argwhere(err > lim)[:5])

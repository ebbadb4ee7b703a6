"""Sum-product with early termination on the GPU (qm_decode_early): per-frame
iteration counts, flags and hard decisions against the FP64 oracle's
early-stopping decode; every frame equal to a fixed-iteration GPU decode at
its own count (bit-exact), which checks that stopped frames stay frozen
through the compaction of frame slots; edge cases."""
import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.gpu_util import APP_TOL, FP16_EXTRA, compare, say, to_dev

pytestmark = pytest.mark.gpu

SMALL = W.RATE01_SMALL


def _early(H, Z, L, S, T, flags=0, tuning=None):
    import torch
    F = L.shape[0]
    code = Q.Code(H, Z)
    dec = Q.Decoder([code], [F], flags=flags | Q.QM_EARLY_STOP, tuning=tuning)
    hard, app, fl, it = dec.decode_early(to_dev(L), to_dev(S), T)
    torch.cuda.synchronize()
    return (hard.cpu().numpy().reshape(F, -1), app.cpu().numpy().reshape(F, -1), fl.cpu().numpy(),
            it.cpu().numpy())


def _fixed(H, Z, L, S, T, flags=0, tuning=None):
    import torch
    F = L.shape[0]
    code = Q.Code(H, Z)
    dec = Q.Decoder([code], [F], flags=flags, tuning=tuning)
    hard, app, fl = dec.decode(to_dev(L), to_dev(S), T)
    torch.cuda.synchronize()
    return hard.cpu().numpy().reshape(F, -1), app.cpu().numpy().reshape(F, -1), fl.cpu().numpy()


def _frames(spec, F, snr, seed):
    wl = W.build(spec, F, snr=snr, frame_seed=seed)
    return wl.shifts, wl.llr, wl.s


def _assert_frozen_equal_fixed(H, Z, L, S, res, flags=0, tuning=None):
    """Each frame of an early-stopping decode equals a fixed decode of the
    whole batch at that frame's iteration count (bit-exact)."""
    hard, app, fl, it = res
    for t in sorted(set(it.tolist())):
        idx = np.nonzero(it == t)[0]
        hf, af, ff = _fixed(H, Z, L, S, int(t), flags=flags, tuning=tuning)
        assert np.array_equal(hf[idx], hard[idx]), t
        assert np.array_equal(af[idx].view(np.uint32), app[idx].view(np.uint32)), t
        assert np.array_equal(ff[idx], fl[idx]), t


@pytest.mark.parametrize("fp16", [False, True])
def test_early_matches_oracle(fp16):
    T = 25
    H, L, S = _frames(SMALL, 16, 0.25, 11)
    say(f"early small fp16={fp16}")
    hard, app, fl, it = _early(H, SMALL.Z, L, S, T, flags=Q.QM_MSG_FP16 if fp16 else 0)
    appo, hardo, flo, ito = oracle.decode_sp_early(H, SMALL.Z, L, S, T, fp16_messages=fp16)
    say("iters gpu", it.tolist(), "oracle", ito.tolist())
    assert flo.sum() >= 6 and (ito < T).sum() >= 6 and len(set(ito.tolist())) >= 3
    assert np.array_equal(it, ito)
    assert np.array_equal(fl, flo)
    rows = compare(app, hard, fl, appo, hardo, flo, extra=FP16_EXTRA if fp16 else 0.0)
    for r in rows:
        if r["flag_o"]:
            assert r["bits_diff"] == 0 and r["app_viol"] == 0, r


@pytest.mark.parametrize("fpl", [2, 1])
@pytest.mark.parametrize("ft", [1, 4, 16, 32, 64])
def test_early_frames_equal_fixed_decodes(ft, fpl):
    # 64 frames at a waterfall SNR: frames stop after 3 to 6 sweeps or never,
    # so tiles empty at several sweeps and frames are compacted several times;
    # every packed layout (frames per tile and per lane) of the tests
    T = 30
    H, L, S = _frames(SMALL, 64, 0.25, 12)
    tun = {"frames_per_tile": ft, "frames_per_lane": fpl}
    say(f"early vs fixed, FT={ft}, {fpl} frames per lane")
    res = _early(H, SMALL.Z, L, S, T, tuning=tun)
    say("iters", np.bincount(res[3]).tolist())
    assert (res[3] < T).sum() >= 16
    _assert_frozen_equal_fixed(H, SMALL.Z, L, S, res, tuning=tun)


# (SNR, frames, seed) groups of a 64-frame batch for the small rate-0.1 code.
# The SNR-0.25 group (seed 32) stops at sweeps 3-5 except 3 frames that never
# converge; with the fast frames that leaves 7 frames at the poll after
# sweep 4 and 3 at the next one: two narrowings (to 8, then 4 frames per
# tile), into each of the two tile regions in turn.  One never-converging
# frame among fast ones narrows to a single frame per tile (1 frame per lane).
NARROW_CASES = {
    "two_steps": ((0.6, 52, 31), (0.25, 12, 32)),
    "one_frame": ((0.6, 63, 31), (0.161, 1, 33)),
}


@pytest.mark.parametrize("flags", [0, Q.QM_MSG_FP16], ids=["fp32", "fp16"])
@pytest.mark.parametrize("case", sorted(NARROW_CASES))
def test_early_narrowed_tiles_equal_fixed_decodes(case, flags):
    # the frames still decoding are moved into narrower tiles, and every
    # frame still equals a fixed decode of the batch at its own count
    import torch
    T = 40
    H = W.make_code(SMALL, 0)
    parts = [W.make_frames(H, SMALL.Z, snr, F, seed=seed)[1:] for snr, F, seed in NARROW_CASES[case]]
    L = np.concatenate([p[0] for p in parts])
    S = np.concatenate([p[1] for p in parts])
    tun = {"frames_per_tile": 16}
    code = Q.Code(H, SMALL.Z)
    dec = Q.Decoder([code], [64], flags=flags | Q.QM_EARLY_STOP, tuning=tun)
    dec.profile(reset=True)
    hard, app, fl, it = dec.decode_early(to_dev(L), to_dev(S), T)
    torch.cuda.synchronize()
    narrowed = dec.profile(reset=True)["et_narrowings"]
    res = (hard.cpu().numpy().reshape(64, -1), app.cpu().numpy().reshape(64, -1), fl.cpu().numpy(), it.cpu().numpy())
    say(case, "narrowed", narrowed, "iters", np.bincount(res[3]).tolist())
    assert narrowed >= (2 if case == "two_steps" else 1)
    assert (res[3] == T).sum() >= 1
    _assert_frozen_equal_fixed(H, SMALL.Z, L, S, res, flags=flags, tuning=tun)


def test_early_fp16_frames_equal_fixed_decodes():
    T = 30
    H, L, S = _frames(SMALL, 48, 0.25, 13)
    tun = {"frames_per_tile": 8}
    res = _early(H, SMALL.Z, L, S, T, flags=Q.QM_MSG_FP16, tuning=tun)
    _assert_frozen_equal_fixed(H, SMALL.Z, L, S, res, flags=Q.QM_MSG_FP16, tuning=tun)


def test_early_zero_iterations_and_zero_noise():
    H = W.make_code(SMALL, 0)
    X, L, S = W.make_frames(H, SMALL.Z, 0.161, 5, seed=3, zero_noise=True)
    hard, app, fl, it = _early(H, SMALL.Z, L, S, 20)
    assert (it == 0).all() and fl.all() and np.array_equal(hard, X)
    assert np.array_equal(app, L)
    # max_iters = 0 on noisy frames: the channel decisions
    H2, L2, S2 = _frames(SMALL, 5, 0.3, 4)
    hard, app, fl, it = _early(H2, SMALL.Z, L2, S2, 0)
    assert (it == 0).all() and np.array_equal(app, L2) and np.array_equal(hard, (L2 < 0).astype(np.uint8))


def test_early_never_converging_runs_all_sweeps():
    T = 6
    H, L, S = _frames(SMALL, 8, 0.161, 5)
    hard, app, fl, it = _early(H, SMALL.Z, L, S, T)
    assert (it == T).all() and not fl.any()
    hf, af, ff = _fixed(H, SMALL.Z, L, S, T)
    assert np.array_equal(hf, hard) and np.array_equal(af.view(np.uint32), app.view(np.uint32))


def test_early_two_codes():
    import torch
    T = 25
    H1, L1, S1 = _frames(SMALL, 12, 0.25, 21)
    spec2 = W.RATE005.with_Z(32)
    H2, L2, S2 = _frames(spec2, 6, 0.15, 22)
    c1, c2 = Q.Code(H1, SMALL.Z), Q.Code(H2, spec2.Z)
    dec = Q.Decoder([c1, c2], [12, 6], flags=Q.QM_EARLY_STOP)
    Lc = np.concatenate([L1.reshape(-1), L2.reshape(-1)])
    Sc = np.concatenate([S1.reshape(-1), S2.reshape(-1)])
    hard, app, fl, it = dec.decode_early(to_dev(Lc), to_dev(Sc), T)
    torch.cuda.synchronize()
    it = it.cpu().numpy()
    fl = fl.cpu().numpy()
    hard = hard.cpu().numpy()
    n1 = 12 * SMALL.n
    _, h1, f1, i1 = oracle.decode_sp_early(H1, SMALL.Z, L1, S1, T)
    _, h2, f2, i2 = oracle.decode_sp_early(H2, spec2.Z, L2, S2, T)
    say("two codes iters", it.tolist(), i1.tolist() + i2.tolist())
    assert np.array_equal(it, np.concatenate([i1, i2]))
    assert np.array_equal(fl, np.concatenate([f1, f2]))
    conv = np.concatenate([f1, f2]).astype(bool)
    hg = np.concatenate([hard[:n1].reshape(12, -1)[f1 == 1].reshape(-1), hard[n1:].reshape(6, -1)[f2 == 1].reshape(-1)])
    ho = np.concatenate([h1[f1 == 1].reshape(-1), h2[f2 == 1].reshape(-1)])
    assert conv.sum() >= 4 and np.array_equal(hg, ho)


def test_early_needs_flag():
    code = Q.Code(W.make_code(SMALL, 0), SMALL.Z)
    dec = Q.Decoder([code], [4])
    import torch
    L = torch.zeros(4 * SMALL.n, device="cuda")
    S = torch.zeros(4 * SMALL.m, dtype=torch.uint8, device="cuda")
    with pytest.raises(Q.QMError) as e:
        dec.decode_early(L, S, 5)
    assert e.value.code == Q.QM_ERR_UNSUPPORTED


def test_early_fullsize_frames_equal_fixed_decodes():
    # rate 0.1, n = 10^6, 128 frames at SNR 0.6 in the default launch
    # configuration: frames that stop are bit-identical to a fixed decode at
    # their count; a sample is checked against the oracle's count
    import torch
    T = 60
    spec = W.RATE01
    wl = W.build(spec, 128, snr=0.6, frame_seed=3)
    code = Q.Code(wl.shifts, spec.Z)
    dec = Q.Decoder([code], [128], flags=Q.QM_EARLY_STOP)
    hard, app, fl, it = dec.decode_early(to_dev(wl.llr), to_dev(wl.s), T)
    torch.cuda.synchronize()
    it = it.cpu().numpy()
    say("full-size iters histogram", np.bincount(it).tolist())
    assert (it < T).sum() >= 64
    del dec
    torch.cuda.empty_cache()
    hard = hard.cpu().numpy().reshape(128, -1)
    fl = fl.cpu().numpy()
    fx = Q.Decoder([code], [128])
    for t in sorted(set(it.tolist()))[:3] + [int(it.max())]:
        idx = np.nonzero(it == t)[0]
        hf, _, ff = fx.decode(to_dev(wl.llr), to_dev(wl.s), int(t))
        torch.cuda.synchronize()
        hf = hf.cpu().numpy().reshape(128, -1)
        assert np.array_equal(hf[idx], hard[idx]) and np.array_equal(ff.cpu().numpy()[idx], fl[idx]), t
    f0 = int(np.argmin(it))
    _, ho, flo, ito = oracle.decode_sp_early(wl.shifts, spec.Z, wl.llr[f0:f0 + 1], wl.s[f0:f0 + 1], T)
    say("oracle frame", f0, "iters", int(ito[0]), "gpu", int(it[f0]))
    assert int(ito[0]) == int(it[f0]) and flo[0] == fl[f0]
    assert np.array_equal(ho[0], hard[f0])
    # the first 16 frames against the oracle's early-stopping decode: the
    # same stopping sweep, flag and 10^6 hard decisions, frame by frame
    frames = list(range(16))
    _, ho, flo, ito = oracle.decode_sp_early(wl.shifts, spec.Z, wl.llr[frames], wl.s[frames], T, threads=8)
    say("oracle iters", ito.tolist(), "gpu", it[frames].tolist())
    assert np.array_equal(ito, it[frames]) and np.array_equal(flo, fl[frames])
    for i, f in enumerate(frames):
        assert np.array_equal(ho[i], hard[f]), f"frame {f}"


def test_early_fullsize_fp16_against_oracle():
    # binary16 messages with early termination at n = 10^6 (128 frames, SNR
    # 0.6): the first 8 frames stop at the oracle's binary16-mode count with
    # its flag, and a converged frame's hard decisions and APPs agree with
    # it (APPs within the FP32 tolerance plus the binary16 allowance)
    import torch
    T = 60
    spec = W.RATE01
    wl = W.build(spec, 128, snr=0.6, frame_seed=3)
    code = Q.Code(wl.shifts, spec.Z)
    dec = Q.Decoder([code], [128], flags=Q.QM_EARLY_STOP | Q.QM_MSG_FP16)
    hard, app, fl, it = dec.decode_early(to_dev(wl.llr), to_dev(wl.s), T)
    torch.cuda.synchronize()
    it, fl = it.cpu().numpy(), fl.cpu().numpy()
    hard = hard.cpu().numpy().reshape(128, -1)
    app = app.cpu().numpy().reshape(128, -1)
    frames = list(range(8))
    appo, ho, flo, ito = oracle.decode_sp_early(wl.shifts, spec.Z, wl.llr[frames], wl.s[frames], T,
                                                fp16_messages=True, threads=8)
    say("oracle binary16 iters", ito.tolist(), "gpu", it[frames].tolist())
    assert np.array_equal(ito, it[frames]) and np.array_equal(flo, fl[frames])
    for i, f in enumerate(frames):
        rows = compare(app[f:f + 1], hard[f:f + 1], fl[f:f + 1], appo[i:i + 1], ho[i:i + 1], flo[i:i + 1],
                       extra=FP16_EXTRA)
        assert rows[0]["bits_diff_confident"] == 0 and rows[0]["flag_o"] == rows[0]["flag_g"], (f, rows[0])
        if rows[0]["flag_o"]:
            # a converged frame: every hard decision and every APP in tolerance
            assert rows[0]["bits_diff"] == 0 and rows[0]["app_viol"] == 0, (f, rows[0])



def _many_column_code(C, rowdeg, Z, seed):
    """mb = 2C/rowdeg rows; C columns of degree 2, rowdeg per row, and one
    degree-1 column per row: nb = C + mb base columns."""
    rng = np.random.default_rng(seed)
    mb = 2 * C // rowdeg
    slots = rng.permutation(np.repeat(np.arange(C), 2)).reshape(mb, rowdeg)
    for _ in range(100):
        bad = [i for i in range(mb) if len(set(slots[i].tolist())) < rowdeg]
        if not bad:
            break
        for i in bad:  # swap a repeated column with a random slot elsewhere
            j, a, b = int(rng.integers(0, mb)), int(rng.integers(0, rowdeg)), int(rng.integers(0, rowdeg))
            slots[i, b], slots[j, a] = slots[j, a], slots[i, b]
    assert all(len(set(r.tolist())) == rowdeg for r in slots)
    H = np.full((mb, C + mb), -1, dtype=np.int32)
    for i in range(mb):
        H[i, slots[i]] = rng.integers(0, Z, rowdeg)
        H[i, C + i] = rng.integers(0, Z)
    return H


def _sparse_frames(H, Z, snrs, seed):
    mb, nb = H.shape
    n, m = nb * Z, mb * Z
    rng = np.random.default_rng(seed)
    ii, jj = np.nonzero(H >= 0)
    k = np.arange(Z)
    rows = (ii[:, None] * Z + k[None, :]).ravel()
    cols = (jj[:, None] * Z + (k[None, :] + H[ii, jj][:, None]) % Z).ravel()
    L, S = [], []
    for snr in snrs:
        x = rng.integers(0, 2, n).astype(np.uint8)
        y = 1.0 - 2.0 * x + rng.normal(0.0, np.sqrt(1.0 / snr), n)
        s = np.zeros(m, dtype=np.uint8)
        np.bitwise_xor.at(s, rows, x[cols])
        L.append((2.0 * y * snr).astype(np.float32))
        S.append(s)
    return np.array(L), np.array(S)


def test_early_very_many_base_columns():
    # 40000 base columns (a column-to-row table of them would take 160 KB,
    # more than one workgroup's LDS): the output pass forms every stopped
    # frame's degree-1 APPs, bit-exact against fixed decodes at its count
    T, Z = 12, 2
    H = _many_column_code(32000, 8, Z, 0)
    assert H.shape == (8000, 40000)
    L, S = _sparse_frames(H, Z, np.repeat([4.0, 5.0, 6.0, 8.0], 4), 1)
    say("early, 40000 base columns")
    res = _early(H, Z, L, S, T)
    say("iters", res[3].tolist())
    assert (res[3] < T).sum() >= 4 and len(set(res[3].tolist())) >= 3
    _assert_frozen_equal_fixed(H, Z, L, S, res)

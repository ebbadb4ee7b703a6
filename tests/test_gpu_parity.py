"""GPU decode (through the C ABI) against the FP64 oracle on the same seeded
inputs.  Criteria: T0 -- after a few sweeps every APP within 1e-3 relative
(absolute below 1) and hard decisions identical wherever |APP| > 1e-3;
T1 -- per-frame syndrome flags identical; T2 -- frames the oracle decodes
to a valid word have identical hard decisions and APPs within tolerance."""
import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.gpu_util import APP_TOL, FP16_EXTRA, assert_tiered, compare, gpu_decode, precision_bound, say, to_dev

pytestmark = pytest.mark.gpu

SMALL = W.RATE01_SMALL        # rate 0.1, 45 x 50, Z = 64, n = 3200


def _wl(spec, F, snr=None, seed=0, graph_seed=0):
    return W.build(spec, F, graph_seed=graph_seed, frame_seed=seed, snr=snr)


def test_zero_iterations_return_channel_decisions():
    wl = _wl(SMALL, 4)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 0)
    assert np.array_equal(app, wl.llr)
    assert np.array_equal(hard, (wl.llr < 0).astype(np.uint8))
    _, _, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, 0)
    assert np.array_equal(fl, flo)


@pytest.mark.parametrize("T", [1, 2, 3])
def test_first_sweeps_match_oracle_everywhere(T):
    wl = _wl(SMALL, 4)
    say(f"T0 small T={T}")
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, T)
    rows = compare(app, hard, fl, appo, hardo, flo)
    say(rows)
    for r in rows:
        assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0, r
    assert np.array_equal(fl, flo)


def test_small_config_50_iterations():
    # rate 0.1, Z = 64, 4 frames, SNR 0.161, 50 iterations
    wl = _wl(SMALL, 4)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 50)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, 50)
    rows = compare(app, hard, fl, appo, hardo, flo)
    say("small cfg 50 it:", rows)
    assert_tiered(rows)


@pytest.mark.parametrize("snr", [0.45, 0.8])
def test_converging_frames_are_bit_exact(snr):
    wl = _wl(SMALL, 24, snr=snr, seed=3)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 50)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, 50)
    rows = compare(app, hard, fl, appo, hardo, flo)
    say(f"snr {snr}: converged {int(flo.sum())}/24", [r for r in rows if r["bits_diff"] or r["app_viol"]])
    assert_tiered(rows)
    assert flo.sum() >= 1


def test_ragged_lift_and_padded_frames():
    # Z = 37 and 5 frames: partial workgroups, a padded frame tile
    spec = SMALL.with_Z(37)
    wl = _wl(spec, 5, snr=0.6, seed=4)
    for T in (1, 2):
        hard, app, fl = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, T)
        appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, spec.Z, wl.llr, wl.s, T)
        for r in compare(app, hard, fl, appo, hardo, flo):
            assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0, r
    hard, app, fl = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, 40)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, spec.Z, wl.llr, wl.s, 40)
    assert_tiered(compare(app, hard, fl, appo, hardo, flo))


def test_rate002_and_rate005_structures_small_lift():
    for spec in (W.RATE005.with_Z(24), W.RATE002.with_Z(24)):
        wl = _wl(spec, 6, snr=spec.snr * 3, seed=5)
        for T in (1, 3):
            hard, app, fl = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, T)
            appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, spec.Z, wl.llr, wl.s, T)
            for r in compare(app, hard, fl, appo, hardo, flo):
                assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0, (spec.name, T, r)


def test_zero_noise_frames_decode_to_truth():
    X, L, S = W.make_frames(W.make_code(SMALL, 0), SMALL.Z, 0.161, 8, seed=7, zero_noise=True)
    hard, app, fl = gpu_decode(W.make_code(SMALL, 0), SMALL.Z, L, S, 5)
    assert fl.all() and np.array_equal(hard, X)


def test_codes_without_degree1_columns_and_tiny_checks():
    # a general QC code: no degree-1 columns, a row with a single entry,
    # an empty column; Z = 5
    H = np.array([[0, 1, -1, 3, -1], [2, -1, 4, 0, -1], [-1, 3, 1, -1, -1], [-1, -1, -1, 2, -1]], dtype=np.int32)
    Z = 5
    rng = np.random.default_rng(8)
    from tests.helpers import dense_H, frame_for
    Hd = dense_H(H, Z)
    L, S = [], []
    for f in range(3):
        x = rng.integers(0, 2, Hd.shape[1]).astype(np.uint8)
        l, s = frame_for(Hd, x, 1.0, rng)
        L.append(l); S.append(s)
    L, S = np.array(L), np.array(S)
    for T in (1, 4):
        hard, app, fl = gpu_decode(H, Z, L, S, T)
        appo, hardo, flo, _ = oracle.decode_sp(H, Z, L, S, T)
        for r in compare(app, hard, fl, appo, hardo, flo):
            assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0 and r["flag_o"] == r["flag_g"], r


# ------------------------------------------------- FP16 message storage --

@pytest.mark.parametrize("T", [1, 2])
def test_fp16_messages_match_oracle_binary16_mode(T):
    wl = _wl(SMALL, 4)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T, flags=Q.QM_MSG_FP16)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, T, fp16_messages=True)
    rows = compare(app, hard, fl, appo, hardo, flo, extra=FP16_EXTRA)
    say(f"fp16 T={T}", rows)
    # float32 and FP64 messages straddle a binary16 rounding boundary now and
    # then; how many APPs that moves outside the float32 tolerance, and how
    # far, is bounded by the oracle-only study in
    # tests/golden/make_precision_bounds.py
    b = precision_bound(f"fp16_layered_T{T}")
    for r in rows:
        assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0, r
        assert r["strict_viol"] <= b["bound_max_frac"] * SMALL.n, (r, b)
        assert r["max_rel"] <= b["bound_max_rel"], (r, b)


def test_fp16_messages_converging_frames():
    wl = _wl(SMALL, 16, snr=0.8, seed=3)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 40, flags=Q.QM_MSG_FP16)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, 40, fp16_messages=True)
    rows = compare(app, hard, fl, appo, hardo, flo, extra=FP16_EXTRA)
    say("fp16 converging:", int(flo.sum()), [r for r in rows if r["bits_diff"] or r["app_viol"]])
    assert_tiered(rows)


# ------------------------------------------------- GPU-vs-GPU invariants --

def test_tunings_are_bit_identical():
    wl = _wl(SMALL, 16, snr=0.3, seed=2)
    ref = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 12)
    for tun in (dict(frames_per_tile=1, frames_per_lane=1), dict(frames_per_tile=4, block=64, frames_per_lane=1), dict(frames_per_tile=8, block=128, frames_per_lane=2),
                dict(frames_per_tile=16, merge=0), dict(frames_per_tile=2, block=128, merge=0),
                dict(frames_per_tile=16, graph=1), dict(stream_hint=1), dict(frames_per_tile=32, stream_hint=1, merge=0)):
        got = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 12, tuning=tun)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2]), tun


def test_frames_are_independent_on_gpu():
    wl = _wl(SMALL, 12, snr=0.3, seed=6)
    allf = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9)
    part = gpu_decode(wl.shifts, SMALL.Z, wl.llr[5:8], wl.s[5:8], 9)
    assert np.array_equal(allf[1][5:8], part[1]) and np.array_equal(allf[0][5:8], part[0])


def test_multi_code_decoder_equals_single_code_decoders():
    import torch
    specs = [SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)]
    Fs = [6, 3, 5]
    wls = [_wl(s, F, snr=s.snr * 2, seed=1) for s, F in zip(specs, Fs)]
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    dec = Q.Decoder(codes, Fs)
    L = np.concatenate([w.llr.reshape(-1) for w in wls])
    S = np.concatenate([w.s.reshape(-1) for w in wls])
    hard, app, fl = dec.decode(to_dev(L), to_dev(S), 7)
    torch.cuda.synchronize()
    hard, app, fl = hard.cpu().numpy(), app.cpu().numpy(), fl.cpu().numpy()
    on = of = 0
    for w, s, F in zip(wls, specs, Fs):
        h1, a1, f1 = gpu_decode(w.shifts, s.Z, w.llr, w.s, 7)
        assert np.array_equal(app[on:on + F * s.n], a1.reshape(-1))
        assert np.array_equal(hard[on:on + F * s.n], h1.reshape(-1))
        assert np.array_equal(fl[of:of + F], f1)
        on += F * s.n
        of += F


def test_graph_replays_match_eager():
    import torch
    wl = _wl(SMALL, 8, snr=0.3, seed=9)
    ref = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 6)
    code = Q.Code(wl.shifts, SMALL.Z)
    dec = Q.Decoder([code], [8], tuning=dict(graph=1))
    L, S = to_dev(wl.llr), to_dev(wl.s)
    out = dec.alloc_outputs()
    for rep in range(4):
        dec.decode(L, S, 6, out=out)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(out[1].cpu().numpy().reshape(8, -1), ref[1]), rep
        assert np.array_equal(out[2].cpu().numpy(), ref[2]), rep
        out[1].fill_(7.0)
        out[0].fill_(3)


def test_validation_flag_rejects_bad_inputs():
    wl = _wl(SMALL, 2)
    code = Q.Code(wl.shifts, SMALL.Z)
    dec = Q.Decoder([code], [2], flags=Q.QM_VALIDATE)
    L = wl.llr.copy()
    L[1, 17] = np.nan
    with pytest.raises(Q.QMError) as e:
        dec.decode(to_dev(L), to_dev(wl.s), 2)
    assert e.value.code == Q.QM_ERR_INPUT
    S = wl.s.copy()
    S[0, 3] = 2
    with pytest.raises(Q.QMError) as e:
        dec.decode(to_dev(wl.llr), to_dev(S), 2)
    assert e.value.code == Q.QM_ERR_INPUT
    hard, app, fl = dec.decode(to_dev(wl.llr), to_dev(wl.s), 2)   # clean inputs pass


# ------------------------------------------------------- mixed batches --

def _mixed(specs, Fs, snr_scale=2.0, T=6):
    import torch
    wls = [_wl(s, F, snr=s.snr * snr_scale, seed=1) for s, F in zip(specs, Fs)]
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    L = to_dev(np.concatenate([w.llr.reshape(-1) for w in wls]))
    S = to_dev(np.concatenate([w.s.reshape(-1) for w in wls]))
    return wls, codes, L, S


def test_fused_mixed_batch_equals_unfused_and_single_code():
    import torch
    specs = [SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)]
    Fs = [64, 32, 32]
    wls, codes, L, S = _mixed(specs, Fs)
    outs = {}
    # fused launches with each code's layers spread over the launches, or
    # every code from the first launch on; each code on its own stream, with
    # the shorter chains' residency capped at the default 10, at 3 or not at
    # all; codes one after another
    modes = {"fused": dict(fuse_codes=1, spread_codes=1), "fused_unspread": dict(fuse_codes=1, spread_codes=0),
             "streams": dict(fuse_codes=2), "streams_cap3": dict(fuse_codes=2, resident_cap=3),
             "streams_nocap": dict(fuse_codes=2, resident_cap=0), "sequential": dict(fuse_codes=0)}
    for name, tun in modes.items():
        for flags in (0, Q.QM_MSG_FP16):
            dec = Q.Decoder(codes, Fs, flags=flags, tuning=tun)
            h, a, f = dec.decode(L, S, 9)
            torch.cuda.synchronize()
            outs[(name, flags)] = (h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy())
    for flags in (0, Q.QM_MSG_FP16):
        for name in modes:
            for x, y in zip(outs[("fused", flags)], outs[(name, flags)]):
                assert np.array_equal(x, y), (name, flags)
    # and against one decoder per code (FP32)
    on = of = 0
    for w, s, F in zip(wls, specs, Fs):
        h1, a1, f1 = gpu_decode(w.shifts, s.Z, w.llr, w.s, 9)
        assert np.array_equal(outs[("fused", 0)][1][on:on + F * s.n], a1.reshape(-1))
        assert np.array_equal(outs[("fused", 0)][2][of:of + F], f1)
        on += F * s.n
        of += F


def test_codes_without_frames():
    # a code given 0 frames takes no part (every mixed-batch mode, early
    # termination); a decoder with no frame at all decodes nothing, with
    # empty buffers
    import torch
    specs = [SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)]
    Fs = [5, 0, 3]
    wls = [_wl(s, max(F, 1), snr=0.4, seed=13 + i) for i, (s, F) in enumerate(zip(specs, Fs))]
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    L = to_dev(np.concatenate([w.llr[:F].reshape(-1) for w, F in zip(wls, Fs)]))
    S = to_dev(np.concatenate([w.s[:F].reshape(-1) for w, F in zip(wls, Fs)]))
    ref = [gpu_decode(w.shifts, s.Z, w.llr[:F], w.s[:F], 7) if F else None for w, s, F in zip(wls, specs, Fs)]
    for tun in (dict(fuse_codes=0), dict(fuse_codes=1), dict(fuse_codes=2)):
        dec = Q.Decoder(codes, Fs, tuning=tun)
        h, a, f = dec.decode(L, S, 7)
        torch.cuda.synchronize()
        h, a, f = h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()
        on = of = 0
        for r, s, F in zip(ref, specs, Fs):
            if not F:
                continue
            assert np.array_equal(a[on:on + F * s.n], r[1].reshape(-1)), tun
            assert np.array_equal(h[on:on + F * s.n], r[0].reshape(-1)), tun
            assert np.array_equal(f[of:of + F], r[2]), tun
            on += F * s.n
            of += F
    dec = Q.Decoder(codes, Fs, flags=Q.QM_EARLY_STOP)
    h, a, f, it = dec.decode_early(L, S, 7)
    torch.cuda.synchronize()
    assert h.numel() == sum(F * s.n for s, F in zip(specs, Fs)) and it.numel() == sum(Fs)
    it = it.cpu().numpy()
    assert ((it >= 0) & (it <= 7)).all()
    for flags in (0, Q.QM_EARLY_STOP):
        empty = Q.Decoder([codes[0]], [0], flags=flags)
        e = torch.empty(0, device="cuda")
        e8 = torch.empty(0, dtype=torch.uint8, device="cuda")
        if flags:
            out = empty.decode_early(e, e8, 5)
        else:
            out = empty.decode(e, e8, 5)
        torch.cuda.synchronize()
        assert all(x is None or x.numel() == 0 for x in out)


def test_code_streams_graph_replays_match_eager():
    # each code on its own stream (fuse_codes = 2) inside a captured graph,
    # replayed with eager work between the replays
    import torch
    specs = [SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)]
    Fs = [32, 16, 16]
    wls, codes, L, S = _mixed(specs, Fs)
    ref = Q.Decoder(codes, Fs, tuning=dict(fuse_codes=0))
    rh, ra, rf = (t.cpu().numpy() for t in ref.decode(L, S, 7))
    dec = Q.Decoder(codes, Fs, tuning=dict(fuse_codes=2, graph=1))
    for _ in range(3):
        h, a, f = dec.decode(L, S, 7)
        torch.cuda.synchronize()
        assert np.array_equal(h.cpu().numpy(), rh)
        assert np.array_equal(a.cpu().numpy().view(np.uint32), ra.view(np.uint32))
        assert np.array_equal(f.cpu().numpy(), rf)
        torch.ones(8, device="cuda").mul_(2.0)


@pytest.mark.parametrize("fp16", [False, True], ids=["fp32", "fp16"])
@pytest.mark.parametrize("fuse", [1, 2], ids=["fused", "streams"])
def test_fused_mixed_batch_matches_oracle_per_code(fuse, fp16):
    # each code's frames of a mixed batch against the oracle's decode of that
    # code alone, with fused launches and with a stream per code; binary16
    # messages against the oracle's binary16 mode
    import torch
    specs = [SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)]
    Fs = [5, 3, 4]
    wls, codes, L, S = _mixed(specs, Fs, snr_scale=3.0)
    dec = Q.Decoder(codes, Fs, flags=Q.QM_MSG_FP16 if fp16 else 0, tuning=dict(fuse_codes=fuse))
    for T in (1, 2):
        h, a, f = dec.decode(L, S, T)
        torch.cuda.synchronize()
        a, h, f = a.cpu().numpy(), h.cpu().numpy(), f.cpu().numpy()
        on = of = 0
        for w, s, F in zip(wls, specs, Fs):
            appo, hardo, flo, _ = oracle.decode_sp(w.shifts, s.Z, w.llr, w.s, T, fp16_messages=fp16)
            rows = compare(a[on:on + F * s.n].reshape(F, -1), h[on:on + F * s.n].reshape(F, -1), f[of:of + F],
                           appo, hardo, flo, extra=FP16_EXTRA if fp16 else 0.0)
            for r in rows:
                assert r["app_viol"] == 0 and r["bits_diff_confident"] == 0 and r["flag_o"] == r["flag_g"], (s.name, r)
            on += F * s.n
            of += F


def test_autotune_picks_a_result_preserving_tuning(tmp_path):
    import json
    import torch
    specs = [SMALL, W.RATE002.with_Z(16)]
    Fs = [32, 16]
    wls, codes, L, S = _mixed(specs, Fs)
    dec = Q.Decoder(codes, Fs)
    ref = [t.cpu().numpy() for t in dec.decode(L, S, 7)]
    log = str(tmp_path / "tune.jsonl")
    tun = dec.autotune(L, S, 7, cache_path=log)
    trials = [json.loads(l) for l in open(log)]
    assert len(trials) >= 12
    got = [t.cpu().numpy() for t in dec.decode(L, S, 7)]
    torch.cuda.synchronize()
    for x, y in zip(ref, got):
        assert np.array_equal(x, y), tun


def test_tile_groups_are_bit_identical():
    # frame tiles split into groups on their own streams: frames never
    # depend on other frames, so every output is unchanged
    import torch
    wl = _wl(SMALL, 64, snr=0.3, seed=9)
    ref = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, tuning=dict(frames_per_tile=8))
    for tun in (dict(frames_per_tile=8, tile_groups=2), dict(frames_per_tile=8, tile_groups=4),
                dict(frames_per_tile=8, tile_groups=8), dict(frames_per_tile=4, tile_groups=4, merge=0),
                dict(frames_per_tile=16, tile_groups=8)):
        got = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, tuning=tun)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), tun
    fp16 = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, flags=Q.QM_MSG_FP16, tuning=dict(frames_per_tile=8))
    got = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, flags=Q.QM_MSG_FP16,
                     tuning=dict(frames_per_tile=8, tile_groups=4))
    for x, y in zip(got, fp16):
        assert np.array_equal(x, y)
    # captured graph with forked group streams, replayed with eager work between
    code = Q.Code(wl.shifts, SMALL.Z)
    dec = Q.Decoder([code], [64], tuning=dict(frames_per_tile=8, tile_groups=4, graph=1))
    L, S = to_dev(wl.llr), to_dev(wl.s)
    for _ in range(3):
        h, a, f = dec.decode(L, S, 9)
        torch.cuda.synchronize()
        assert np.array_equal(h.cpu().numpy().reshape(64, -1), ref[0])
        assert np.array_equal(a.cpu().numpy().reshape(64, -1), ref[1])
        torch.ones(8, device="cuda").mul_(2.0)


def test_frame_batches_are_bit_identical():
    # frame tiles decoded in batches, one batch's sweeps after another's
    # (with and without tile groups inside a batch, and a last batch that is
    # smaller): every output is unchanged
    wl = _wl(SMALL, 56, snr=0.3, seed=10)
    ref = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, tuning=dict(frames_per_tile=8))
    for tun in (dict(frames_per_tile=8, frames_per_batch=16), dict(frames_per_tile=8, frames_per_batch=24),
                dict(frames_per_tile=8, frames_per_batch=8, merge=0),
                dict(frames_per_tile=8, frames_per_batch=32, tile_groups=2), dict(frames_per_tile=8, frames_per_batch=5)):
        got = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, tuning=tun)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), tun
    fp16 = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, flags=Q.QM_MSG_FP16, tuning=dict(frames_per_tile=8))
    got = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 9, flags=Q.QM_MSG_FP16,
                     tuning=dict(frames_per_tile=8, frames_per_batch=16))
    for x, y in zip(got, fp16):
        assert np.array_equal(x, y)


def test_frame_batches_graph_replays_match_eager():
    # batched sweeps inside a captured graph, replayed with eager work between
    # replays: every replay equals the unbatched eager decode
    import torch
    wl = _wl(SMALL, 40, snr=0.3, seed=12)
    ref = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 7, tuning=dict(frames_per_tile=8))
    code = Q.Code(wl.shifts, SMALL.Z)
    dec = Q.Decoder([code], [40], tuning=dict(frames_per_tile=8, frames_per_batch=16, graph=1))
    L, S = to_dev(wl.llr), to_dev(wl.s)
    out = dec.alloc_outputs()
    for rep in range(3):
        dec.decode(L, S, 7, out=out)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.array_equal(out[0].cpu().numpy().reshape(40, -1), ref[0]), rep
        assert np.array_equal(out[1].cpu().numpy().reshape(40, -1), ref[1]), rep
        assert np.array_equal(out[2].cpu().numpy(), ref[2]), rep
        out[1].fill_(7.0)
        out[0].fill_(3)


def test_tile_groups_fullsize():
    import torch
    spec = W.RATE01
    wl = W.build(spec, 128, frame_seed=0)
    code = Q.Code(wl.shifts, spec.Z)
    outs = []
    for g in (1, 2):
        dec = Q.Decoder([code], [128], tuning=dict(tile_groups=g))
        h, a, f = dec.decode(to_dev(wl.llr), to_dev(wl.s), 3)
        torch.cuda.synchronize()
        outs.append((h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()))
        del dec
        torch.cuda.empty_cache()
    for x, y in zip(*outs):
        assert np.array_equal(x, y)

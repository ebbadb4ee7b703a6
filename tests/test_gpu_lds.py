"""LDS-resident decoding (tuning lds_resident = 1): one workgroup per frame
keeps the frame's degree>=2 APPs in LDS through every sweep.  Its per-check
arithmetic is the layer kernels', so every output must be bit-identical to
the tiled path (which is itself checked against the FP64 oracle); codes that
do not fit fall back to the tiled path."""
import numpy as np
import pytest

from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.gpu_util import gpu_decode, say, to_dev

pytestmark = pytest.mark.gpu


def _both(spec, F, T, flags=0, snr=None, seed=1):
    wl = W.build(spec, F, snr=snr, frame_seed=seed)
    ref = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, T, flags=flags)
    got = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, T, flags=flags, tuning=dict(lds_resident=1))
    return ref, got


def _assert_same(ref, got, what):
    assert np.array_equal(ref[0], got[0]), what
    assert np.array_equal(ref[1].view(np.uint32), got[1].view(np.uint32)), what
    assert np.array_equal(ref[2], got[2]), what


@pytest.mark.parametrize("flags", [0, Q.QM_MSG_FP16, Q.QM_MSG_FP8])
@pytest.mark.parametrize("spec", [W.RATE002.with_Z(64), W.RATE01_SMALL, W.RATE005.with_Z(16)], ids=lambda s: s.name)
def test_lds_resident_equals_layer_kernels(spec, flags):
    for T in (1, 7):
        ref, got = _both(spec, 12, T, flags=flags, snr=spec.snr * 2)
        _assert_same(ref, got, (spec.name, flags, T))


def test_lds_resident_converging_frames():
    spec = W.RATE01_SMALL
    ref, got = _both(spec, 16, 30, snr=0.4, seed=3)
    assert ref[2].sum() >= 8
    _assert_same(ref, got, "converging")


def test_lds_resident_fullsize_rate002():
    # n = 10^6, 2 x 10^4 degree>=2 variables: 80 KB of LDS per frame
    import torch
    spec = W.RATE002
    F, T = 8, 4
    wl = W.build(spec, F, frame_seed=0)
    code = Q.Code(wl.shifts, spec.Z)
    outs = []
    for lds in (0, 1):
        dec = Q.Decoder([code], [F], tuning=dict(lds_resident=lds))
        dec.set_profiling(True)
        h, a, f = dec.decode(to_dev(wl.llr), to_dev(wl.s), T)
        torch.cuda.synchronize()
        p = dec.profile()
        say(f"lds_resident={lds}: profile", p)
        assert (p["lds_launches"] == 1) == (lds == 1)
        outs.append((h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()))
        del dec
    _assert_same(outs[0], outs[1], "full size")


def test_lds_resident_auto_takes_codes_with_a_frame_per_compute_unit():
    # lds_resident 2 (the default) runs the LDS-resident kernel only for a
    # code with at least as many frames as the device has compute units;
    # either way the outputs equal the layer kernels'
    import torch
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    spec = W.RATE002.with_Z(16)
    for F, want in ((ncu - 1, 0), (ncu + 3, 1)):
        wl = W.build(spec, F, snr=0.3, frame_seed=21)
        code = Q.Code(wl.shifts, spec.Z)
        outs = []
        for lds in (0, 2):
            dec = Q.Decoder([code], [F], tuning=dict(lds_resident=lds))
            dec.set_profiling(True)
            h, a, f = dec.decode(to_dev(wl.llr), to_dev(wl.s), 5)
            torch.cuda.synchronize()
            p = dec.profile()
            assert p["lds_launches"] == (want if lds == 2 else 0), (F, lds, p)
            outs.append((h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()))
        _assert_same(outs[0], outs[1], f"auto, {F} frames")
    # an early-terminating decoder keeps the layer kernels (and its frame
    # tiles) whatever lds_resident says
    dec = Q.Decoder([code], [F], flags=Q.QM_EARLY_STOP, tuning=dict(lds_resident=1))
    dec.set_profiling(True)
    dec.decode(to_dev(wl.llr), to_dev(wl.s), 5)
    dec.decode_early(to_dev(wl.llr), to_dev(wl.s), 5)
    torch.cuda.synchronize()
    assert dec.profile()["lds_launches"] == 0


def test_lds_resident_falls_back_when_too_big():
    # rate 0.1 at Z = 20000: 5 x 20000 x 4 B = 400 KB does not fit
    import torch
    spec = W.RATE01
    wl = W.build(spec, 2, frame_seed=0)
    code = Q.Code(wl.shifts, spec.Z)
    dec = Q.Decoder([code], [2], tuning=dict(lds_resident=1))
    dec.set_profiling(True)
    h, a, f = dec.decode(to_dev(wl.llr), to_dev(wl.s), 3)
    torch.cuda.synchronize()
    p = dec.profile()
    assert p["lds_launches"] == 0 and p["launches"] > 0
    ref = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, 3)
    assert np.array_equal(ref[1].reshape(-1).view(np.uint32), a.cpu().numpy().view(np.uint32))


def test_lds_resident_in_a_mixed_decoder():
    import torch
    specs = [W.RATE01, W.RATE002]          # the second fits in LDS, the first does not
    Fs = [2, 6]
    wls = [W.build(s, F, frame_seed=5) for s, F in zip(specs, Fs)]
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    L = to_dev(np.concatenate([w.llr.reshape(-1) for w in wls]))
    S = to_dev(np.concatenate([w.s.reshape(-1) for w in wls]))
    outs = []
    for lds in (0, 1):
        dec = Q.Decoder(codes, Fs, tuning=dict(lds_resident=lds))
        h, a, f = dec.decode(L, S, 3)
        torch.cuda.synchronize()
        outs.append((h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()))
        del dec
    _assert_same(outs[0], outs[1], "mixed")


def test_lds_resident_graph_replay():
    import torch
    spec = W.RATE002.with_Z(64)
    wl = W.build(spec, 8, frame_seed=2)
    code = Q.Code(wl.shifts, spec.Z)
    dec = Q.Decoder([code], [8], tuning=dict(lds_resident=1, graph=1))
    L, S = to_dev(wl.llr), to_dev(wl.s)
    eager = gpu_decode(wl.shifts, spec.Z, wl.llr, wl.s, 5)
    for _ in range(3):
        h, a, f = dec.decode(L, S, 5)
        torch.cuda.synchronize()
        _assert_same(eager, (h.cpu().numpy().reshape(8, -1), a.cpu().numpy().reshape(8, -1), f.cpu().numpy()),
                     "graph replay")


def test_lds_resident_mixed_graph_replay_forks_a_side_stream():
    # a tiled code and an LDS-resident code in one decoder run concurrently
    # (side stream forked and joined with events), also inside a captured
    # graph; every replay equals the eager decode with lds_resident = 0
    import torch
    specs = [W.RATE01, W.RATE002.with_Z(64)]   # the first cannot fit in LDS (400 KB per frame)
    Fs = [2, 8]
    wls = [W.build(s, F, frame_seed=8) for s, F in zip(specs, Fs)]
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    L = to_dev(np.concatenate([w.llr.reshape(-1) for w in wls]))
    S = to_dev(np.concatenate([w.s.reshape(-1) for w in wls]))
    ref_dec = Q.Decoder(codes, Fs, tuning=dict(lds_resident=0, frames_per_tile=16))
    h0, a0, f0 = ref_dec.decode(L, S, 6)
    torch.cuda.synchronize()
    ref = (h0.cpu().numpy(), a0.cpu().numpy(), f0.cpu().numpy())
    dec = Q.Decoder(codes, Fs, tuning=dict(lds_resident=1, frames_per_tile=16, graph=1))
    for _ in range(3):
        h, a, f = dec.decode(L, S, 6)
        torch.cuda.synchronize()
        _assert_same(ref, (h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()), "mixed graph")
        torch.zeros(1, device="cuda").add_(1.0)  # eager work between replays

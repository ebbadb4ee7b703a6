"""8-bit float message storage (QM_MSG_FP8) on the GPU against the FP64
oracle in its e4m3 message mode.

The GPU rounds a float32 message and the oracle an FP64 one; the FP8 step
is 1/16 to 1/8 relative, so a value within float32 rounding of a step
boundary lands on different sides now and then, and the difference
propagates through the rest of the sweep.  The allowances for the first
sweeps (mean and worst-frame fraction of APPs outside the float32 tolerance,
largest relative deviation) come from the oracle-only perturbation study in
tests/golden/make_precision_bounds.py, which also finds converged frames
unaffected; those are required to match exactly.  GPU-against-GPU
invariants (tunings, fused codes, early termination) are bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.gpu_util import compare, gpu_decode, precision_bound, say, to_dev

pytestmark = pytest.mark.gpu

SMALL = W.RATE01_SMALL
FP8 = Q.QM_MSG_FP8


def _wl(F, snr, seed):
    return W.build(SMALL, F, snr=snr, frame_seed=seed)


@pytest.mark.parametrize("T", [1, 2])
def test_fp8_first_sweeps_match_oracle_e4m3_mode(T):
    b = precision_bound(f"fp8_layered_T{T}")
    mean_bound, frame_bound, rel_bound = b["bound_mean_frac"], b["bound_max_frac"], b["bound_max_rel"]
    wl = _wl(16, 0.161, 7)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, T, flags=FP8)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, T, fp8_messages=True)
    rows = compare(app, hard, fl, appo, hardo, flo)
    frac = np.array([r["strict_viol"] / SMALL.n for r in rows])
    say(f"fp8 T={T}: outside tolerance per frame", np.round(frac, 4).tolist(),
        "max rel", max(r["max_rel"] for r in rows))
    assert all(r["flag_o"] == r["flag_g"] for r in rows)
    assert frac.mean() <= mean_bound and frac.max() <= frame_bound
    assert max(r["max_rel"] for r in rows) <= rel_bound


@pytest.mark.parametrize("snr", [0.4, 0.6])
def test_fp8_converging_frames_match_oracle(snr):
    wl = _wl(32, snr, 9)
    hard, app, fl = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 30, flags=FP8)
    appo, hardo, flo, _ = oracle.decode_sp(wl.shifts, SMALL.Z, wl.llr, wl.s, 30, fp8_messages=True)
    say(f"fp8 snr {snr}: converged gpu {int(fl.sum())} oracle {int(flo.sum())}")
    assert flo.sum() >= 20
    assert (fl != flo).sum() <= 1
    both = np.nonzero((fl == 1) & (flo == 1))[0]
    for f in both:
        assert np.array_equal(hard[f], hardo[f]), f


def test_fp8_tunings_are_bit_identical():
    wl = _wl(16, 0.3, 2)
    ref = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 10, flags=FP8)
    for tun in (dict(frames_per_tile=1, frames_per_lane=1), dict(frames_per_tile=4, block=64),
                dict(frames_per_tile=16, merge=0), dict(frames_per_tile=8, graph=1), dict(stream_hint=0)):
        got = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, 10, flags=FP8, tuning=tun)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), tun


def test_fp8_messages_are_e4m3_values():
    # two degree-2 checks on the same two variables (two layers): a degree-2
    # check passes the other edge's q through (Phi(Phi(x)) = x), so after one
    # sweep the APPs follow in closed form with every message on the e4m3
    # grid (torch's float8_e4m3fn conversion gives the grid values)
    import torch
    H = np.array([[0, 0], [0, 0]], dtype=np.int32)
    rng = np.random.default_rng(4)
    F = 16
    L = rng.normal(0, 3, (F, 2)).astype(np.float32)
    S = rng.integers(0, 2, (F, 2)).astype(np.uint8)
    hard, app, fl = gpu_decode(H, 1, L, S, 1, flags=FP8)
    e4 = lambda x: torch.from_numpy(np.asarray(x, np.float32)).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    s0 = np.where(S[:, 0] == 1, -1.0, 1.0).astype(np.float32)
    s1 = np.where(S[:, 1] == 1, -1.0, 1.0).astype(np.float32)
    a0 = L[:, 0] + e4(s0 * L[:, 1])          # layer 0
    a1 = L[:, 1] + e4(s0 * L[:, 0])
    b0 = a0 + e4(s1 * a1)                    # layer 1 (its old messages are 0)
    b1 = a1 + e4(s1 * a0)
    assert np.allclose(app[:, 0], b0, rtol=1e-5, atol=1e-5) and np.allclose(app[:, 1], b1, rtol=1e-5, atol=1e-5)


def test_fp8_early_termination_equals_fixed_decodes():
    import torch
    T = 30
    wl = _wl(48, 0.25, 13)
    code = Q.Code(wl.shifts, SMALL.Z)
    dec = Q.Decoder([code], [48], flags=FP8 | Q.QM_EARLY_STOP, tuning=dict(frames_per_tile=8))
    hard, app, fl, it = dec.decode_early(to_dev(wl.llr), to_dev(wl.s), T)
    torch.cuda.synchronize()
    hard, app, fl, it = (hard.cpu().numpy().reshape(48, -1), app.cpu().numpy().reshape(48, -1), fl.cpu().numpy(),
                         it.cpu().numpy())
    say("fp8 early iters", np.bincount(it).tolist())
    assert (it < T).sum() >= 10
    for t in sorted(set(it.tolist())):
        idx = np.nonzero(it == t)[0]
        h, a, f = gpu_decode(wl.shifts, SMALL.Z, wl.llr, wl.s, int(t), flags=FP8, tuning=dict(frames_per_tile=8))
        assert np.array_equal(h[idx], hard[idx]) and np.array_equal(a[idx].view(np.uint32), app[idx].view(np.uint32))
        assert np.array_equal(f[idx], fl[idx])


def test_fp8_fused_mixed_batch_equals_unfused():
    import torch
    specs = [SMALL, W.RATE005.with_Z(16), W.RATE002.with_Z(16)]
    Fs = [16, 8, 8]
    wls = [W.build(s, F, snr=s.snr, frame_seed=3) for s, F in zip(specs, Fs)]
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    L = to_dev(np.concatenate([w.llr.reshape(-1) for w in wls]))
    S = to_dev(np.concatenate([w.s.reshape(-1) for w in wls]))
    outs = []
    for fuse in (1, 0):
        dec = Q.Decoder(codes, Fs, flags=FP8, tuning=dict(fuse_codes=fuse))
        h, a, f = dec.decode(L, S, 7)
        torch.cuda.synchronize()
        outs.append((h.cpu().numpy(), a.cpu().numpy(), f.cpu().numpy()))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_fp8_flag_combinations_rejected():
    code = Q.Code(W.make_code(SMALL, 0), SMALL.Z)
    with pytest.raises(Q.QMError):
        Q.Decoder([code], [4], flags=FP8 | Q.QM_MSG_FP16)
    dec = Q.Decoder([code], [4], flags=FP8)
    with pytest.raises(Q.QMError):
        dec.nms_bind(5)

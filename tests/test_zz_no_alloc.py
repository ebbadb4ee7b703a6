"""The allocation-free decode (qm_decode_noalloc, for callers that cannot
allocate) through the C ABI against qm_decode with a bound workspace on the
same inputs: bit-identical hard decisions, APPs and flags, on calls in a row
whose second input is smaller, with and without a bound workspace; decoders
beyond the static scratch are rejected before any device work."""
import numpy as np
import pytest

from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _inputs(specs, Fs, snr_scale, seed):
    wls = [W.build(s, F, snr=s.snr * snr_scale, frame_seed=seed) for s, F in zip(specs, Fs)]
    L = to_dev(np.concatenate([w.llr.reshape(-1) for w in wls]))
    S = to_dev(np.concatenate([w.s.reshape(-1) for w in wls]))
    return wls, L, S


def _bound_decode(codes, Fs, L, S, T, flags=0, tuning=None):
    import torch
    dec = Q.Decoder(codes, Fs, flags=flags, tuning=tuning)
    h, a, f = dec.decode(L, S, T)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (h, a, f)]


def _noalloc(handle, n, F, L, S, T):
    import torch
    hard = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    app = torch.full((n,), 123.0, dtype=torch.float32, device="cuda")
    flags = torch.full((F,), 9, dtype=torch.uint8, device="cuda")
    Q.qm_decode_noalloc(handle, L, S, T, hard, app, flags)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (hard, app, flags)]


def _same(got, ref, what):
    assert np.array_equal(got[0], ref[0]), what
    assert np.array_equal(got[1].view(np.uint32), ref[1].view(np.uint32)), what
    assert np.array_equal(got[2], ref[2]), what


def test_noalloc_equals_bound_decode_on_calls_in_a_row():
    small = W.RATE01_SMALL
    specs1, Fs1, T1 = [small, W.RATE002.with_Z(16)], [40, 9], 12
    specs2, Fs2, T2 = [small.with_Z(37)], [5], 7
    wls1, L1, S1 = _inputs(specs1, Fs1, 2.5, 1)
    wls2, L2, S2 = _inputs(specs2, Fs2, 3.0, 2)
    codes1 = [Q.Code(w.shifts, s.Z) for w, s in zip(wls1, specs1)]
    codes2 = [Q.Code(w.shifts, s.Z) for w, s in zip(wls2, specs2)]
    n1, n2 = sum(F * s.n for s, F in zip(specs1, Fs1)), sum(F * s.n for s, F in zip(specs2, Fs2))
    ref1 = _bound_decode(codes1, Fs1, L1, S1, T1)
    ref2 = _bound_decode(codes2, Fs2, L2, S2, T2)
    assert ref1[2].sum() >= 1 and ref2[2].sum() >= 1   # some frames converge
    # a decoder that never had a workspace bound
    h1 = Q.qm_decoder_create([c.handle for c in codes1], Fs1, 0)
    try:
        assert Q.qm_decoder_workspace_bytes(h1) <= Q.QM_NOALLOC_SCRATCH_BYTES
        say("no-alloc call 1: 2 codes, 40 + 9 frames")
        _same(_noalloc(h1, n1, sum(Fs1), L1, S1, T1), ref1, "call 1")
        # second call, smaller input, a decoder with its own bound workspace
        dec2 = Q.Decoder(codes2, Fs2)
        say("no-alloc call 2: 1 code, 5 frames")
        _same(_noalloc(dec2.handle, n2, sum(Fs2), L2, S2, T2), ref2, "call 2")
        # the bound workspace still decodes as before
        import torch
        h, a, f = dec2.decode(L2, S2, T2)
        torch.cuda.synchronize()
        _same([x.cpu().numpy() for x in (h, a, f)], ref2, "bound decode after the no-alloc call")
        # the first decoder again: nothing of the second call leaks into it
        say("no-alloc call 3: the first decoder again")
        _same(_noalloc(h1, n1, sum(Fs1), L1, S1, T1), ref1, "call 3")
    finally:
        Q.qm_decoder_destroy(h1)


@pytest.mark.parametrize("flags,tuning", [(Q.QM_MSG_FP16, None), (0, dict(fuse_codes=2, graph=1)),
                                          (0, dict(tile_groups=2, frames_per_tile=8))])
def test_noalloc_other_modes_equal_bound_decode(flags, tuning):
    # message storage and tunings that the no-alloc call replaces by its
    # single-stream sequence (graph, code streams, tile groups) decode to the
    # same bits
    specs, Fs, T = [W.RATE01_SMALL, W.RATE005.with_Z(16)], [32, 6], 9
    wls, L, S = _inputs(specs, Fs, 2.5, 3)
    codes = [Q.Code(w.shifts, s.Z) for w, s in zip(wls, specs)]
    n = sum(F * s.n for s, F in zip(specs, Fs))
    ref = _bound_decode(codes, Fs, L, S, T, flags=flags, tuning=tuning)
    dec = Q.Decoder(codes, Fs, flags=flags, tuning=tuning)
    for rep in range(2):
        _same(_noalloc(dec.handle, n, sum(Fs), L, S, T), ref, (flags, tuning, rep))


def test_noalloc_rejects_what_it_cannot_run():
    import torch
    spec = W.RATE01
    code = Q.Code(W.make_code(spec, 0), spec.Z)
    h = Q.qm_decoder_create([code.handle], [8], 0)
    try:
        assert Q.qm_decoder_workspace_bytes(h) > Q.QM_NOALLOC_SCRATCH_BYTES
        n = 8 * spec.n
        L = torch.zeros(n, dtype=torch.float32, device="cuda")
        S = torch.zeros(8 * spec.m, dtype=torch.uint8, device="cuda")
        with pytest.raises(Q.QMError) as e:
            _noalloc(h, n, 8, L, S, 3)
        assert e.value.code == Q.QM_ERR_NO_WORKSPACE
    finally:
        Q.qm_decoder_destroy(h)
    small = W.RATE01_SMALL
    c2 = Q.Code(W.make_code(small, 0), small.Z)
    for flags in (Q.QM_EARLY_STOP, Q.QM_FLOODING):
        h = Q.qm_decoder_create([c2.handle], [2], flags)
        try:
            L = torch.zeros(2 * small.n, dtype=torch.float32, device="cuda")
            S = torch.zeros(2 * small.m, dtype=torch.uint8, device="cuda")
            with pytest.raises(Q.QMError) as e:
                _noalloc(h, 2 * small.n, 2, L, S, 3)
            assert e.value.code == Q.QM_ERR_UNSUPPORTED
        finally:
            Q.qm_decoder_destroy(h)

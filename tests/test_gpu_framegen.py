"""GPU training-frame generator against its definition (Philox4x32-10 +
Box-Muller in FP64 on the CPU) and s = H x from the seeded workload module."""
import numpy as np
import pytest

from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W
from tests.helpers import philox_frame

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("spec", [W.RATE01_SMALL, W.RATE01_SMALL.with_Z(37)], ids=lambda s: s.name)
def test_frames_match_definition(spec):
    import torch
    H = W.make_code(spec, 0)
    code = Q.Code(H, spec.Z)
    F, seed, first, snr = 5, 0x1234_5678_9ABC, 2**32 + 7, 0.161
    dec = Q.Decoder([code], [F])
    x = torch.empty(F * spec.n, dtype=torch.uint8, device="cuda")
    llr = torch.empty(F * spec.n, dtype=torch.float32, device="cuda")
    syn = torch.empty(F * spec.m, dtype=torch.uint8, device="cuda")
    Q.qm_generate_frames(dec.handle, 0, seed, first, snr, F, x, llr, syn)
    torch.cuda.synchronize()
    x, llr, syn = (t.cpu().numpy().reshape(F, -1) for t in (x, llr, syn))
    sigma = np.sqrt(1.0 / snr)
    for f in range(F):
        xr, nr = philox_frame(spec.n, seed, first + f, snr)
        assert np.array_equal(x[f], xr)
        ref = 2.0 * snr * ((1.0 - 2.0 * xr) + sigma * nr)
        assert np.max(np.abs(llr[f] - ref)) < 1e-3
        assert np.array_equal(syn[f], W.syndrome(H, spec.Z, x[f]))


def test_frames_depend_only_on_their_index():
    import torch
    spec = W.RATE01_SMALL
    code = Q.Code(W.make_code(spec, 0), spec.Z)
    dec = Q.Decoder([code], [8])
    bufs = []
    for first, F in ((10, 8), (13, 2)):
        x = torch.empty(F * spec.n, dtype=torch.uint8, device="cuda")
        llr = torch.empty(F * spec.n, dtype=torch.float32, device="cuda")
        syn = torch.empty(F * spec.m, dtype=torch.uint8, device="cuda")
        Q.qm_generate_frames(dec.handle, 0, 99, first, 0.3, F, x, llr, syn)
        bufs.append(llr.cpu().numpy().reshape(F, -1))
    torch.cuda.synchronize()
    assert np.array_equal(bufs[0][3:5], bufs[1])

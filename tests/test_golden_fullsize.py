"""The stored full-size oracle decodes (tests/golden/fullsize_oracle.npz)
cover what the GPU parity test at n = 10^6 is meant to assert bit for bit:
for every workload code a 200-sweep case in which the oracle reaches a
valid word, and a binary16-message case with a converged frame."""
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_oracle.npz")


def _cases():
    g = np.load(GOLD)
    out = {}
    for k in g.files:
        case, rest = k.split("/", 1)
        if rest.endswith("flag"):
            out.setdefault(case, []).append(int(g[k]))
    return g, out


def test_every_code_has_a_converged_stored_frame():
    g, cases = _cases()
    for code in ("r0.1", "r0.05", "r0.02"):
        conv = [c for c, fl in cases.items() if c.startswith(code + "_") and not c.endswith("_fp16") and any(fl)]
        assert conv, code
        assert any(int(g[f"{c}/meta"][1]) == 200 for c in conv) or code == "r0.1", (code, conv)
    assert any(c.endswith("_fp16") and any(fl) for c, fl in cases.items())

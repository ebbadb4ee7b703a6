"""The stored oracle convergence record (tests/golden/convergence_oracle.json,
written by tests/golden/make_convergence_golden.py) is complete and
self-consistent: every mode at both SNRs for all 128 frames, rates that
match the per-frame records, a decoded transmitted word only where the
syndrome is satisfied, and the waterfall falling with SNR."""
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "convergence_oracle.json")
MODES = ("fp64", "fp16", "fp64_pert", "fp16_pert")


def _gold():
    with open(GOLD) as fh:
        return json.load(fh)


def test_record_is_complete_and_consistent():
    g = _gold()
    assert g["frames"] == 128 and g["sweeps"] == 200 and g["graph_seed"] == 0 and g["frame_seed"] == 0
    assert set(g["snr"]) == {"0.5", "0.6"}
    for snr, rec in g["snr"].items():
        assert set(rec) == set(MODES), snr
        for mode, r in rec.items():
            flag, correct = np.array(r["flag"]), np.array(r["correct"])
            assert flag.shape == (128,) and correct.shape == (128,)
            assert set(np.unique(flag)) <= {0, 1} and set(np.unique(correct)) <= {0, 1}
            assert abs(r["syndrome_fail"] - (1.0 - flag.mean())) < 1e-12, (snr, mode)
            assert abs(r["fer"] - (1.0 - correct.mean())) < 1e-12, (snr, mode)
            # the transmitted word satisfies its own syndrome
            assert np.all(flag[correct == 1] == 1), (snr, mode)
    for mode in MODES:
        assert g["snr"]["0.6"][mode]["syndrome_fail"] <= g["snr"]["0.5"][mode]["syndrome_fail"], mode


def test_perturbation_allowances_are_small():
    # the GPU test allows twice the perturbed oracle's discordance plus two
    # frames; a record in which a 2e-6 perturbation moved many frames would
    # make that allowance meaningless
    g = _gold()
    for snr, rec in g["snr"].items():
        for ref, pert in (("fp64", "fp64_pert"), ("fp16", "fp16_pert")):
            d = int((np.array(rec[ref]["flag"]) != np.array(rec[pert]["flag"])).sum())
            assert d <= 4, (snr, ref, d)

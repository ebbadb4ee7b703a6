"""The stored allowances of the reduced-precision message modes
(tests/golden/precision_bounds.json) follow from their committed study:
a fresh, smaller run of the same oracle-only study stays inside them, and
each stored bound is twice the figure the study measured."""
import json
import os

import pytest

from tests.golden import make_precision_bounds as M

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision_bounds.json")


def test_stored_bounds_are_twice_the_measured_figures():
    data = json.load(open(GOLD))
    assert data["eps"] == M.EPS and data["tol"] == M.TOL
    names = {f"{c[0]}_T{T}" for c in M.CASES for T in c[5]}
    assert set(data["cases"]) == names
    for key, c in data["cases"].items():
        m = c["measured"]
        assert c["bound_mean_frac"] == M.up(m["mean_frac"]), key
        assert c["bound_max_frac"] == M.up(m["max_frac"]), key
        assert c["bound_max_rel"] == M.up(m["max_rel"]), key
        assert m["flag_diff"] == 0, key


@pytest.mark.parametrize("case", M.CASES, ids=[c[0] for c in M.CASES])
def test_a_fresh_study_stays_inside_the_bounds(case):
    data = json.load(open(GOLD))["cases"]
    name, kind, mode, snr, F, Ts, batch = case
    for T in Ts:
        r = M.study(kind, mode, snr, batch, T, batch, trials=2, seed=7)
        b = data[f"{name}_T{T}"]
        assert r["mean_frac"] <= b["bound_mean_frac"], (name, T, r, b)
        assert r["max_frac"] <= b["bound_max_frac"], (name, T, r, b)
        assert r["max_rel"] <= b["bound_max_rel"], (name, T, r, b)
        assert r["flag_diff"] == 0, (name, T, r)

"""The oracle's pins must catch plausible mistakes: each mutant below plants
one (a dropped syndrome flip, a self-inclusive sum, a reversed shift, ...) in
a copy of the oracle source, built on the CPU, and at least one pin test has
to fail against it."""
import os

import pytest

import oracle
from tests import test_oracle_pins as P

MUTANTS = {
    "no_syndrome_flip": ("int neg = s[chk] & 1;\n                        for (int b = 0; b < d; b++) {",
                         "int neg = 0;\n                        for (int b = 0; b < d; b++) {"),
    "sum_includes_self": ("if (b == a) continue;\n                            S += ph[b];",
                          "S += ph[b];"),
    "q_adds_old_message": ("q[a] = app[c->chk_vn[e0 + a]] - r[e0 + a];\n                        ph[a]",
                           "q[a] = app[c->chk_vn[e0 + a]] + r[e0 + a];\n                        ph[a]"),
    "shift_left": ("c->chk_vn[e] = j * Z + (k + a) % Z;", "c->chk_vn[e] = j * Z + (k + Z - a) % Z;"),
    "app_drops_q": ("app[c->chk_vn[e0 + a]] = q[a] + rn[a];\n                    }\n                }\n            }\n        }\n    }\n    x->flags",
                    "app[c->chk_vn[e0 + a]] = rn[a];\n                    }\n                }\n            }\n        }\n    }\n    x->flags"),
    "phi_factor": ("return log1p(2.0 / expm1(x));", "return log1p(1.0 / expm1(x));"),
    "half_one_bit_short": ("int qe = e - 11;", "int qe = e - 10;"),
    "greedy_skips_rows": ("for (int cand = first + 1; cand < mb; cand++) {", "for (int cand = first + 2; cand < mb; cand++) {"),
    "minsum_includes_self": ("if (b == a) continue;\n        double v = fabs(q[b]);", "double v = fabs(q[b]);"),
    "backward_rold_sign": ("gR[e0 + a] = -gq[a];", "gR[e0 + a] = gq[a];"),
    "backward_beta_sign": ("gb[w] -= gz;", "gb[w] += gz;"),
    "backward_argmin_sign": ("gq[arg] += gz * dabs(q[arg]);", "gq[arg] += gz;"),
    "minsum_unsaturated": ("if (mu > QO_X_HI) {\n        mu = QO_X_HI;", "if (mu > 1e300) {\n        mu = QO_X_HI;"),
    "gradient_through_saturation": ("mu = QO_X_HI;\n        best = -1;", "mu = QO_X_HI;"),
    "early_stop_counts_late": ("used = t + 1;\n        for (int g = 0; g < x->G; g++) {", "used = t + 2;\n        for (int g = 0; g < x->G; g++) {"),
    "early_stop_one_sweep_late": ("if (x->early_stop && hard_and_check(c, app, s, hard)) break;", "if (x->early_stop && t > 0 && hard_and_check(c, app, s, hard)) break;"),
    "e4m3_one_bit_short": ("int qe = e - 4;", "int qe = e - 3;"),
    "e4m3_no_subnormals": ("if (qe < -9) qe = -9;", "if (qe < -6) qe = -6;"),
    "flood_fresh_app": ("for (size_t e = 0; e < (size_t)c->E; e++) r[e] = rn[e];\n        for (int v = 0; v < n; v++) app[v] = (double)llr[v];",
                        "for (size_t e = 0; e < (size_t)c->E; e++) r[e] = rn[e];\n        for (int v = 0; v < n; v++) app[v] = 0.0;"),
    "flood_drops_old_message": ("q[a] = app[c->chk_vn[e0 + a]] - r[e0 + a];\n                ph[a] = qo_phi(qo_clip(fabs(q[a])));\n            }\n            for (int a = 0; a < d; a++) {\n                double S = 0.0;\n                int neg = s[chk] & 1;",
                                "q[a] = app[c->chk_vn[e0 + a]];\n                ph[a] = qo_phi(qo_clip(fabs(q[a])));\n            }\n            for (int a = 0; a < d; a++) {\n                double S = 0.0;\n                int neg = s[chk] & 1;"),
    "loss_normalised_by_frames_only": ("double norm = 1.0 / ((double)F * (double)c.n);", "double norm = 1.0 / (double)F;"),
    "loss_and_gradient_sign": ("sum += softplus(-sg * app[v]);\n        gA[v] = -sg * sigmoid(-sg * app[v]);",
                               "sum -= softplus(-sg * app[v]);\n        gA[v] = sg * sigmoid(-sg * app[v]);"),
    "window_one_sweep_long": ("int lo = t - x->window + 1;", "int lo = t - x->window;"),
    "sweep_terms_unweighted": ("x->every_sweep ? 1.0 / (double)T : 1.0", "1.0"),
    "sweep_terms_skip_first": ("if (x->want_grad && (x->every_sweep || t == T - 1)) {", "if (x->want_grad && ((x->every_sweep && t > 0) || t == T - 1)) {"),
    "loss_sign": ("gA[v] = -sg * sigmoid(-sg * app[v]);", "gA[v] = sg * sigmoid(-sg * app[v]);"),
}

PINS = [getattr(P, n) for n in dir(P) if n.startswith("test_")]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = oracle.build_variant(src.replace(old, new), str(tmp_path / f"libmut_{name}.so"))
    caught = []
    oracle.use_library(path)
    try:
        for fn in PINS:
            try:
                fn()
            except Exception:
                caught.append(fn.__name__)
    finally:
        oracle.use_library(None)
    assert caught, f"no pin caught mutant {name}"

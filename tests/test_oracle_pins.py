"""Pins of the FP64 oracle against facts that do not come from the oracle:
the paper's merge examples and table arithmetic, closed forms, brute-force
MAP/ML decoding, textbook special cases and exact invariants."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import workload as W
from tests.helpers import dense_H, map_llr, ml_word, random_tree_base, lift, frame_for

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Phi --

def test_phi_matches_definition():
    # Methods, step 2: Phi(x) = -ln(tanh(x/2)); compare with numpy's tanh/log
    # where that direct form is well conditioned.
    for x in np.linspace(0.05, 12.0, 200):
        ref = -math.log(math.tanh(x / 2.0))
        assert abs(oracle.phi(x) - ref) <= 1e-13 * max(1.0, abs(ref))


def test_phi_self_inverse_on_clip_interval():
    lo, hi = oracle.x_lo(), oracle.x_hi()
    assert hi == 30.0
    assert abs(oracle.phi(hi) - lo) == 0.0
    for x in np.geomspace(lo, hi, 400):
        assert abs(oracle.phi(oracle.phi(x)) - x) <= 1e-12 * x


def test_phi_asymptotics():
    # Phi(x) ~ 2 e^-x for large x and ~ ln(2/x) for small x
    for x in (20.0, 25.0, 30.0):
        assert abs(oracle.phi(x) / (2 * math.exp(-x)) - 1) < 1e-8
    for x in (1e-8, 1e-10, 1e-12):
        assert abs(oracle.phi(x) - math.log(2 / x)) < 1e-6


def test_clip():
    assert oracle.clip(0.0) == oracle.x_lo()
    assert oracle.clip(1e9) == 30.0
    assert oracle.clip(3.5) == 3.5


def test_round_half_matches_numpy_float16():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.normal(0, 10, 3000), rng.normal(0, 1e-5, 1000),
                        (rng.integers(0, 2048, 500) + 0.5) * 2.0 ** -10,   # exact ties
                        (rng.integers(0, 1024, 200) + 0.5) * 2.0 ** -24,   # subnormal ties
                        [0.0, -0.0, 65504.0, 30.0, -30.0, 1.8715e-13]])
    ref = v.astype(np.float16).astype(np.float64)
    got = np.array([oracle.round_half(a) for a in v])
    assert np.array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_round_e4m3_matches_torch_float8():
    # torch's float8_e4m3fn conversion (round to nearest even) is an
    # implementation independent of the oracle's
    import torch
    rng = np.random.default_rng(7)
    grid = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    g = np.unique(np.abs(grid[np.isfinite(grid)]))
    mids = (g[1:] + g[:-1]) / 2                      # exact ties
    v = np.concatenate([g, -g, mids, -mids, rng.normal(0, 8, 3000), rng.uniform(-30, 30, 3000),
                        rng.normal(0, 1e-2, 1000), np.geomspace(1e-5, 440, 500), [0.0, -0.0, 30.0, 448.0]])
    v = v.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([oracle.round_e4m3(a) for a in v])
    assert np.array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))
    assert oracle.round_e4m3(1000.0) == 448.0


# ------------------------------------------------------------ schedule --

def test_greedy_merge_reproduces_paper_examples():
    data = json.load(open(os.path.join(GOLD, "merge_examples.json")))
    for ex in data["examples"]:
        H = np.array(ex["H"], dtype=np.int32)
        gptr, rows = oracle.greedy_schedule(H)
        groups = [list(rows[gptr[g]:gptr[g + 1]]) for g in range(len(gptr) - 1)]
        assert groups == ex["groups"], ex["eq"]


def test_schedule_validator_rejects_conflicts():
    H = np.array([[1, 0, -1], [2, 1, 1], [0, 2, 0]], dtype=np.int32)
    assert oracle.check_schedule(H, [0, 2, 3], [0, 1, 2]) != 0      # rows 0,1 share col 0
    assert oracle.check_schedule(H, [0, 1, 2, 3], [0, 1, 2]) == 0
    assert oracle.check_schedule(H, [0, 1, 2, 3], [0, 0, 2]) != 0   # not a permutation


def test_greedy_groups_are_column_disjoint_on_workloads():
    for spec in (W.RATE01_SMALL, W.RATE005.with_Z(8), W.RATE002.with_Z(8)):
        H = W.make_code(spec, 0)
        gptr, rows = oracle.greedy_schedule(H)
        assert oracle.check_schedule(H, gptr, rows) == 0
        assert sorted(rows.tolist()) == list(range(spec.mb))


# ----------------------------------------------- closed forms & special cases --

def test_single_check_tanh_rule():
    # One check of degree d, Z = 1: after one layer r_j = (-1)^s 2 atanh(prod_{j'!=j} tanh(l_j'/2))
    rng = np.random.default_rng(1)
    for d in (2, 3, 4, 6):
        for s in (0, 1):
            H = np.zeros((1, d), dtype=np.int32)
            llr = rng.normal(0, 2.0, d).astype(np.float32)
            app, _, _, _ = oracle.decode_sp(H, 1, llr[None], np.array([[s]], np.uint8), 1)
            l64 = llr.astype(np.float64)
            for j in range(d):
                prod = np.prod(np.tanh(np.delete(l64, j) / 2.0))
                r = (-1) ** s * 2.0 * np.arctanh(prod)
                assert abs(app[0, j] - (l64[j] + r)) <= 1e-12 * max(1.0, abs(r))


def test_single_check_fp16_messages_round_to_binary16():
    rng = np.random.default_rng(2)
    d = 4
    H = np.zeros((1, d), dtype=np.int32)
    llr = rng.normal(0, 2.0, d).astype(np.float32)
    app, _, _, _ = oracle.decode_sp(H, 1, llr[None], np.zeros((1, 1), np.uint8), 1, fp16_messages=True)
    l64 = llr.astype(np.float64)
    for j in range(d):
        r = 2.0 * np.arctanh(np.prod(np.tanh(np.delete(l64, j) / 2.0)))
        r16 = float(np.float64(r).astype(np.float16))
        assert abs(app[0, j] - (l64[j] + r16)) <= 1e-12


def test_single_check_fp8_messages_round_to_e4m3():
    import torch
    rng = np.random.default_rng(3)
    d = 5
    H = np.zeros((1, d), dtype=np.int32)
    llr = rng.normal(0, 2.0, d).astype(np.float32)
    app, _, _, _ = oracle.decode_sp(H, 1, llr[None], np.ones((1, 1), np.uint8), 1, fp8_messages=True)
    l64 = llr.astype(np.float64)
    for j in range(d):
        r = -2.0 * np.arctanh(np.prod(np.tanh(np.delete(l64, j) / 2.0)))
        r8 = float(torch.tensor([r], dtype=torch.float64).to(torch.float8_e4m3fn).to(torch.float64)[0])
        assert abs(app[0, j] - (l64[j] + r8)) <= 1e-12


def _cycle_code(nb, Z, rng):
    # every row has exactly two entries -> all checks have degree 2
    H = np.full((nb, nb), -1, dtype=np.int32)
    for i in range(nb):
        H[i, i] = rng.integers(0, Z)
        H[i, (i + 1) % nb] = rng.integers(0, Z)
    return H


def test_degree2_checks_pass_the_other_message_through():
    # Phi(Phi(x)) = x: a degree-2 check sends r = (-1)^s q' (clip range aside)
    H = np.array([[0, 0]], dtype=np.int32)
    llr = np.array([[1.25, -3.5]], dtype=np.float32)
    for s in (0, 1):
        app, _, _, _ = oracle.decode_sp(H, 1, llr, np.array([[s]], np.uint8), 1)
        sg = -1.0 if s else 1.0
        assert abs(app[0, 0] - (1.25 + sg * -3.5)) < 1e-12
        assert abs(app[0, 1] - (-3.5 + sg * 1.25)) < 1e-12


def test_sp_equals_minsum_on_degree2_codes():
    # On all-degree-2 codes sum-product, min-sum and NMS(alpha=1, beta=0) coincide
    rng = np.random.default_rng(3)
    Z, nb, T = 16, 6, 4
    H = _cycle_code(nb, Z, rng)
    Hd = dense_H(H, Z)
    x = rng.integers(0, 2, nb * Z).astype(np.uint8)
    llr, s = frame_for(Hd, x, 2.0, rng)
    llr = np.clip(llr, -3, 3)  # keep every message below the clip level 30
    app_sp, _, _, _ = oracle.decode_sp(H, Z, llr[None], s[None], T)
    app_ms, _, _, _ = oracle.nms_decode(H, Z, llr[None], s[None], T, 1.0, 0.0)
    assert np.max(np.abs(app_sp - app_ms)) < 1e-11


# ------------------------------------------------------ brute force --

def test_tree_lift_gives_exact_map():
    # A cycle-free base graph lifts to a forest, where BP is exact (bitwise MAP)
    rng = np.random.default_rng(4)
    ran = 0
    for trial in range(6):
        base = random_tree_base(rng, n_rows=int(rng.integers(2, 5)), max_new=2)
        Z = 2
        H = lift(base, Z, rng)
        if H.shape[1] * Z > 16:
            continue
        Hd = dense_H(H, Z)
        x = rng.integers(0, 2, Hd.shape[1]).astype(np.uint8)
        llr, s = frame_for(Hd, x, 0.5, rng)
        ref = map_llr(Hd, s, llr)
        app, _, _, _ = oracle.decode_sp(H, Z, llr[None], s[None], 12)
        assert np.max(np.abs(app[0] - ref)) < 1e-9, trial
        ran += 1
    assert ran >= 3, ran


def test_tiny_loopy_codes_high_snr_match_ml_and_truth():
    rng = np.random.default_rng(6)
    hits = 0
    for trial in range(8):
        mb, nb, Z = 3, 5, 3
        base = np.where(rng.random((mb, nb)) < 0.7, 0, -1)
        base[:, 0] = 0
        H = lift(base, Z, rng)
        Hd = dense_H(H, Z)
        x = rng.integers(0, 2, nb * Z).astype(np.uint8)
        llr, s = frame_for(Hd, x, 12.0, rng)
        ml = ml_word(Hd, s, llr)
        _, hard, flags, _ = oracle.decode_sp(H, Z, llr[None], s[None], 20)
        assert np.array_equal(ml, x)
        assert np.array_equal(hard[0], ml)
        assert flags[0] == 1
        hits += 1
    assert hits == 8


def test_zero_noise_and_high_snr_decode_to_truth():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 3, seed=9, zero_noise=True)
    _, hard, flags, _ = oracle.decode_sp(H, Z, L, S, 5)
    assert flags.all() and np.array_equal(hard, X)
    X, L, S = W.make_frames(H, Z, 10.0, 3, seed=9)
    _, hard, flags, _ = oracle.decode_sp(H, Z, L, S, 20)
    assert flags.all() and np.array_equal(hard, X)


def test_flagged_frames_satisfy_syndrome():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.6, 8, seed=3)
    _, hard, flags, _ = oracle.decode_sp(H, Z, L, S, 30)
    for f in range(8):
        ok = np.array_equal(W.syndrome(H, Z, hard[f]), S[f])
        assert bool(flags[f]) == ok


def test_zero_iterations_returns_channel_decisions():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 2, seed=1)
    app, hard, _, _ = oracle.decode_sp(H, Z, L, S, 0)
    assert np.array_equal(app, L.astype(np.float64))
    assert np.array_equal(hard, (L < 0).astype(np.uint8))


# ------------------------------------------------------- invariants --

def test_coset_symmetry_is_exact():
    # decode(l * (1-2c), s ^ Hc) = decode(l, s) ^ c with APP sign-flipped, bit-exact
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.3, 2, seed=4)
    rng = np.random.default_rng(7)
    c = rng.integers(0, 2, L.shape).astype(np.uint8)
    L2 = np.where(c == 1, -L, L).astype(np.float32)
    S2 = S ^ W.syndrome(H, Z, c)
    app1, hard1, fl1, _ = oracle.decode_sp(H, Z, L, S, 7)
    app2, hard2, fl2, _ = oracle.decode_sp(H, Z, L2, S2, 7)
    assert np.array_equal(np.where(c == 1, -app1, app1), app2)
    assert np.array_equal(fl1, fl2)


def test_merged_equals_serial_in_the_same_row_order():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 2, seed=5)
    gptr, rows = oracle.greedy_schedule(H)
    app_m, _, _, _ = oracle.decode_sp(H, Z, L, S, 6, schedule=(gptr, rows))
    app_s, _, _, _ = oracle.decode_sp(H, Z, L, S, 6, schedule=oracle.serial_schedule(H.shape[0], rows))
    assert np.array_equal(app_m, app_s)
    # and the row order matters in general (a different permutation differs)
    app_n, _, _, _ = oracle.decode_sp(H, Z, L, S, 6, schedule=oracle.serial_schedule(H.shape[0]))
    assert not np.array_equal(app_m, app_n)


def test_frames_are_independent():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 5, seed=6)
    app_all, hard_all, fl_all, _ = oracle.decode_sp(H, Z, L, S, 4, threads=3)
    app_one, hard_one, fl_one, _ = oracle.decode_sp(H, Z, L[3:4], S[3:4], 4, threads=1)
    assert np.array_equal(app_all[3], app_one[0])


# ------------------------------------------------------- min-sum NMS --

def test_nms_beta0_is_scale_invariant():
    # with beta = 0 and no minimum reaching the saturation level, the min-sum
    # update is positively homogeneous: halving the LLRs halves every APP
    # exactly (|LLR| <= 0.4 keeps every |q| of one sweep below 0.4 * 30)
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.3, 2, seed=8)
    L = np.clip(L, -0.4, 0.4).astype(np.float32)
    T = 1
    rng = np.random.default_rng(9)
    alpha = rng.uniform(0.5, 1.0, (T, H.shape[0], 2))
    a1, _, _, _ = oracle.nms_decode(H, Z, (L / 2).astype(np.float32), S, T, alpha, 0.0)
    a2, _, _, _ = oracle.nms_decode(H, Z, L, S, T, alpha, 0.0)
    assert np.abs(a2).max() < 30
    assert np.array_equal(2 * a1, a2)


def test_nms_minimum_saturates_at_30():
    # a single check of degree 3 with very reliable inputs: each message is
    # alpha * (min(others, 30) - beta) with the check's sign rule
    H = np.zeros((1, 3), dtype=np.int32)
    llr = np.array([[100.0, -200.0, 12.0]], dtype=np.float32)
    alpha, beta = 0.75, 0.5
    app, _, _, _ = oracle.nms_decode(H, 1, llr, np.array([[0]], np.uint8), 1, alpha, beta)
    # r0 from {-200, 12}: sign -, min 12; r1 from {100, 12}: sign +, min 12;
    # r2 from {100, -200}: sign -, min 100 -> saturated at 30
    expect = [100 - alpha * (12 - beta), -200 + alpha * (12 - beta), 12 - alpha * (30 - beta)]
    assert np.allclose(app[0], expect, rtol=0, atol=1e-12)


def test_nms_early_stop_counts_iterations():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 2, seed=2, zero_noise=True)
    _, hard, flags, iters = oracle.nms_decode(H, Z, L, S, 10, 1.0, 0.0, early_stop=True)
    assert flags.all() and (iters == 0).all()
    X, L, S = W.make_frames(H, Z, 3.0, 3, seed=2)
    _, hard, flags, iters = oracle.nms_decode(H, Z, L, S, 30, 0.8, 0.0, early_stop=True)
    assert flags.all() and np.array_equal(hard, X)
    assert (iters >= 1).all() and (iters < 30).all()


def test_sp_early_stop_is_the_first_valid_sweep_count():
    # Results, Table tabearly: a frame stops once its hard decisions satisfy
    # the syndrome.  Each frame's output must equal a fixed-T decode with
    # T = its iteration count, and the syndrome (checked here with a dense H,
    # not the oracle's own test) must fail at every smaller count.
    spec = W.RATE01_SMALL
    H = W.make_code(spec, 0)
    Z = spec.Z
    Hd = dense_H(H, Z)
    X, L, S = W.make_frames(H, Z, 0.9, 6, seed=21)
    Tmax = 25
    app, hard, flags, iters = oracle.decode_sp_early(H, Z, L, S, Tmax)
    assert iters.min() >= 1 and (flags == 1).sum() >= 3
    for f in range(len(L)):
        t_f = int(iters[f])
        a_t, h_t, fl_t, _ = oracle.decode_sp(H, Z, L[f:f + 1], S[f:f + 1], t_f)
        assert np.array_equal(a_t[0], app[f]) and np.array_equal(h_t[0], hard[f]) and fl_t[0] == flags[f]
        ok = lambda h: not np.any((Hd.dot(h.astype(np.int64)) + S[f]) % 2)
        assert flags[f] == ok(hard[f])
        if t_f < Tmax:
            assert flags[f] == 1
        for t in range(t_f):
            _, h_s, _, _ = oracle.decode_sp(H, Z, L[f:f + 1], S[f:f + 1], t)
            assert not ok(h_s[0]), (f, t)


def test_sp_early_stop_zero_noise_stops_at_zero():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 2, seed=2, zero_noise=True)
    _, hard, flags, iters = oracle.decode_sp_early(H, Z, L, S, 10)
    assert np.all(iters == 0) and np.all(flags == 1) and np.array_equal(hard, X)


def test_flood_single_check_is_the_tanh_rule():
    rng = np.random.default_rng(31)
    d = 4
    H = np.zeros((1, d), dtype=np.int32)
    llr = rng.normal(0, 2.0, d).astype(np.float32)
    app, _, _, _ = oracle.decode_flood(H, 1, llr[None], np.array([[1]], np.uint8), 1)
    l64 = llr.astype(np.float64)
    for j in range(d):
        r = -2.0 * np.arctanh(np.prod(np.tanh(np.delete(l64, j) / 2.0)))
        assert abs(app[0, j] - (l64[j] + r)) <= 1e-12 * max(1.0, abs(r))


def test_flood_tree_lift_gives_exact_map():
    rng = np.random.default_rng(32)
    done = 0
    for trial in range(8):
        base = random_tree_base(rng, n_rows=int(rng.integers(2, 5)), max_new=2)
        Z = 2
        H = lift(base, Z, rng)
        if H.shape[1] * Z > 16:
            continue
        Hd = dense_H(H, Z)
        x = rng.integers(0, 2, Hd.shape[1]).astype(np.uint8)
        llr, s = frame_for(Hd, x, 0.5, rng)
        ref = map_llr(Hd, s, llr)
        app, _, _, _ = oracle.decode_flood(H, Z, llr[None], s[None], 12)
        assert np.max(np.abs(app[0] - ref)) < 1e-9, trial
        done += 1
    assert done >= 3


def test_flood_does_not_depend_on_row_order():
    # every check of an iteration reads the same APPs, so permuting the base
    # rows changes only the order of the final additions (layered decoding,
    # by contrast, depends on the row order)
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 2, seed=33)
    perm = np.random.default_rng(34).permutation(H.shape[0])
    Hp = H[perm]
    Sp = S.reshape(2, H.shape[0], Z)[:, perm].reshape(2, -1)
    a1, h1, f1, _ = oracle.decode_flood(H, Z, L, S, 6)
    a2, h2, f2, _ = oracle.decode_flood(Hp, Z, L, Sp, 6)
    assert np.max(np.abs(a1 - a2) / np.maximum(np.abs(a1), 1.0)) < 1e-12
    assert np.array_equal(h1, h2) and np.array_equal(f1, f2)
    l1, _, _, _ = oracle.decode_sp(H, Z, L, S, 6)
    l2, _, _, _ = oracle.decode_sp(Hp, Z, L, Sp, 6)
    assert np.max(np.abs(l1 - l2)) > 1.0


def test_flood_equals_layered_when_rows_share_no_variable():
    # each variable in a single check: one flooding iteration and one
    # layered sweep perform the same updates
    rng = np.random.default_rng(35)
    Z = 8
    H = np.full((3, 7), -1, dtype=np.int32)
    H[0, 0:3] = rng.integers(0, Z, 3)
    H[1, 3:5] = rng.integers(0, Z, 2)
    H[2, 5:7] = rng.integers(0, Z, 2)
    Hd = dense_H(H, Z)
    x = rng.integers(0, 2, 7 * Z).astype(np.uint8)
    llr, s = frame_for(Hd, x, 1.0, rng)
    for T in (1, 3):
        af, hf, ff, _ = oracle.decode_flood(H, Z, llr[None], s[None], T)
        al, hl, fl, _ = oracle.decode_sp(H, Z, llr[None], s[None], T)
        assert np.max(np.abs(af - al)) < 1e-12 and np.array_equal(hf, hl)


def test_flood_zero_noise_decodes_to_truth():
    H = W.make_code(W.RATE01_SMALL, 0)
    Z = W.RATE01_SMALL.Z
    X, L, S = W.make_frames(H, Z, 0.161, 2, seed=36, zero_noise=True)
    _, hard, flags, _ = oracle.decode_flood(H, Z, L, S, 3)
    assert flags.all() and np.array_equal(hard, X)


def _fd_setup():
    spec = W.RATE01_SMALL.with_Z(8)
    H = W.make_code(spec, 0)
    Z = spec.Z
    X, L, S = W.make_frames(H, Z, 0.5, 2, seed=11)
    return H, Z, X, L, S


def test_nms_gradients_match_finite_differences():
    H, Z, X, L, S = _fd_setup()
    T, mb = 3, H.shape[0]
    rng = np.random.default_rng(12)
    alpha = rng.uniform(0.6, 1.0, (T, mb, 2))
    beta = rng.uniform(0.0, 0.3, (T, mb, 2))
    loss, ga, gb, _ = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, beta)
    h = 1e-6
    checked = 0
    for (t, i, tau) in [(0, 0, 0), (1, 3, 0), (2, 5, 0), (2, 7, 1), (0, 10, 0), (1, 20, 0), (2, 30, 1)]:
        for which, P, G in (("a", alpha, ga), ("b", beta, gb)):
            Pp = P.copy(); Pp[t, i, tau] += h
            Pm = P.copy(); Pm[t, i, tau] -= h
            if which == "a":
                lp = oracle.nms_loss_grad(H, Z, L, S, X, T, Pp, beta)[0]
                lm = oracle.nms_loss_grad(H, Z, L, S, X, T, Pm, beta)[0]
            else:
                lp = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, Pp)[0]
                lm = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, Pm)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[t, i, tau]) <= 1e-6 * max(abs(fd), 1e-4) + 1e-9, (which, t, i, tau, fd, G[t, i, tau])
            checked += 1
    assert checked == 14


def test_nms_gradients_match_finite_differences_under_saturation():
    # reliable inputs drive many minima past 30; the loss is flat in q there,
    # so the exact gradient carries nothing through an active saturation
    H, Z, X, L, S = _fd_setup()
    L = (L * 12).astype(np.float32)
    T, mb = 3, H.shape[0]
    rng = np.random.default_rng(13)
    alpha = rng.uniform(0.6, 1.0, (T, mb, 2))
    beta = rng.uniform(0.0, 0.3, (T, mb, 2))
    _, ga, gb, _ = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, beta)
    h = 1e-5
    worst = 0.0
    for (t, i, tau) in [(0, 0, 0), (0, 4, 0), (1, 3, 0), (1, 8, 0), (2, 5, 0), (2, 7, 1), (1, 20, 0), (2, 30, 1)]:
        Pp = alpha.copy(); Pp[t, i, tau] += h
        Pm = alpha.copy(); Pm[t, i, tau] -= h
        fd = (oracle.nms_loss_grad(H, Z, L, S, X, T, Pp, beta)[0]
              - oracle.nms_loss_grad(H, Z, L, S, X, T, Pm, beta)[0]) / (2 * h)
        worst = max(worst, abs(fd - ga[t, i, tau]) / max(abs(fd), 1e-7))
    assert worst < 1e-4, worst


def test_nms_degree1_weights_only_act_in_the_last_iteration():
    # a degree-1 variable has a single check, so q for it stays the channel
    # LLR and its message only reaches the output at the last iteration
    H, Z, X, L, S = _fd_setup()
    T, mb = 3, H.shape[0]
    alpha = np.full((T, mb, 2), 0.9)
    beta = np.full((T, mb, 2), 0.1)
    _, ga, gb, _ = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, beta)
    assert np.all(ga[:T - 1, :, 1] == 0) and np.all(gb[:T - 1, :, 1] == 0)
    assert np.any(ga[T - 1, :, 1] != 0)
    assert np.any(ga[:, :, 0] != 0)


def test_nms_sweep_mean_loss_and_windowed_gradients():
    # loss over every sweep: the mean over tau = 1..T of the final-sweep loss
    # after tau sweeps.  With a window of W sweeps, the gradient for the
    # weights of sweep t collects the terms whose window reaches back to t,
    # tau = t+1 .. min(T, t+W); the state before a window does not depend on
    # the weights inside it, so each contribution is that term's full
    # derivative, taken here by central differences of final-sweep losses
    H, Z, X, L, S = _fd_setup()
    T, W_, mb = 4, 2, H.shape[0]
    rng = np.random.default_rng(15)
    alpha = rng.uniform(0.6, 1.0, (T, mb, 2))
    beta = rng.uniform(0.0, 0.3, (T, mb, 2))

    def final_loss(tau, a, b):
        return oracle.nms_loss_grad(H, Z, L, S, X, tau, a[:tau], b[:tau])[0]

    loss, ga, gb, _ = oracle.nms_train_grad(H, Z, L, S, X, T, alpha, beta, True, W_)
    ref = np.mean([final_loss(tau, alpha, beta) for tau in range(1, T + 1)])
    assert abs(loss - ref) <= 1e-13 * ref, (loss, ref)
    h = 1e-6
    checked = 0
    for (t, i, tau_e) in [(0, 0, 0), (1, 3, 0), (2, 5, 0), (3, 7, 1), (1, 10, 1), (0, 20, 0), (2, 30, 0)]:
        for which, P, G in (("a", alpha, ga), ("b", beta, gb)):
            fd = 0.0
            for tau in range(t + 1, min(T, t + W_) + 1):
                Pp = P.copy(); Pp[t, i, tau_e] += h
                Pm = P.copy(); Pm[t, i, tau_e] -= h
                if which == "a":
                    fd += (final_loss(tau, Pp, beta) - final_loss(tau, Pm, beta)) / (2 * h)
                else:
                    fd += (final_loss(tau, alpha, Pp) - final_loss(tau, alpha, Pm)) / (2 * h)
            fd /= T
            assert abs(fd - G[t, i, tau_e]) <= 1e-6 * max(abs(fd), 1e-4) + 1e-9, (which, t, i, tau_e, fd, G[t, i, tau_e])
            checked += 1
    assert checked == 14
    # the final-sweep loss with a full window is the exact gradient of that loss
    l0, ga0, gb0, _ = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, beta)
    l1, ga1, gb1, _ = oracle.nms_train_grad(H, Z, L, S, X, T, alpha, beta, False, T)
    assert l0 == l1 and np.array_equal(ga0, ga1) and np.array_equal(gb0, gb1)


def test_nms_loss_is_the_mean_bce_of_the_final_app():
    # the loss is the binary cross-entropy with logits, P(bit = 1) =
    # sigmoid(-APP), averaged over every frame and every one of the n bits:
    # softplus(-(1 - 2x) APP) summed and divided by F*n.  The APPs come from
    # the forward decode alone (which computes no loss) and the sum is numpy's
    H, Z, X, L, S = _fd_setup()
    T, mb = 3, H.shape[0]
    rng = np.random.default_rng(14)
    alpha = rng.uniform(0.6, 1.0, (T, mb, 2))
    beta = rng.uniform(0.0, 0.3, (T, mb, 2))
    app, _, _, _ = oracle.nms_decode(H, Z, L, S, T, alpha, beta)
    loss, _, _, app_l = oracle.nms_loss_grad(H, Z, L, S, X, T, alpha, beta)
    assert np.array_equal(app, app_l)
    sign = 1.0 - 2.0 * X.astype(np.float64)
    ref = np.logaddexp(0.0, -sign * app).sum() / (X.shape[0] * X.shape[1])
    assert loss > 0.0
    assert abs(loss - ref) <= 1e-12 * ref, (loss, ref)


def test_nms_loss_hand_case():
    # one degree-2 check (Z = 1) on bits x = (0, 1), LLRs (1.5, -0.5),
    # syndrome 0, one min-sum sweep with alpha = 1, beta = 0: each message is
    # the other bit's LLR, so both APPs are 1.5 - 0.5 = 1.0.  Bit 0 costs
    # ln(1 + e^-1), bit 1 costs ln(1 + e^1); the loss is their mean.
    H = np.array([[0, 0]], dtype=np.int32)
    L = np.array([[1.5, -0.5]], dtype=np.float32)
    S = np.array([[0]], dtype=np.uint8)
    X = np.array([[0, 1]], dtype=np.uint8)
    loss, _, _, app = oracle.nms_loss_grad(H, 1, L, S, X, 1, 1.0, 0.0)
    assert np.array_equal(app[0], [1.0, 1.0])
    hand = 0.5 * (math.log(1.0 + math.exp(-1.0)) + math.log(1.0 + math.exp(1.0)))
    assert abs(loss - hand) <= 1e-15, (loss, hand)


# --------------------------------------------------- paper table arithmetic --

def test_paper_table_arithmetic():
    t = json.load(open(os.path.join(GOLD, "paper_tables.json")))
    bits = t["codeword_bits"]
    tab1 = t["tab1"]
    # speed = codeword bits / per-codeword latency
    for lat, mbps in zip(tab1["latency_s"], tab1["mbit_s"]):
        assert abs(bits / lat / 1e6 - mbps) / mbps < 0.01
    for lat, mbps in zip(t["tabnoC_single"]["latency_s"], t["tabnoC_single"]["mbit_s"]):
        assert abs(bits / lat / 1e6 - mbps) / mbps < 0.01
    # beta = R / C with C = log2(1 + SNR) / 2
    for R, snr, b in zip(tab1["rate"], tab1["snr"], tab1["beta_percent"]):
        assert abs(100 * R / (0.5 * math.log2(1 + snr)) - b) < 0.01
    # FER counts whole frames out of 128; edge counts are multiples of Z
    for fer in tab1["fer"]:
        assert abs(fer * t["codewords"] - round(fer * t["codewords"])) < 1e-3
    for e in tab1["edges"]:
        assert e % t["expansion_factor"] == 0

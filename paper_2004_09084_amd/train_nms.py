"""Train and evaluate the learned (normalized/offset min-sum) decoder on the GPU.

Training: every step draws fresh frames on the GPU (Philox4x32-10; half at
each training SNR), runs T unrolled min-sum sweeps recording each sweep's
q's, a binary cross-entropy loss on the APPs and its gradient by reverse
sweeps (qm_nms_train_grad), then one Adam step (qm_adam_step).  Weights
start at plain min-sum (alpha = 1, beta = 0).

The default objective is the mean over the T sweeps of the BCE of each
sweep's APPs, each term's gradient taken back through `window` sweeps (its
own and the ones before it, the state before them held fixed).  At the
training SNRs the unrolled min-sum dynamics are chaotic: the exact gradient
of the final sweep's loss grows about 20x per sweep (1e32 after 25 sweeps),
beyond float32 and meaningless as a descent direction, while a short window
keeps every term's gradient exact and small.  --loss final --window T gives
the final-sweep loss with the full unroll; the training log reports how
many adjoint components reached the library's bound (0 = exact gradients).

Evaluation: a seeded batch from the workload module, decoded by the trained
min-sum with per-sweep syndrome tests (early stop, mean iterations); frames
that do not reach a valid word are decoded again from their channel LLRs by
plain sum-product, which also serves as the reference.  Reports FER, mean
iterations and decoded Mbit/s for: trained min-sum + sum-product fallback,
untrained min-sum + fallback, plain sum-product.

Every step of the decoders runs in libqcmet's kernels; this file only
sequences calls and moves a few scalars to the host for logging.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_2004_09084_amd import qcmet as Q  # noqa: E402
from paper_2004_09084_amd import workload as W  # noqa: E402


def plain_minsum_weights(T, mb, device="cuda"):
    import torch
    w = torch.zeros((T, mb, 2, 2), dtype=torch.float32, device=device)
    w[..., 0] = 1.0
    return w


def extend_weights(w, T):
    """Weights for T sweeps: sweeps past the trained ones reuse the last."""
    import torch
    if w.shape[0] >= T:
        return w[:T].contiguous()
    tail = w[-1:].expand(T - w.shape[0], *w.shape[1:])
    return torch.cat([w, tail], dim=0).contiguous()


def train(spec, shifts, steps=2000, frames=16, T=100, lr=1e-3, snrs=(0.161, 0.15), seed=0, log_every=100,
          weights=None, log=print, every_sweep=True, window=2):
    import torch
    code = Q.Code(shifts, spec.Z)
    dec = Q.Decoder([code], [frames])
    dec.nms_bind(T, train=True)
    w = plain_minsum_weights(T, spec.mb) if weights is None else weights.clone()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    x = torch.empty(frames * spec.n, dtype=torch.uint8, device="cuda")
    llr = torch.empty(frames * spec.n, dtype=torch.float32, device="cuda")
    syn = torch.empty(frames * spec.m, dtype=torch.uint8, device="cuda")
    per = frames // len(snrs)
    history = []
    clamp_total = torch.zeros(1, dtype=torch.int64, device="cuda")
    clamp_logged = 0
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        for i, snr in enumerate(snrs):
            F = per if i < len(snrs) - 1 else frames - per * (len(snrs) - 1)
            o = i * per
            Q.qm_generate_frames(dec.handle, 0, seed, (step * frames + o), snr, F,
                                 x[o * spec.n:(o + F) * spec.n], llr[o * spec.n:(o + F) * spec.n],
                                 syn[o * spec.m:(o + F) * spec.m])
        loss, grad, clamped = dec.nms_train_grad(w, llr, syn, x, T, every_sweep, window)
        clamp_total += clamped
        Q.qm_adam_step(w, grad, m, v, lr, 0.9, 0.999, 1e-8, step)
        if step % log_every == 0 or step == 1 or step == steps:
            lv = float(loss.item())
            history.append((step, lv))
            # gradients through long unrolls can exceed float32 range (the
            # library bounds the adjoints, Adam skips non-finite entries):
            # report how many entries are finite and the largest of those
            gd = grad.double()
            fin = torch.isfinite(gd)
            gmax = float(gd[fin].abs().max().item()) if bool(fin.any()) else None
            ct = int(clamp_total.item())
            log(json.dumps({"step": step, "loss": round(lv, 6), "grad_finite_frac": round(float(fin.double().mean()), 4),
                            "grad_absmax_finite": gmax, "clamped_adjoints": ct - clamp_logged,
                            "clamped_adjoints_total": ct,
                            "alpha_mean": float(w[..., 0].mean().item()), "beta_mean": float(w[..., 1].mean().item()),
                            "elapsed_s": round(time.perf_counter() - t0, 1)}))
            clamp_logged = ct
    torch.cuda.synchronize()
    return w, history, time.perf_counter() - t0, int(clamp_total.item())


def heldout_loss(spec, shifts, weights, T, frames=16, snrs=(0.161, 0.15), seed=1, batches=8, every_sweep=True):
    """Mean training loss (BCE of the APPs against the transmitted bits: the
    mean over the T sweeps, or of the last sweep only) over fresh frames
    drawn with another generator seed."""
    import torch
    code = Q.Code(shifts, spec.Z)
    dec = Q.Decoder([code], [frames])
    dec.nms_bind(T, train=True)
    x = torch.empty(frames * spec.n, dtype=torch.uint8, device="cuda")
    llr = torch.empty(frames * spec.n, dtype=torch.float32, device="cuda")
    syn = torch.empty(frames * spec.m, dtype=torch.uint8, device="cuda")
    per = frames // len(snrs)
    w = weights[:T].contiguous()
    total = 0.0
    for b in range(batches):
        for i, snr in enumerate(snrs):
            F = per if i < len(snrs) - 1 else frames - per * (len(snrs) - 1)
            o = i * per
            Q.qm_generate_frames(dec.handle, 0, seed, b * frames + o, snr, F, x[o * spec.n:(o + F) * spec.n],
                                 llr[o * spec.n:(o + F) * spec.n], syn[o * spec.m:(o + F) * spec.m])
        loss, _, _ = dec.nms_train_grad(w, llr, syn, x, T, every_sweep, 1)
        total += float(loss.item())
    return total / batches


def evaluate(spec, shifts, weights, T_nms=100, T_sp=200, frames=128, frame_seed=2, snr=None, log=print):
    """FER / mean iterations / Mbit/s of min-sum (+ sum-product fallback) and
    of plain sum-product on one seeded batch."""
    import torch
    wl = W.build(spec, frames, graph_seed=0, frame_seed=frame_seed, snr=snr)
    L = torch.from_numpy(wl.llr.reshape(-1)).cuda()
    S = torch.from_numpy(wl.s.reshape(-1)).cuda()
    code = Q.Code(shifts, spec.Z)

    def bit_errors(hard):
        h = hard.cpu().numpy().reshape(frames, -1) if hasattr(hard, "cpu") else hard
        return (h != wl.x)

    def frame_errors(hard):
        return bit_errors(hard).any(axis=1)

    # plain sum-product (the fallback decoder and the reference)
    sp = Q.Decoder([code], [frames])
    sp.decode(L, S, T_sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs, _, fs = sp.decode(L, S, T_sp)
    torch.cuda.synchronize()
    t_sp = time.perf_counter() - t0
    be_sp = bit_errors(hs)
    err_sp = be_sp.any(axis=1)

    res = {"snr": wl.meta["snr"], "frames": frames,
           "sum_product": {"fer": float(err_sp.mean()), "ber": float(be_sp.mean()), "syndrome_fail": float(1 - fs.cpu().numpy().mean()),
                           "iterations": T_sp, "mbit_s": frames * spec.n / 1e6 / t_sp}}
    nm = Q.Decoder([code], [frames])
    nm.nms_bind(T_nms, train=False)
    for name, w in (("trained_minsum", weights), ("plain_minsum", plain_minsum_weights(T_nms, spec.mb))):
        w = w[:T_nms].contiguous()
        nm.nms_decode(w, L, S, T_nms, early_stop=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hn, an, fn, it = nm.nms_decode(w, L, S, T_nms, early_stop=True)
        torch.cuda.synchronize()
        t_nms = time.perf_counter() - t0
        ok = fn.cpu().numpy().astype(bool)
        hard = hn.cpu().numpy().reshape(frames, -1).copy()
        t_fb = 0.0
        nfail = int((~ok).sum())
        if nfail:
            idx = np.nonzero(~ok)[0]
            fb = Q.Decoder([code], [nfail])
            Lf = torch.from_numpy(wl.llr[idx].reshape(-1)).cuda()
            Sf = torch.from_numpy(wl.s[idx].reshape(-1)).cuda()
            fb.decode(Lf, Sf, T_sp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hf, _, _ = fb.decode(Lf, Sf, T_sp)
            torch.cuda.synchronize()
            t_fb = time.perf_counter() - t0
            hard[idx] = hf.cpu().numpy().reshape(nfail, -1)
        be = bit_errors(hard)
        err = be.any(axis=1)
        res[name] = {"fer_minsum_only": float(frame_errors(hn).mean()),
                     "ber_minsum_only": float(bit_errors(hn).mean()),
                     "syndrome_fail_minsum_only": float(1 - ok.mean()),
                     "converged": int(ok.sum()),
                     "ber_with_fallback": float(be.mean()),
                     "mean_iterations": float(it.cpu().numpy().mean()),
                     "fer_with_fallback": float(err.mean()),
                     "fallback_frames": nfail,
                     "mbit_s_with_fallback": frames * spec.n / 1e6 / (t_nms + t_fb),
                     "seconds_minsum": t_nms, "seconds_fallback": t_fb}
    log(json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--spec", default="r0.1_Z20000")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--T", type=int, default=100, help="min-sum sweeps at evaluation")
    ap.add_argument("--T-train", type=int, default=None,
                    help="unrolled sweeps while training (default T); later sweeps reuse the last trained sweep's "
                         "weights")
    ap.add_argument("--loss", choices=("sweeps", "final"), default="sweeps",
                    help="BCE averaged over every sweep's APPs, or of the last sweep's only")
    ap.add_argument("--window", type=int, default=2,
                    help="sweeps each loss term's gradient runs back through (0 = all)")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-frames", type=int, default=128, help="0: no evaluation")
    ap.add_argument("--train-snrs", default="0.161,0.15",
                    help="SNRs of the training frames, an equal share of each batch per SNR")
    ap.add_argument("--eval-snrs", default="0.161")
    ap.add_argument("--save", default=None, help="write trained weights (.npy)")
    ap.add_argument("--load", default=None, help="start from weights (.npy)")
    args = ap.parse_args()
    import torch
    spec = W.SPECS[args.spec]
    shifts = W.make_code(spec, 0)
    w0 = None
    if args.load:
        w0 = torch.from_numpy(np.load(args.load)).cuda()
    w = w0
    T_train = args.T_train or args.T
    if args.steps > 0:
        snrs = tuple(float(x) for x in args.train_snrs.split(",") if x)
        every = args.loss == "sweeps"
        win = args.window if args.window > 0 else T_train
        w, hist, secs, clamped = train(spec, shifts, steps=args.steps, frames=args.frames, T=T_train, lr=args.lr, snrs=snrs,
                              seed=args.seed, weights=None if w0 is None else w0[:T_train].contiguous(),
                              every_sweep=every, window=win)
        print(json.dumps({"trained_steps": args.steps, "T_train": T_train, "train_snrs": snrs, "loss": args.loss,
                          "window": win, "train_seconds": round(secs, 1), "clamped_adjoints_total": clamped,
                          "loss_first": hist[0][1], "loss_last": hist[-1][1]}), flush=True)
    if w is None:
        w = plain_minsum_weights(args.T, spec.mb)
    if args.steps > 0:
        # the training objective on frames it never saw, trained against plain min-sum
        snrs = tuple(float(x) for x in args.train_snrs.split(",") if x)
        lt = heldout_loss(spec, shifts, w, T_train, frames=args.frames, snrs=snrs, seed=args.seed + 1,
                          every_sweep=every)
        lp = heldout_loss(spec, shifts, plain_minsum_weights(T_train, spec.mb), T_train, frames=args.frames, snrs=snrs,
                          seed=args.seed + 1, every_sweep=every)
        print(json.dumps({"heldout_loss_trained": round(lt, 6), "heldout_loss_plain_minsum": round(lp, 6)}), flush=True)
    w = extend_weights(w, args.T)
    if args.save:
        np.save(args.save, w.cpu().numpy())
    for snr in [float(s) for s in args.eval_snrs.split(",") if s] if args.eval_frames > 0 else []:
        evaluate(spec, shifts, w, T_nms=args.T, frames=args.eval_frames, snr=snr)


if __name__ == "__main__":
    main()

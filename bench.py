"""Decode-throughput benchmark on one MI355X.

A step is one qm_decode of the whole batch: init, `iters` layered
sum-product sweeps, syndrome flags and the frame-major outputs.  Default
workload: rate-0.1 QC-MET-LDPC code (45 x 50 base, Z = 20000, n = 10^6),
128 frames at SNR 0.161, 200 iterations, FP32 messages; the inputs are
generated once (seeded, synthetic) and are resident in HBM before the timed
region starts.

Prints one JSON line: decoded Mbit/s (frames x 10^6 bits per second), the
layer kernel's achieved algorithmic HBM bandwidth against the 8 TB/s peak
(timed live with HIP events on the decode stream), FER at the SNR, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "decoded Mbit/s (N frames x 10^6 bits, fixed iters) + HBM GB/s; FER at SNR"

WORKLOADS = {
    # name: ([(spec name, frames), ...], iterations)
    "r0.1": ([("r0.1_Z20000", 128)], 200),
    "r0.05": ([("r0.05_Z10000", 128)], 200),
    "r0.02": ([("r0.02_Z10000", 128)], 200),
    "small": ([("r0.1_Z64", 4)], 50),
    # mixed-rate batch: 64 + 32 + 32 frames of the three codes, fused launches
    "mixed": ([("r0.1_Z20000", 64), ("r0.05_Z10000", 32), ("r0.02_Z10000", 32)], 200),
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("layer.h", "phi.h", "device_common.h", "qcmet_internal.h", "layer_f32.hip", "layer_f16.hip",
              "layer_f8.hip"):
        with open(os.path.join(ROOT, "paper_2004_09084_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload_key: str, msg: str):
    """Off-chip bytes per layer launch from the committed rocprofv3 counter
    runs (FETCH_SIZE, WRITE_SIZE, calibrated), if they were taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "layer_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    key = f"{workload_key}{'_' + msg if msg else ''}"
    ent = data.get(key)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def host_cpus():
    """What the host offers this process: the CPUs in its affinity mask, the
    cgroup CPU quota (cpu.max, in CPUs; None when unlimited) and the CPU
    model name."""
    aff = len(os.sched_getaffinity(0))
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = round(int(q) / int(period), 2)
    except (OSError, ValueError):
        pass
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return aff, quota, model


def cpu_baseline(spec, shifts, frames_llr, frames_s, iters_full, target_s=10.0):
    """The FP64 oracle, as it stands, on a bounded sample: one frame per CPU
    of the process's affinity mask (the whole host share, no cap), timed over
    as many iterations as take about `target_s` seconds (2 to 64, from a
    2-iteration probe); scaled to Mbit/s at the full iteration count (with
    early termination: the GPU's mean count)."""
    import oracle
    aff, quota, model = host_cpus()
    threads = aff
    F = min(threads, frames_llr.shape[0])
    t0 = time.perf_counter()
    oracle.decode_sp(shifts, spec.Z, frames_llr[:F], frames_s[:F], 2, threads=threads)
    probe = time.perf_counter() - t0
    sample_iters = int(max(2, min(64, round(target_s / max(probe / 2, 1e-3)))))
    t0 = time.perf_counter()
    _, _, _, used = oracle.decode_sp(shifts, spec.Z, frames_llr[:F], frames_s[:F], sample_iters, threads=threads)
    dt = time.perf_counter() - t0
    per_decode = dt * iters_full / sample_iters          # seconds for F frames at full iterations
    return {"value": round(F * spec.n / 1e6 / per_decode, 4), "unit": "Mbit/s", "cores": int(used),
            "kind": "oracle", "affinity_cpus": aff, "cgroup_cpu_quota": quota, "cpu_model": model,
            "sample": f"{F} frames x {sample_iters} iterations of the same code and inputs "
                      f"({dt:.1f} s wall), scaled to {iters_full:g} iterations"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="r0.1", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=None, help="frames (single-code workloads)")
    ap.add_argument("--snr", type=float, default=None, help="override the workload SNR")
    ap.add_argument("--frame-seed", type=int, default=None,
                    help="frame seed (default 0; 1 for the mixed batch, whose frames differ from the single-code ones)")
    ap.add_argument("--autotune", action="store_true", help="run qm_autotune before timing")
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--fp16", action="store_true", help="store messages as binary16")
    ap.add_argument("--fp8", action="store_true", help="store messages as 8-bit floats (e4m3)")
    ap.add_argument("--tuning", default=None, help="JSON dict of qm_tuning fields")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--flooding", action="store_true", help="flooding schedule instead of layers")
    ap.add_argument("--early-stop", action="store_true",
                    help="qm_decode_early: frames stop once H c = s (iterations = the maximum)")
    ap.add_argument("--gpu-frames", action="store_true",
                    help="draw the frames on the GPU (library Philox generator) instead of numpy on the host; "
                         "for large --frames (no CPU baseline then)")
    ap.add_argument("--end-to-end", action="store_true",
                    help="also time decodes that include copying the LLRs and syndromes from pinned host memory "
                         "and the hard decisions and flags back (reported beside the value, never as it)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library decodes on a single MI355X "
              "(frames would shard across GPUs with no exchange; not built). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2004_09084_amd import qcmet as Q
    from paper_2004_09084_amd import workload as W

    if args.frame_seed is None:
        args.frame_seed = 1 if args.workload == "mixed" else 0
    parts, iters = WORKLOADS[args.workload]
    if args.frames and len(parts) == 1:
        parts = [(parts[0][0], args.frames)]
    iters = args.iters if args.iters is not None else iters
    specs = [W.SPECS[p[0]] for p in parts]
    Fs = [p[1] for p in parts]
    F = sum(Fs)
    torch.cuda.set_device(0)

    tuning = json.loads(args.tuning) if args.tuning else None
    flags = (Q.QM_MSG_FP16 if args.fp16 else 0) | (Q.QM_MSG_FP8 if args.fp8 else 0) \
        | (Q.QM_EARLY_STOP if args.early_stop else 0) | (Q.QM_FLOODING if args.flooding else 0)
    msg_name = "FP16" if args.fp16 else "FP8 (e4m3)" if args.fp8 else "FP32"
    if args.gpu_frames:
        # frames drawn on the device by the library's Philox generator (keyed
        # by the frame seed and frame index): for large frame counts, whose
        # host generation would take minutes; same code construction
        import types
        args.no_cpu_baseline = True
        codes, wls = [], []
        for spec in specs:
            shifts = W.make_code(spec, 0)
            codes.append(Q.Code(shifts, spec.Z))
            wls.append(types.SimpleNamespace(shifts=shifts, meta={"snr": spec.snr if args.snr is None else args.snr}))
        dec = Q.Decoder(codes, Fs, flags=flags, tuning=tuning)
        n_all = sum(Fc * spec.n for Fc, spec in zip(Fs, specs))
        m_all = sum(Fc * spec.m for Fc, spec in zip(Fs, specs))
        x = torch.empty(n_all, dtype=torch.uint8, device="cuda")
        llr = torch.empty(n_all, dtype=torch.float32, device="cuda")
        syn = torch.empty(m_all, dtype=torch.uint8, device="cuda")
        on = om = 0
        for c, (spec, Fc, w) in enumerate(zip(specs, Fs, wls)):
            print(f"[bench] drawing {Fc} frames of {spec.name} (n={spec.n}) at SNR {w.meta['snr']} on the GPU",
                  file=sys.stderr, flush=True)
            Q.qm_generate_frames(dec.handle, c, args.frame_seed, 0, w.meta["snr"], Fc, x[on:on + Fc * spec.n],
                                 llr[on:on + Fc * spec.n], syn[om:om + Fc * spec.m])
            on += Fc * spec.n
            om += Fc * spec.m
        torch.cuda.synchronize()
        on = 0
        for spec, Fc, w in zip(specs, Fs, wls):
            w.x = x[on:on + Fc * spec.n].cpu().numpy().reshape(Fc, -1)
            on += Fc * spec.n
        del x
    else:
        wls = []
        for spec, Fc in zip(specs, Fs):
            snr = spec.snr if args.snr is None else args.snr
            print(f"[bench] generating {Fc} frames of {spec.name} (n={spec.n}) at SNR {snr}", file=sys.stderr,
                  flush=True)
            wls.append(W.build(spec, Fc, graph_seed=0, frame_seed=args.frame_seed, snr=snr))
        llr = torch.from_numpy(np.concatenate([w.llr.reshape(-1) for w in wls])).cuda()
        syn = torch.from_numpy(np.concatenate([w.s.reshape(-1) for w in wls])).cuda()
        codes = [Q.Code(w.shifts, spec.Z) for w, spec in zip(wls, specs)]
        dec = Q.Decoder(codes, Fs, flags=flags, tuning=tuning)
    out = dec.alloc_outputs(want_app=True)
    iters_used = None

    def step():
        nonlocal iters_used
        if args.early_stop:
            iters_used = dec.decode_early(llr, syn, iters, out=out)[3]
        else:
            dec.decode(llr, syn, iters, out=out)
    torch.cuda.synchronize()

    if args.calib_copy_mb:
        # known traffic for the counter runs: a fill writes N bytes, an
        # elementwise multiply reads N and writes N bytes
        src = torch.empty(args.calib_copy_mb << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    if args.autotune:
        print("[bench] autotuning", file=sys.stderr, flush=True)
        dec.autotune(llr, syn, iters, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done; timing {args.steps} steps", file=sys.stderr, flush=True)

    dec.set_profiling(not args.no_profile)
    dec.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = dec.profile(reset=True)
    dec.set_profiling(False)

    ms_per_step = dt * 1e3 / args.steps
    bits = sum(Fc * spec.n for Fc, spec in zip(Fs, specs))
    mbit_s = bits / 1e6 / (dt / args.steps)
    hard_all = out[0].cpu().numpy()
    flags = out[2].cpu().numpy()
    per_code = []
    frame_err = []
    on = of = 0
    for w, spec, Fc in zip(wls, specs, Fs):
        err = (hard_all[on:on + Fc * spec.n].reshape(Fc, -1) != w.x).any(axis=1)
        frame_err.append(err)
        per_code.append({"code": spec.name, "frames": Fc, "snr": w.meta["snr"], "fer": float(err.mean()),
                         "syndrome_fail_rate": float(1.0 - flags[of:of + Fc].mean())})
        on += Fc * spec.n
        of += Fc
    fer = float(np.concatenate(frame_err).mean())
    syn_fail = float(1.0 - flags.mean())

    roofline = None
    lds_total = prof.get("lds_ms", 0.0)
    if prof.get("lds_launches", 0) > 0 and prof["launches"] == 0:
        # the LDS-resident decode dominates: one launch per decode, all sweeps;
        # its algorithmic HBM bytes leave out the APPs held in LDS
        avg_ms = lds_total / prof["lds_launches"]
        achieved = prof["lds_bytes"] / prof["lds_launches"] / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_sweeps_lds", "avg_launch_us": round(avg_ms * 1e3, 3),
                    "algorithmic_bytes_per_launch": round(prof["lds_bytes"] / prof["lds_launches"]),
                    "launches_timed": prof["lds_launches"],
                    "timing": "HIP events around each LDS-resident decode launch (all sweeps) on the decode stream",
                    "bytes": "messages read+written and degree-1 terms per check and sweep; APPs once per frame"}
    elif len(codes) > 1 and dec.tuning()["fuse_codes"] == 2 and not args.flooding:
        # each code on its own stream: the kernels of different codes overlap,
        # so the figure is the whole decode's algorithmic bytes over its time
        # (per type-1 edge APP and message read + write, per check K read)
        mb = 2 if args.fp16 else 1 if args.fp8 else 4
        dec_bytes = sum(Fc * c.info.Z * ((8 + 2 * mb) * c.info.n_type1_entries + 4 * c.info.mb) * iters
                        for c, Fc in zip(codes, Fs))
        achieved = dec_bytes / (dt / args.steps) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_layer_sp (each code on its own stream, launches overlapping)",
                    "algorithmic_bytes_per_decode": round(dec_bytes),
                    "timing": "wall time of whole decodes (the codes' launches overlap, so no per-launch figure)"}
    elif prof["launches"] > 0:
        avg_ms = prof["layer_ms"] / prof["launches"]
        bytes_per_launch = prof["layer_bytes"] / prof["launches"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        traffic = load_traffic(args.workload, "fp16" if args.fp16 else "fp8" if args.fp8 else "")
        if args.early_stop:
            traffic = None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": "k_layer_sp_et" if args.early_stop
                              else "k_layer_flood + k_flood_vars (one iteration)" if args.flooding
                              else "k_layer_multi (one launch per step over every code)" if len(codes) > 1
                              else "k_layer_sp",
                    "avg_launch_us": round(avg_ms * 1e3, 3),
                    "algorithmic_bytes_per_launch": round(bytes_per_launch),
                    "launches_timed": prof["launches"],
                    "timing": "HIP events around whole sweeps on the decode stream"
                              + (" (first sweep of each decode, every tile decoding)" if args.early_stop else "")}
        if len(codes) == 1 and not args.early_stop and not args.flooding:
            # the same launches counting only the message and degree-1 bytes:
            # the APP working set (frames x degree>=2 variables x 4 B, 51 MB
            # for 128 frames at rate 0.1) fits in the 256 MB Infinity Cache,
            # so part of the APP traffic may never reach HBM; this is the
            # figure with none of it counted
            mb = 2 if args.fp16 else 1 if args.fp8 else 4
            ci = codes[0].info
            full = 8 + 2 * mb
            ratio = (2 * mb * ci.n_type1_entries + 4 * ci.mb) / (full * ci.n_type1_entries + 4 * ci.mb)
            roofline["messages_only"] = {"bytes_per_launch": round(bytes_per_launch * ratio),
                                         "achieved": round(achieved * ratio, 1),
                                         "frac": round(achieved * ratio / HBM_PEAK_GBS, 4)}

    e2e = None
    if args.end_to_end:
        # pinned host copies of the inputs and outputs (allocated pinned, not
        # registered); each timed step copies in, decodes, copies out
        h_llr = torch.empty(llr.numel(), dtype=llr.dtype, pin_memory=True)
        h_syn = torch.empty(syn.numel(), dtype=syn.dtype, pin_memory=True)
        h_llr.copy_(llr.cpu())
        h_syn.copy_(syn.cpu())
        h_hard = torch.empty(out[0].numel(), dtype=out[0].dtype, pin_memory=True)
        h_flags = torch.empty(out[2].numel(), dtype=out[2].dtype, pin_memory=True)

        def e2e_step():
            llr.copy_(h_llr, non_blocking=True)
            syn.copy_(h_syn, non_blocking=True)
            step()
            h_hard.copy_(out[0], non_blocking=True)
            h_flags.copy_(out[2], non_blocking=True)

        e2e_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e2e_step()
        torch.cuda.synchronize()
        dt_e = (time.perf_counter() - t0) / args.steps
        e2e = {"value": round(bits / 1e6 / dt_e, 3), "unit": "Mbit/s", "ms_per_step": round(dt_e * 1e3, 3),
               "copies": "LLR + syndrome host-to-device, hard decisions + flags device-to-host, pinned host memory, "
                         "not overlapped with the decode"}

    early = None
    cpu_iters = iters
    if args.early_stop:
        it = iters_used.cpu().numpy()
        early = {"max_iterations": iters, "mean_iterations": round(float(it.mean()), 3),
                 "iterations_histogram": np.bincount(it, minlength=iters + 1).tolist()}
        cpu_iters = float(it.mean())

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(specs[0], wls[0].shifts, wls[0].llr, wls[0].s, cpu_iters)

    tun = dec.tuning()
    line = {
        "metric": METRIC.replace("fixed iters", "early termination") if args.early_stop else METRIC,
        "value": round(mbit_s, 3), "unit": "Mbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if msg_name == "FP32" else f"f32 ({msg_name} messages)", "data": "synthetic" + (" (frames drawn on the GPU)" if args.gpu_frames else ""),
        "config": {"workload": " + ".join(
                       f"{Fc} x {spec.name} (rate {spec.rate:.2f} QC-MET-LDPC, {spec.mb}x{spec.nb} base, Z={spec.Z}, "
                       f"n={spec.n}, SNR {w.meta['snr']})" for w, spec, Fc in zip(wls, specs, Fs))
                   + (f", at most {iters} iterations with early termination" if args.early_stop
                      else f", {iters} iterations") + f", {'flooding' if args.flooding else 'layered'} sum-product, "
                   f"{msg_name} messages",
                   "frames": F, "iterations": iters, "layers": [int(c.info.G) for c in codes], "tuning": tun,
                   "per_code": per_code},
        "fer": fer, "syndrome_fail_rate": syn_fail, "early_stop": early,
        "hbm_gbs": None if roofline is None else roofline["achieved"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "end_to_end": e2e,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of the fast aperture-mass path on one MI355X.

A step is one pass of the whole path over one synthetic 1024 x 1024 float32
shear map: Kaiser-Squires inversion, the starlet transform with J = 7 planes
(radii 2..64 px), 256 shear-randomised noise realisations (each its own KS +
starlet pass), per-pixel sigma_j, S/N planes and peak counts above S/N = 3.

value = Mpix*scales/s = (1 + R) * N^2 * J / t / 1e6, i.e. the signal map and
every noise realisation, each producing J planes of N^2 pixels.

Printed as one JSON line.  Extra objects:
  plain        one map through KS + starlet, one launch sequence per map
  roofline     the dominant kernel, timed with HIP events on its stream
  kernels      per-kernel launches and average microseconds
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpix·scales/s starlet+KS (% HBM peak), batched vs plain; p50/p99 latency served"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3

N, J, R_REAL, SEED, THRESH = 1024, 7, 256, 23, 3.0
GRF_SEED, NOISE_SEED = 11, 12


def kernel_model(name, n, J, batch_real):
    """Algorithmic bytes and flops of one launch of each kernel (float32).

    bytes: the kernel's compulsory input + output, each operand read or
    written once per launch (the shared shear map once per launch; the
    double-precision noise accumulators read and written once per launch);
    flops: 5 m log2 m per length-m complex FFT, 6 per complex multiply,
    19 per pixel and starlet scale (two 5-tap B3 filters and a difference),
    4 per pixel and scale for the running mean and squared deviation.
    """
    n2 = float(n * n)
    lg = n.bit_length() - 1
    B = batch_real
    fft1d = 5.0 * n2 * lg  # n transforms of length n
    scales_last = (J - 1) - 3 * ((J - 2) // 3)  # scales in the last stage
    models = {
        "ks_cols_fwd_rotate": (8.0 * n2 + 8.0 * n2 * B, B * (fft1d + 6.0 * n2)),
        "ks_cols_fwd": (16.0 * n2, fft1d),
        "ks_rows": (16.0 * n2 * B, B * (2 * fft1d + 6.0 * n2)),
        "ks_cols_inv": (12.0 * n2 * B, B * fft1d),
        "noise_stage_j1": ((8.0 * B + 96.0) * n2, 3 * (19.0 + 4.0) * n2 * B),
        "noise_stage_j4": ((4.0 * B + 32.0 * scales_last) * n2,
                           scales_last * (19.0 + 4.0) * n2 * B),
        "starlet_stage_j1": (20.0 * n2, 3 * 19.0 * n2),
        "starlet_stage_j4": ((8.0 + 4.0 * scales_last) * n2, scales_last * 19.0 * n2),
        "noise_finalize": ((16.0 + 12.0) * (J - 1) * n2, 3.0 * (J - 1) * n2),
        "count_peaks": (4.0 * (J - 1) * n2, 9.0 * (J - 1) * n2),
    }
    return models.get(name, (None, None))


def cpu_baseline(g1, g2, budget_s):
    """Time the FP64 oracle on a bounded sample: the signal map plus as many
    noise realisations as fit in about ``budget_s`` seconds."""
    import oracle
    t0 = time.perf_counter()
    kE, _ = oracle.ks_invert(g1, g2)
    planes = oracle.starlet_forward(kE, J)
    t_sig = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.noise_sigma(g1, g2, J, 2, SEED)
    per_real = (time.perf_counter() - t1) / 2
    r = max(2, int(budget_s / max(per_real, 1e-3)))
    t2 = time.perf_counter()
    sig = oracle.noise_sigma(g1, g2, J, r, SEED)
    snr = oracle.snr_planes(planes, sig)
    oracle.count_peaks_planes(snr, THRESH)
    t_noise = time.perf_counter() - t2
    units = 1 + r
    total = t_sig + t_noise
    return {"value": units * N * N * J / total / 1e6, "unit": "Mpix·scales/s",
            "cores": 1, "kind": "oracle",
            "sample": "the 1024x1024 map: KS + starlet (J=7) of the signal and %d noise "
                      "realisations with sigma, S/N and peaks, %.1f s" % (r, total),
            "cpu": platform.processor() or platform.machine()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle's timed sample (0 to skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); the "
              "multi-GPU sharding is a design, not built" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_1204_4293_amd as amap

    dev = torch.device("cuda", 0)
    _, g1, g2 = synth.shear_map(N, GRF_SEED, NOISE_SEED)
    t1 = torch.tensor(g1, dtype=torch.float32, device=dev)
    t2 = torch.tensor(g2, dtype=torch.float32, device=dev)
    ctx = amap.Context(0)
    out = {
        "kappa_e": torch.empty((N, N), dtype=torch.float32, device=dev),
        "planes": torch.empty((J, N, N), dtype=torch.float32, device=dev),
        "sigma": torch.empty((J - 1, N, N), dtype=torch.float32, device=dev),
        "snr": torch.empty((J - 1, N, N), dtype=torch.float32, device=dev),
        "peaks": torch.empty(J - 1, dtype=torch.int64, device=dev),
    }

    def step():
        ctx.run_path(t1, t2, J, R_REAL, SEED, THRESH, out=out)

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)

    # timed region: whole steps, wall clock and torch events on the launch stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    units = 1 + R_REAL
    value = units * N * N * J / (ms_per_step * 1e-3) / 1e6
    print("bench: timed %d steps, %.3f ms/step" % (args.steps, ms_per_step), file=sys.stderr,
          flush=True)

    # per-kernel HIP-event timing over the same number of steps
    ctx.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ktimes = ctx.timing_read(reset=True)
    ctx.timing_enable(False)
    B = min(R_REAL, max(1, (1 << 25) // (N * N)))
    kernels = {}
    for name, (launches, tot_ms) in sorted(ktimes.items(), key=lambda kv: -kv[1][1]):
        kernels[name] = {"launches_per_step": launches / args.steps,
                         "avg_us": 1e3 * tot_ms / launches,
                         "ms_per_step": tot_ms / args.steps}
    dom = max(ktimes.items(), key=lambda kv: kv[1][1])[0]
    dom_avg_s = ktimes[dom][1] / ktimes[dom][0] * 1e-3
    b_alg, f_alg = kernel_model(dom, N, J, B)
    for name, rec in kernels.items():
        bb, ff = kernel_model(name, N, J, B)
        if bb is not None:
            rec["alg_GBps"] = bb / (rec["avg_us"] * 1e-6) / 1e9
            rec["alg_TFLOPs"] = ff / (rec["avg_us"] * 1e-6) / 1e12
    roofline = {"kernel": dom, "bound": "hbm",
                "achieved": b_alg / dom_avg_s / 1e9 if b_alg else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None,
                "bytes_per_launch": b_alg, "avg_launch_us": dom_avg_s * 1e6,
                "flops_per_launch": f_alg,
                "tflops": f_alg / dom_avg_s / 1e12 if f_alg else None}
    roofline["frac"] = roofline["achieved"] / roofline["peak"] if b_alg else None

    # plain path: one map, KS + starlet, one launch sequence per map
    ke = out["kappa_e"]
    pl = out["planes"]
    for _ in range(3):
        ctx.ks_invert(t1, t2, kappa_e=ke)
        ctx.starlet_forward(ke, J, planes=pl)
    torch.cuda.synchronize()
    reps = 50
    ev0.record()
    for _ in range(reps):
        ctx.ks_invert(t1, t2, kappa_e=ke)
        ctx.starlet_forward(ke, J, planes=pl)
    ev1.record()
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1) / reps
    b_alg_map = N * N * (8 + 4 * J)
    plain = {"value": N * N * J / (plain_ms * 1e-3) / 1e6, "unit": "Mpix·scales/s",
             "ms_per_map": plain_ms,
             "hbm_alg_frac": b_alg_map / (plain_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}

    line = {
        "metric": METRIC, "value": value, "unit": "Mpix·scales/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1024x1024 float32 shear map (GRF kappa, P(k)~k^-2, rms 0.02, "
                               "E-mode shear + N(0,0.3/sqrt(20)) noise); KS + starlet J=7 + "
                               "256 randomised noise realisations + sigma, S/N, peaks (S/N>3)",
                   "n": N, "J": J, "n_real": R_REAL, "batch_realisations": B},
        "wall_s_timed": wall,
        "hbm_alg_frac": (N * N * (8 + 4 * J) + 8 * (J - 1) * N * N) / (ms_per_step * 1e-3)
                        / (HBM_PEAK_GBS * 1e9),
        "plain": plain, "roofline": roofline, "kernels": kernels,
    }
    ctx.close()
    if args.cpu_seconds > 0:
        print("bench: cpu baseline (oracle, ~%.0f s)" % args.cpu_seconds, file=sys.stderr,
              flush=True)
        line["cpu_baseline"] = cpu_baseline(np.asarray(g1), np.asarray(g2), args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

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
  batched      512 uneven maps (KS + starlet) as one grouped, graph-captured
               plan, and the same maps one launch sequence per map
  served       a Poisson request stream through the library's request loop:
               saturated rate, then p50/p99 latency at 0.25, 0.5 and 0.8 of it
  statistics   plane moments and peak-height histograms on the step's planes
  direct_vs_starlet  map_direct at theta = 2..64 (cut theta, and cut 2 theta)
               vs KS + starlet with J = log2 theta + 1 on the 1024^2 map (the
               paper's comparison)
  small_fp64   one 256^2 float64 map: KS + starlet J = 5 latency, and map_direct
               at theta = 2, 4, 8 (cut 2 theta)
  bounded      a 1000 x 1000 field with edges (a crop of the map): KS of the
               field zero-extended into a 2048^2 grid + starlet J = 7 under the
               mirror edge rule; and its noise sigma, S/N and peaks from 16
               realisations
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
# MI355X vector FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
# = 78.6 TFLOP/s per instruction stream; 157.3 TFLOP/s counts packed
# (two-wide) FP32 instructions, which this build does not emit
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6

N, J, R_REAL, SEED, THRESH = 1024, 7, 256, 23, 3.0
TRAFFIC_PROFILE = "noise_path_1024_J7_R256_traffic.md"
PLAIN_PROFILE = "plain_1024_J7_traffic.md"
BATCHED_PROFILE = "uneven_batch_512_traffic.md"
# tuned stage schedules of the bench's shapes, loaded instead of tuning live
# (so that its kernels are exactly those of the committed profiles)
SCHEDULES = "noise_path_1024_J7_R256_schedules.json"
GRF_SEED, NOISE_SEED = 11, 12


def kernel_model(name, n, J, batch_real, stage_starts=()):
    """Design bytes and algorithmic flops of one launch of each kernel (float32).

    flops follow the per-realisation work of the method: 5 m log2 m per
    length-m complex FFT, so 20 n^2 log2 n for the forward and inverse 2-D
    transforms of one map; 6 per complex multiply (the KS kernel); 50 per
    pixel for the random phase and the rotation; 19 per pixel and starlet
    scale (two 5-tap B3 filters and a difference); 4 per pixel and scale for
    the running mean and squared deviation.  Each kernel is credited with
    the part of that work it carries out: the column pass the forward
    column FFTs (and the phases), the row pass the forward and inverse row
    FFTs and the multiply, the inverse column pass the inverse column FFTs.
    The paired kernels (ks_rows_pair, ks_cols_inv_pair) finish two
    realisations' inverse transforms in one (their kappa_E are the real and
    imaginary parts of one transform), so they complete the credited work
    with half of the inverse arithmetic.

    bytes: the kernel's design hand-offs, each operand read or written once
    per launch (the shared shear map once per launch; the double-precision
    noise accumulators read and written once per launch).  ``stage_starts``
    lists the first scale of each noise stage (from the kernel names), which
    fixes how many scales a stage covers.  The signal's kernels
    (ks_cols_fwd, ks_rows, ks_cols_inv, starlet_stage_*) take one map; the
    noise kernels take the batch.

    The bytes the *method* requires are only the shear in and the planes,
    sigma and S/N out (``compulsory_bytes``): a noise realisation needs no
    HBM traffic at all, so every kernel of the noise loop is bounded by its
    arithmetic.
    """
    n2 = float(n * n)
    lg = n.bit_length() - 1
    B = batch_real
    P = (B + 1) // 2  # realisation pairs
    fft1d = 5.0 * n2 * lg  # n transforms of length n
    models = {
        "ks_cols_fwd_rotate": (8.0 * n2 + 8.0 * n2 * B, B * (fft1d + 50.0 * n2)),
        "ks_cols_fwd": (16.0 * n2, fft1d),
        "ks_rows": (16.0 * n2, 2 * fft1d + 6.0 * n2),
        "ks_cols_inv": (12.0 * n2, fft1d),
        # read B spectra, write P packed ones
        "ks_rows_pair": (8.0 * n2 * (B + P), B * (2 * fft1d + 6.0 * n2)),
        # read P packed spectra, write B real maps
        "ks_cols_inv_pair": (8.0 * n2 * P + 4.0 * n2 * B, B * fft1d),
        "noise_finalize": ((16.0 + 12.0) * (J - 1) * n2, 3.0 * (J - 1) * n2),
        "count_peaks": (4.0 * (J - 1) * n2, 9.0 * (J - 1) * n2),
    }
    starts = sorted(stage_starts)
    for i, j0 in enumerate(starts):
        last = i + 1 == len(starts)
        ns = (J - j0) if last else starts[i + 1] - j0
        # read c_{j0-1}, write c_{j0+ns-1} unless last, M and M2 of ns scales
        rd = 4.0 * B * n2 + 16.0 * ns * n2
        wr = (0.0 if last else 4.0 * B * n2) + 16.0 * ns * n2
        models["noise_stage_j%d" % j0] = (rd + wr, ns * (19.0 + 4.0) * n2 * B)
        # the signal's write-mode stage: read c, write ns planes and the last c
        models["starlet_stage_j%d" % j0] = ((4.0 + 4.0 * ns + 4.0) * n2, ns * 19.0 * n2)
    return models.get(name, (None, None))


NOISE_KERNELS = ("ks_cols_fwd_rotate", "ks_rows_pair", "ks_cols_inv_pair", "merge_partials")


def compulsory_bytes(name, n, J):
    """HBM bytes the method itself requires of one launch: 0 for every
    kernel of the noise loop (realisations live and die on the chip), the
    input and output planes for the signal's kernels, sigma and S/N out
    for the finalize step, the S/N planes in for the peak count."""
    n2 = float(n * n)
    if name in NOISE_KERNELS or name.startswith("noise_stage_j"):
        return 0.0
    return {"ks_cols_fwd": 8.0 * n2, "ks_rows": 0.0, "ks_cols_inv": 4.0 * n2,
            "noise_finalize": 8.0 * (J - 1) * n2 + 4.0 * J * n2,
            "count_peaks": 4.0 * (J - 1) * n2}.get(name, 4.0 * n2 if name.startswith("starlet_stage_j") else None)


def roofline_of(name, n, J, B, starts, avg_s):
    """The binding roofline of one kernel: HBM if its required bytes take
    longer at 8 TB/s than its algorithmic flops at the FP32 peak, else ALU."""
    b_des, f_alg = kernel_model(name, n, J, B, starts)
    b_req = compulsory_bytes(name, n, J)
    if f_alg is None or b_req is None:
        return None
    t_hbm = b_req / (HBM_PEAK_GBS * 1e9)
    t_alu = f_alg / (FP32_PEAK_TFLOPS * 1e12)
    if t_hbm >= t_alu:
        ach = b_req / avg_s / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS}
    ach = f_alg / avg_s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP32_PEAK_TFLOPS, "peak_nonpacked": FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": ach / FP32_NONPACKED_TFLOPS}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def kernel_sources_sha256():
    """Digest of the library's kernel sources (every source but the host-only
    api.hip); a stored counter summary is only used while it matches."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1204_4293_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".h")) and f != "api.hip":  # api.hip is host code only
            with open(os.path.join(src, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def profile_line(profile, key):
    """The JSON value of the line ``key: ...`` of a committed rocprofv3
    summary under profiles/, or None when the summary is missing, lacks the
    line, or was taken on other kernel sources (its digest differs)."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    sha, val = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("kernel-sources-sha256:"):
                sha = line.split(":", 1)[1].strip()
            elif line.startswith(key + ":"):
                val = json.loads(line.split(":", 1)[1])
    if sha != kernel_sources_sha256():
        return None
    return val


def measured_traffic(kernel, profile=TRAFFIC_PROFILE):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of the noise path (each counter scaled
    by its reading for a copy of known size), or None when that summary was
    taken on other kernel sources or does not cover the kernel."""
    table = profile_line(profile, "traffic-json")
    if not table or kernel not in table:
        return None
    return table[kernel]["bytes_per_launch"]


def _oracle_moments(args):
    """One worker's run of realisations through the oracle (bench leg only)."""
    import oracle
    g1, g2, J_, seed, a, b = args
    return oracle.noise_moments(g1, g2, J_, seed, a, b)


def cpu_baseline(g1, g2, budget_s):
    """Time the FP64 oracle on a bounded sample of the step: the signal map
    plus as many noise realisations as fit in about ``budget_s`` seconds,
    first on one core, then on all cores of the host (at most 16) with the
    realisations spread over a process pool, each worker running the oracle
    unchanged on a consecutive run of realisations and the runs merged by
    the oracle's pairwise update."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

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
    total1 = t_sig + t_noise
    single = {"value": (1 + r) * N * N * J / total1 / 1e6, "cores": 1,
              "sample": "the signal and %d noise realisations, %.1f s" % (r, total1)}

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    each = max(2, int(budget_s / max(per_real, 1e-3)))
    r_all = cores * each
    jobs = [(g1, g2, J, SEED, k * each, (k + 1) * each) for k in range(cores)]
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_moments, [(g1, g2, J, SEED, 0, 1)] * cores))  # start the workers
        t3 = time.perf_counter()
        acc = (0, 0.0, 0.0)
        for part in ex.map(_oracle_moments, jobs):
            acc = oracle.merge_moments(acc, part)
        sig = oracle.sigma_from_moments(acc[0], acc[2])
        snr = oracle.snr_planes(planes, sig)
        oracle.count_peaks_planes(snr, THRESH)
        t_all = time.perf_counter() - t3
    total = t_sig + t_all
    return {"value": (1 + r_all) * N * N * J / total / 1e6, "unit": "Mpix·scales/s",
            "cores": cores, "kind": "oracle",
            "sample": "the 1024x1024 map: KS + starlet (J=7) of the signal (one core, %.1f s) and "
                      "%d noise realisations with sigma, S/N and peaks spread over %d worker "
                      "processes (%d each, %.1f s)" % (t_sig, r_all, cores, each, t_all),
            "cpu": cpu_model(), "single_core": single}


def _gen_map(args):
    """One synthetic shear map (bench set-up, worker process)."""
    import numpy as np

    import synth
    n, grf_seed, noise_seed = args
    _, g1, g2 = synth.shear_map(n, grf_seed, noise_seed)
    return np.asarray(g1, dtype=np.float32), np.asarray(g2, dtype=np.float32)


GEN_WORKERS = 16


def generate_maps(specs):
    """synth.shear_map for each (n, grf_seed, noise_seed), spread over up to
    GEN_WORKERS worker processes (1: in this process); float32 arrays in the
    order given."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(GEN_WORKERS, cores, len(specs)))
    if cores == 1:
        return [_gen_map(sp) for sp in specs]
    # largest first, so the pool ends together
    order = sorted(range(len(specs)), key=lambda i: -specs[i][0])
    out = [None] * len(specs)
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        for i, res in zip(order, ex.map(_gen_map, [specs[i] for i in order], chunksize=4)):
            out[i] = res
    return out


def uneven_batch(ctx, reps):
    """The uneven batch: 512 float32 maps, sides drawn from {128..2048}
    (weights 4:4:3:2:1, seed 31), J = log2 N - 2, KS + starlet per map, as
    one grouped graph-captured plan and as one launch sequence per map.
    Every map is its own synthetic field (seeds 1000 + i and 5000 + i), so
    the 2.2 GB of inputs come from HBM, not from the 256 MB last-level
    cache; every job has its own output planes."""
    import torch

    import synth
    import paper_1204_4293_amd as amap

    dev = torch.device("cuda", 0)
    sides = synth.uneven_batch_sides(512, 31)
    maps = generate_maps([(n, 1000 + i, 5000 + i) for i, n in enumerate(sides)])
    jobs = []
    units = 0.0
    b_alg = 0.0
    for i, n in enumerate(sides):
        J = n.bit_length() - 1 - 2
        g1, g2 = maps[i]
        jobs.append({"g1": torch.from_numpy(g1).to(dev), "g2": torch.from_numpy(g2).to(dev),
                     "planes": torch.empty((J, n, n), dtype=torch.float32, device=dev)})
        units += n * n * J
        b_alg += n * n * (8.0 + 4.0 * J)
    del maps
    plan = amap.BatchPlan(ctx, jobs)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan.run()  # captures the graph
        plan.run()
    side.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(side):
        e0.record()
        for _ in range(reps):
            plan.run()
        e1.record()
    side.synchronize()
    t_batched = e0.elapsed_time(e1) / reps * 1e-3

    def plain_pass():
        for j in jobs:
            k, _ = ctx.ks_invert(j["g1"], j["g2"])
            ctx.starlet_forward(k, j["planes"].shape[0], planes=j["planes"])

    plain_pass()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(max(1, reps // 2)):
        plain_pass()
    e1.record()
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / max(1, reps // 2) * 1e-3
    plan.close()
    meas = profile_line(BATCHED_PROFILE, "batched-bytes-per-run")
    counts = {str(n): sides.count(n) for n in sorted(set(sides))}
    return {"workload": "512 distinct float32 maps (seeds 1000+i), sides %s, J = log2 N - 2, "
                        "KS + starlet" % counts,
            "value": units / t_batched / 1e6, "unit": "Mpix·scales/s", "ms_per_batch": t_batched * 1e3,
            "hbm_alg_GBps": b_alg / t_batched / 1e9,
            "hbm_alg_frac": b_alg / t_batched / (HBM_PEAK_GBS * 1e9),
            "hbm_meas_bytes": meas,
            "hbm_meas_frac": meas / t_batched / (HBM_PEAK_GBS * 1e9) if meas else None,
            "bytes_alg": b_alg,
            "plain": {"value": units / t_plain / 1e6, "ms_per_batch": t_plain * 1e3,
                      "hbm_alg_frac": b_alg / t_plain / (HBM_PEAK_GBS * 1e9)}}


def served_stream(ctx, requests):
    """The served stream: Poisson arrivals of float32 maps with sides
    log-uniform over 256..4096 (seeds 41, 42), J = min(9, log2 N - 2), 32 noise
    realisations each (noise seed 6000 + id), through the library's request
    loop (footprint admission, 8 concurrent slots).  Inputs come from a
    device-resident pool of eight generated maps per side; outputs come from
    a fixed set of buffers per side (requests wait for one on the client
    side, inside their latency).  First a burst gives the saturated request
    rate mu, then the stream runs ``requests`` requests at each of 0.25,
    0.5 and 0.8 mu; latency is arrival -> completion seen by polling."""
    import numpy as np
    import torch

    import synth
    import paper_1204_4293_amd as amap

    dev = torch.device("cuda", 0)
    R = 32
    sizes = (256, 512, 1024, 2048, 4096)
    specs = [(n, 7000 + 8 * n + k, 9000 + 8 * n + k) for n in sizes for k in range(8)]
    maps = generate_maps(specs)
    pool = {n: [] for n in sizes}
    for (n, _, _), (g1, g2) in zip(specs, maps):
        pool[n].append((torch.from_numpy(g1).to(dev), torch.from_numpy(g2).to(dev)))
    del maps
    srv = amap.Server(ctx, torch.float32, mem_budget=48 << 30, max_inflight=8, max_queued=100000)
    # output buffers: a fixed set per side, reused; a request waits on the
    # client side (inside its latency) until a set of its side is free
    depth = {256: 16, 512: 16, 1024: 12, 2048: 8, 4096: 6}
    free = {}
    for n, dpt in depth.items():
        J = min(9, n.bit_length() - 1 - 2)
        free[n] = [{"planes": torch.empty((J, n, n), device=dev),
                    "sigma": torch.empty((J - 1, n, n), device=dev),
                    "snr": torch.empty((J - 1, n, n), device=dev),
                    "peaks": torch.empty(J - 1, dtype=torch.int64, device=dev)} for _ in range(dpt)]

    def run(times, sides):
        t0 = time.perf_counter()
        pending, lat, units, i, done_at = {}, [], 0.0, 0, t0
        backlog = []
        while i < len(times) or backlog or pending:
            now = time.perf_counter()
            while i < len(times) and t0 + times[i] <= now:
                backlog.append(i)
                i += 1
            while backlog and free[sides[backlog[0]]]:
                k = backlog.pop(0)
                n = sides[k]
                J = min(9, n.bit_length() - 1 - 2)
                outs = free[n].pop()
                g1, g2 = pool[n][k % 8]
                job = dict(outs, g1=g1, g2=g2, n_real=R, seed=6000 + k, threshold=3.0)
                pending[srv.submit(job)] = (t0 + times[k], (1 + R) * n * n * J, n, outs)
            fin = srv.completed()
            if fin:
                done_at = time.perf_counter()
            for t in fin:
                arr, u, n, outs = pending.pop(t)
                free[n].append(outs)
                lat.append(done_at - arr)
                units += u
        span = done_at - t0
        lat = np.array(lat) * 1e3
        return {"requests": len(times), "seconds": span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "maps_per_s": len(times) / span,
                "value": units / span / 1e6, "unit": "Mpix·scales/s"}

    # warm up every size once, then the saturated burst
    run(np.zeros(5), list(sizes))
    _, sides = synth.served_stream(96, 1.0)
    burst = run(np.zeros(96), sides)
    mu = burst["maps_per_s"]
    out = {"workload": "Poisson arrivals, float32 sides log-uniform 256..4096, J = min(9, log2 N - 2), "
                       "R = 32 per request, 8 slots, footprint admission, 8 input maps per side",
           "saturated": burst, "levels": {}}
    for frac in (0.25, 0.5, 0.8):
        qps = frac * mu
        times, sides = synth.served_stream(requests, qps)
        out["levels"]["%.2f_mu" % frac] = dict(run(times, sides), qps=qps)
        print("bench: served %.2f mu done" % frac, file=sys.stderr, flush=True)
    srv.close()
    return out


def profile_workload(ctx, which, t1, t2):
    """The fixed workloads of --profile (for counter runs): no timing."""
    import torch

    import synth
    import paper_1204_4293_amd as amap
    dev = t1.device
    if which == "plain":
        ke = torch.empty_like(t1)
        pl = torch.empty((J, N, N), dtype=torch.float32, device=dev)
        for _ in range(10):
            ctx.ks_invert(t1, t2, kappa_e=ke)
            ctx.starlet_forward(ke, J, planes=pl)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "plain", "maps": 10, "n": N, "J": J}), flush=True)
        return 0
    sides = synth.uneven_batch_sides(512, 31)
    maps = generate_maps([(n, 1000 + i, 5000 + i) for i, n in enumerate(sides)])
    jobs = []
    for i, n in enumerate(sides):
        g1, g2 = maps[i]
        jobs.append({"g1": torch.from_numpy(g1).to(dev), "g2": torch.from_numpy(g2).to(dev),
                     "planes": torch.empty((n.bit_length() - 3, n, n), dtype=torch.float32, device=dev)})
    del maps
    plan = amap.BatchPlan(ctx, jobs)  # one direct run at creation
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan.run()  # capture, launch
        plan.run()
    side.synchronize()
    plan.close()
    print(json.dumps({"profile": "batched", "maps": len(jobs), "runs": 3}), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle's timed sample (0 to skip)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the uneven-batch and served-stream measurements (profiler runs)")
    ap.add_argument("--profile", choices=("plain", "batched"), default=None,
                    help="only run a fixed workload for a profiler's counters: 'plain' = 10 "
                         "single-map KS + starlet (J=7) sequences on the 1024^2 map, 'batched' = "
                         "the uneven batch's plan (one run at creation, two graph runs)")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes generating the batched and served inputs (1: none; for "
                         "profiler runs, whose preload would follow the workers)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests at each load level of the served stream (0 skips the stream)")
    ap.add_argument("--schedules", default=os.path.join(ROOT, "profiles", SCHEDULES),
                    help="JSON of tile schedules to load (amap_plans_load) instead of tuning; "
                         "'none' tunes live")
    ap.add_argument("--save-schedules", default=None,
                    help="write the context's schedules (amap_plans_read) to this file at the end")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    global GEN_WORKERS
    GEN_WORKERS = max(1, args.gen_workers)
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
    schedules_source = "tuned live"
    if args.schedules and args.schedules != "none" and os.path.exists(args.schedules):
        with open(args.schedules) as f:
            ctx.plans_load(f.read())
        schedules_source = os.path.relpath(args.schedules, ROOT)
    if args.profile:
        return profile_workload(ctx, args.profile, t1, t2)
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

    # per-kernel table: HIP events around every launch, over K untimed steps
    ctx.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ktimes = ctx.timing_read(reset=True)
    B = amap.noise_batch(N, R_REAL)
    kernels = {}
    for name, (launches, tot_ms) in sorted(ktimes.items(), key=lambda kv: -kv[1][1]):
        kernels[name] = {"launches_per_step": launches / args.steps,
                         "avg_us": 1e3 * tot_ms / launches,
                         "ms_per_step": tot_ms / args.steps}
    dom = max(ktimes.items(), key=lambda kv: kv[1][1])[0]
    starts = [int(k.rsplit("_j", 1)[1]) for k in ktimes if k.startswith("noise_stage_j")]

    # timed region: K whole steps; only the dominant kernel carries HIP
    # events (on its own launch stream), for its live average duration
    ctx.timing_select(dom)
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
    live = ctx.timing_read(reset=True)
    ctx.timing_enable(False)
    print("bench: timed %d steps, %.3f ms/step" % (args.steps, ms_per_step), file=sys.stderr,
          flush=True)

    dom_avg_s = live[dom][1] / live[dom][0] * 1e-3
    b_alg, f_alg = kernel_model(dom, N, J, B, starts)
    step_flops = 0.0
    loop_traffic = 0.0
    loop_complete = True
    for name, rec in kernels.items():
        bb, ff = kernel_model(name, N, J, B, starts)
        if bb is not None:
            rec["design_GBps"] = bb / (rec["avg_us"] * 1e-6) / 1e9
            rec["alg_TFLOPs"] = ff / (rec["avg_us"] * 1e-6) / 1e12
            step_flops += ff * rec["launches_per_step"]
        rl = roofline_of(name, N, J, B, starts, rec["avg_us"] * 1e-6)
        if rl:
            rec["bound"] = rl["bound"]
            rec["frac"] = rl["frac"]
        tb = measured_traffic(name)
        if tb is not None:
            rec["hbm_meas_GBps"] = tb / (rec["avg_us"] * 1e-6) / 1e9
        if name in NOISE_KERNELS or name.startswith("noise_stage_j"):
            if tb is None:
                loop_complete = False
            else:
                loop_traffic += tb * rec["launches_per_step"]
    traffic = measured_traffic(dom)
    roofline = {"kernel": dom}
    roofline.update(roofline_of(dom, N, J, B, starts, dom_avg_s))
    roofline.update({
        "traffic": traffic,
        "flops_per_launch": f_alg, "avg_launch_us": dom_avg_s * 1e6,
        "launches_timed": live[dom][0],
        # the kernel's own hand-offs (c planes, float64 accumulators) and the
        # counters' HBM bytes beside them: the kernel is not bound by them,
        # the ratio shows the re-reads of its tile halos
        "design_bytes_per_launch": b_alg,
        "hbm_meas_GBps": traffic / dom_avg_s / 1e9 if traffic else None,
        "hbm_meas_frac": traffic / dom_avg_s / (HBM_PEAK_GBS * 1e9) if traffic else None,
        "traffic_over_design_bytes": traffic / b_alg if (traffic and b_alg) else None,
    })
    # the whole step's algorithmic flops per second, and the counters' HBM
    # bytes of the noise loop's kernels (everything but the signal's one-map
    # kernels, finalize and peak count: ~2% of the step) per step
    step = {"alg_TFLOPs": step_flops / (ms_per_step * 1e-3) / 1e12,
            "alg_flops": step_flops,
            "frac_fp32": step_flops / (ms_per_step * 1e-3) / (FP32_PEAK_TFLOPS * 1e12),
            "noise_loop_hbm_meas_bytes": loop_traffic if loop_complete else None,
            "noise_loop_hbm_meas_frac": (loop_traffic / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9)
                                         if loop_complete else None)}

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
    meas = profile_line(PLAIN_PROFILE, "plain-bytes-per-map")
    plain["hbm_meas_bytes"] = meas
    plain["hbm_meas_frac"] = meas / (plain_ms * 1e-3) / (HBM_PEAK_GBS * 1e9) if meas else None

    # direct aperture mass vs the starlet on the 1024^2 map: map_direct at
    # theta = 2..64 px with the starlet filter truncated at cut = theta, vs
    # KS + starlet with J = log2(theta) + 1 planes (all scales up to theta)
    direct = {}
    for theta in (2, 4, 8, 16, 32, 64):
        Jt = theta.bit_length()
        dm = torch.empty((N, N), dtype=torch.float32, device=dev)
        pt = torch.empty((Jt, N, N), dtype=torch.float32, device=dev)
        ctx.map_direct(t1, t2, float(theta), amap.FILTER_STARLET, 0.0, float(theta), out=dm)
        ctx.starlet_forward(ctx.ks_invert(t1, t2, kappa_e=ke)[0], Jt, planes=pt)
        torch.cuda.synchronize()
        reps = 5 if theta >= 32 else 20
        ev0.record()
        for _ in range(reps):
            ctx.map_direct(t1, t2, float(theta), amap.FILTER_STARLET, 0.0, float(theta), out=dm)
        ev1.record()
        torch.cuda.synchronize()
        t_dir = ev0.elapsed_time(ev1) / reps
        ev0.record()
        for _ in range(20):
            ctx.ks_invert(t1, t2, kappa_e=ke)
            ctx.starlet_forward(ke, Jt, planes=pt)
        ev1.record()
        torch.cuda.synchronize()
        t_sw = ev0.elapsed_time(ev1) / 20
        # the filter's natural support (cut = 2 theta for the starlet Q)
        ctx.map_direct(t1, t2, float(theta), amap.FILTER_STARLET, 0.0, 0.0, out=dm)
        torch.cuda.synchronize()
        reps2 = 3 if theta >= 32 else 20
        ev0.record()
        for _ in range(reps2):
            ctx.map_direct(t1, t2, float(theta), amap.FILTER_STARLET, 0.0, 0.0, out=dm)
        ev1.record()
        torch.cuda.synchronize()
        t_dir2 = ev0.elapsed_time(ev1) / reps2
        direct["theta_%d" % theta] = {"J": Jt, "map_direct_ms": t_dir, "ks_starlet_ms": t_sw,
                                      "speedup": t_dir / t_sw, "map_direct_cut_2theta_ms": t_dir2,
                                      "speedup_cut_2theta": t_dir2 / t_sw}

    # the small double-precision case: one 256^2 FP64 map (GRF seed 1, shape
    # noise seed 2), KS + starlet J = 5 per call, and map_direct at theta =
    # 2, 4, 8 (the starlet Q's natural support, cut = 2 theta), latency per
    # map on an idle GPU
    _, s1, s2 = synth.shear_map(256, 1, 2)
    d1 = torch.tensor(s1, dtype=torch.float64, device=dev)
    d2 = torch.tensor(s2, dtype=torch.float64, device=dev)
    dke = torch.empty((256, 256), dtype=torch.float64, device=dev)
    dpl = torch.empty((5, 256, 256), dtype=torch.float64, device=dev)
    ddm = torch.empty((256, 256), dtype=torch.float64, device=dev)

    def small_once():
        ctx.ks_invert(d1, d2, kappa_e=dke)
        ctx.starlet_forward(dke, 5, planes=dpl)
    small_once()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(50):
        small_once()
    ev1.record()
    torch.cuda.synchronize()
    small = {"workload": "256x256 float64 map (GRF seed 1, noise seed 2), KS + starlet J=5",
             "ms_per_map": ev0.elapsed_time(ev1) / 50, "map_direct_ms": {}}
    for theta in (2, 4, 8):
        ctx.map_direct(d1, d2, float(theta), amap.FILTER_STARLET, 0.0, 0.0, out=ddm)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(20):
            ctx.map_direct(d1, d2, float(theta), amap.FILTER_STARLET, 0.0, 0.0, out=ddm)
        ev1.record()
        torch.cuda.synchronize()
        small["map_direct_ms"]["theta_%d" % theta] = ev0.elapsed_time(ev1) / 20

    # statistics of the step's planes: central moments of the J planes and
    # the peak-height histogram of the S/N planes, 20 calls each
    mom = torch.empty((J, 4), dtype=torch.float64, device=dev)
    hist = torch.empty((J - 1, 40), dtype=torch.int64, device=dev)
    stats = {}
    for name, fn, nbytes in (
            ("plane_moments", lambda: ctx.plane_moments(out["planes"], out=mom), 4.0 * J * N * N),
            ("peak_histogram", lambda: ctx.peak_histogram(out["snr"], -2.0, 8.0, 40, 1, hist=hist),
             4.0 * (J - 1) * N * N)):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(20):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) / 20 * 1e3
        stats[name] = {"us_per_call": us, "alg_bytes": nbytes, "alg_GBps": nbytes / us / 1e3,
                       "hbm_alg_frac": nbytes / us / 1e3 / HBM_PEAK_GBS}

    # a field with edges and a side that is not a power of two: the map's
    # 1000 x 1000 corner, KS zero-extended into 2048^2, starlet J = 7 under
    # the mirror rule
    NB, PB = 1000, 2048
    b1, b2 = t1[:NB, :NB].contiguous(), t2[:NB, :NB].contiguous()
    bk = torch.empty((NB, NB), dtype=torch.float32, device=dev)
    bpl = torch.empty((J, NB, NB), dtype=torch.float32, device=dev)

    def bounded_once():
        ctx.ks_invert_padded(b1, b2, PB, kappa_e=bk)
        ctx.starlet_forward_bc(bk, J, amap.BC_MIRROR, planes=bpl)
    bounded_once()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(20):
        bounded_once()
    ev1.record()
    torch.cuda.synchronize()
    t_b = ev0.elapsed_time(ev1) / 20
    RB_REAL = 16
    bpk = torch.empty(J - 1, dtype=torch.int64, device=dev)

    def bounded_noise():
        _, snr_b = ctx.noise_maps_bc(b1, b2, PB, J, amap.BC_MIRROR, RB_REAL, 7, planes_signal=bpl)
        ctx.count_peaks_bc(snr_b, 3.0, amap.BC_MIRROR, counts=bpk)
    bounded_noise()
    torch.cuda.synchronize()
    ev0.record()
    bounded_noise()
    ev1.record()
    torch.cuda.synchronize()
    t_bn = ev0.elapsed_time(ev1)
    bounded = {"workload": "1000x1000 float32 field (corner of the step's map), KS zero-extended "
                           "into 2048x2048, starlet J=7, mirror edges",
               "ms_per_map": t_b, "value": NB * NB * J / (t_b * 1e3), "unit": "Mpix·scales/s",
               "noise": {"n_real": RB_REAL, "ms": t_bn, "ms_per_realisation": t_bn / RB_REAL,
                         "value": (1 + RB_REAL) * NB * NB * J / ((t_b + t_bn) * 1e3),
                         "unit": "Mpix·scales/s", "what": "sigma, S/N and peaks (S/N > 3), signal "
                                                          "pass included in value"}}

    batched = served = None
    if not args.no_batched:
        print("bench: uneven batch", file=sys.stderr, flush=True)
        batched = uneven_batch(ctx, max(2, args.steps))
        if args.serve_requests > 0:
            print("bench: served stream", file=sys.stderr, flush=True)
            served = served_stream(ctx, args.serve_requests)

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
        # the job's compulsory HBM bytes (shear in; planes, sigma and S/N out:
        # the realisations never leave the device) per step, as a fraction
        # of HBM peak: the path is nowhere near bound by its inputs and outputs
        "compulsory_hbm_frac": (N * N * (8 + 4 * J) + 8 * (J - 1) * N * N) / (ms_per_step * 1e-3)
                               / (HBM_PEAK_GBS * 1e9),
        "plain": plain, "batched": batched, "served": served, "statistics": stats,
        "direct_vs_starlet": direct,
        "small_fp64": small,
        "bounded": bounded,
        "roofline": roofline,
        "step": step,
        "kernels": kernels,
        # tile schedules the autotuner chose for this run: [j0, scales, tile
        # width, tile sub-rows, realisations per LDS pass] per stage
        "schedules": ctx.plans(),
        "schedules_source": schedules_source,
    }
    if args.save_schedules:
        with open(args.save_schedules, "w") as f:
            json.dump(ctx.plans(), f)
    ctx.close()
    if args.cpu_seconds > 0:
        print("bench: cpu baseline (oracle, ~%.0f s)" % args.cpu_seconds, file=sys.stderr,
              flush=True)
        line["cpu_baseline"] = cpu_baseline(np.asarray(g1), np.asarray(g2), args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Batch plans (grouped maps of uneven sizes, graph-captured) against the
single-map calls and the FP64 oracle.

Grouped maps run the same kernels as single maps, so their outputs are
compared bit for bit with the single-map path; sampled maps are also
checked against the oracle at 1e-5 * rms(kappa) (float32) or 1e-10
(float64), and every map of the uneven batch against the reconstruction
identity kappa = c_{J-1} + sum_j w_j, which holds at any size.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-10}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = amap.Context(0)
    yield c
    c.close()


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.double().cpu().numpy()


def rms(a):
    return float(np.sqrt(np.mean(np.asarray(a, dtype=np.float64) ** 2)))


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))))


def make_jobs(sides, dtype, seed0, want_kappa):
    jobs, refs = [], []
    for i, n in enumerate(sides):
        J = max(2, n.bit_length() - 1 - 2)
        _, g1, g2 = S.shear_map(n, seed0 + i, seed0 + 500 + i)
        job = {"g1": dev(g1, dtype), "g2": dev(g2, dtype),
               "planes": torch.full((J, n, n), float("nan"), dtype=dtype, device="cuda")}
        if want_kappa(i):
            job["kappa_e"] = torch.full((n, n), float("nan"), dtype=dtype, device="cuda")
        jobs.append(job)
        refs.append((g1, g2, J))
    return jobs, refs


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_grouped_plan_replays_match_single_maps_and_oracle(ctx, dtype):
    sides = [64, 128, 64, 256, 128, 64, 32, 256]
    print("grouped plan %s sides=%s" % (dtype, sides), flush=True)
    jobs, refs = make_jobs(sides, dtype, 200, lambda i: i % 3 == 0)
    plan = amap.BatchPlan(ctx, jobs)
    side = torch.cuda.Stream()
    single = []
    for (g1, g2, J), job in zip(refs, jobs):
        k, _ = ctx.ks_invert(job["g1"], job["g2"])
        single.append((k, ctx.starlet_forward(k, J)))
    torch.cuda.synchronize()
    first = None
    for rep in range(3):
        with torch.cuda.stream(side):
            plan.run()       # the first run captures the graph, later runs replay it
        side.synchronize()
        # eager work of the program between replays
        ctx.ks_invert(jobs[0]["g1"], jobs[0]["g2"])
        torch.cuda.synchronize()
        outs = [j["planes"].clone() for j in jobs]
        if first is None:
            first = outs
        for i, (job, (k1, p1)) in enumerate(zip(jobs, single)):
            assert torch.equal(outs[i], first[i]), "replay %d map %d differs" % (rep, i)
            assert torch.equal(outs[i], p1), "map %d differs from the single-map path" % i
            if "kappa_e" in job:
                assert torch.equal(job["kappa_e"], k1)
        for j in jobs:
            j["planes"].fill_(float("nan"))
    # oracle on every map (small sizes)
    with torch.cuda.stream(side):
        plan.run()
    side.synchronize()
    for (g1, g2, J), job in zip(refs, jobs):
        kE, _ = O.ks_invert(g1, g2)
        ref = O.starlet_forward(kE, J)
        assert maxerr(host(job["planes"]), ref) <= TOL[dtype] * rms(kE)
    plan.close()


def test_plan_with_noise_job_matches_run_path(ctx):
    n, J, R, seed = 64, 4, 6, 77
    jobs, refs = make_jobs([64, 64, 128], torch.float32, 300, lambda i: False)
    _, g1, g2 = S.shear_map(n, 310, 311)
    t1, t2 = dev(g1, torch.float32), dev(g2, torch.float32)
    noise_job = {"g1": t1, "g2": t2, "n_real": R, "seed": seed, "threshold": 2.0,
                 "planes": torch.empty((J, n, n), device="cuda"),
                 "sigma": torch.empty((J - 1, n, n), device="cuda"),
                 "snr": torch.empty((J - 1, n, n), device="cuda"),
                 "peaks": torch.zeros(J - 1, dtype=torch.int64, device="cuda")}
    plan = amap.BatchPlan(ctx, jobs + [noise_job])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan.run()
    side.synchronize()
    ref = ctx.run_path(t1, t2, J, R, seed, 2.0)
    torch.cuda.synchronize()
    for key in ("planes", "sigma", "snr", "peaks"):
        assert torch.equal(noise_job[key], ref[key]), key
    for (g1, g2, J), job in zip(refs, jobs):
        kE, _ = O.ks_invert(g1, g2)
        assert maxerr(host(job["planes"]), O.starlet_forward(kE, J)) <= 1e-5 * rms(kE)
    plan.close()


def noise_job(n, J, R, seed, s1, s2, dtype=torch.float32):
    _, g1, g2 = S.shear_map(n, s1, s2)
    return {"g1": dev(g1, dtype), "g2": dev(g2, dtype), "n_real": R, "seed": seed, "threshold": 2.0,
            "planes": torch.empty((J, n, n), dtype=dtype, device="cuda"),
            "sigma": torch.empty((J - 1, n, n), dtype=dtype, device="cuda"),
            "snr": torch.empty((J - 1, n, n), dtype=dtype, device="cuda"),
            "peaks": torch.zeros(J - 1, dtype=torch.int64, device="cuda")}


def test_plan_noise_jobs_as_graph_branches(ctx):
    # noise jobs of a plan run on up to four lanes, forked from and joined
    # back into the caller's stream inside the captured graph; every replay
    # (eager work and synchronisations between them, outputs poisoned before
    # each) equals run_path job by job, and the grouped maps still match
    # the oracle
    specs = [(64, 4, 5, 11), (128, 5, 9, 12), (256, 6, 4, 13), (128, 5, 3, 14), (64, 3, 6, 15),
             (512, 7, 4, 16), (32, 3, 2, 17)]
    njobs = [noise_job(n, J, R, seed, 400 + k, 600 + k) for k, (n, J, R, seed) in enumerate(specs)]
    gjobs, refs = make_jobs([64, 128, 128, 256], torch.float32, 700, lambda i: i % 2 == 0)
    refs_path = []
    for (n, J, R, seed), j in zip(specs, njobs):
        refs_path.append(ctx.run_path(j["g1"], j["g2"], J, R, seed, 2.0))
    torch.cuda.synchronize()
    plan = amap.BatchPlan(ctx, gjobs[:2] + njobs[:4] + gjobs[2:] + njobs[4:])
    side = torch.cuda.Stream()
    scratch = torch.zeros((256, 256), device="cuda")
    for replay in range(4):
        for j in njobs:
            for key in ("planes", "sigma", "snr"):
                j[key].fill_(float("nan"))
            j["peaks"].fill_(-1)
        for j in gjobs:
            j["planes"].fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            plan.run()
        side.synchronize()
        for k, (j, ref) in enumerate(zip(njobs, refs_path)):
            for key in ("planes", "sigma", "snr", "peaks"):
                assert torch.equal(j[key], ref[key]), (replay, k, key)
        for (g1, g2, J), job in zip(refs, gjobs):
            kE, _ = O.ks_invert(g1, g2)
            assert maxerr(host(job["planes"]), O.starlet_forward(kE, J)) <= 1e-5 * rms(kE)
        # eager work of the program's own between replays
        ctx.ks_invert(njobs[2]["g1"], njobs[2]["g2"], kappa_e=scratch)
        scratch.mul_(2.0)
        torch.cuda.synchronize()
    # the direct path (null stream) runs the lanes one after another
    for j in njobs:
        j["sigma"].fill_(float("nan"))
    plan.run_on(None)
    torch.cuda.synchronize()
    for j, ref in zip(njobs, refs_path):
        assert torch.equal(j["sigma"], ref["sigma"])
    plan.close()


def test_uneven_batch_sampled_against_oracle(ctx):
    # the uneven-batch size distribution (sides 128..2048, weights 4:4:3:2:1),
    # first 40 draws; per-map seeds 1000 + i; J = log2 N - 2
    sides = S.uneven_batch_sides(40, 31)
    assert 2048 in sides and 128 in sides
    print("uneven batch sides=%s" % sides, flush=True)
    jobs, refs = make_jobs(sides, torch.float32, 1000, lambda i: True)
    plan = amap.BatchPlan(ctx, jobs)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan.run()
    side.synchronize()
    # every map: exact reconstruction and zero-mean detail planes
    for job in jobs:
        p = job["planes"].double()
        k = job["kappa_e"].double()
        r = float(k.pow(2).mean().sqrt())
        assert float((p.sum(0) - k).abs().max()) <= 1e-5 * r
        assert float(p[:-1].mean(dim=(1, 2)).abs().max()) <= 1e-6 * r
    # sampled maps: the first of each size against the oracle
    seen = set()
    for (g1, g2, J), job, n in zip(refs, jobs, sides):
        if n in seen:
            continue
        seen.add(n)
        kE, _ = O.ks_invert(g1, g2)
        tol = 1e-5 * rms(kE)
        assert maxerr(host(job["kappa_e"]), kE) <= tol
        assert maxerr(host(job["planes"]), O.starlet_forward(kE, J)) <= tol
    plan.close()


def test_plan_rejects_bad_jobs(ctx):
    g = torch.zeros((64, 64), device="cuda")
    with pytest.raises(amap.AmapError):
        amap.BatchPlan(ctx, [{"g1": g, "g2": g, "planes": torch.empty((7, 64, 64), device="cuda")}])
    with pytest.raises(amap.AmapError):
        amap.BatchPlan(ctx, [{"g1": g, "g2": g, "n_real": 1,
                              "planes": torch.empty((3, 64, 64), device="cuda")}])


@pytest.mark.parametrize("n,J", [(256, 6), (1024, 7), (2048, 9)])
def test_autotuned_schedule_matches_analytic(ctx, n, J):
    # tiles and stage splits change only the order of independent work:
    # the starlet planes are bit-identical, noise statistics agree to rounding
    print("autotune vs analytic n=%d J=%d" % (n, J), flush=True)
    plain = amap.Context(0)
    plain.set_autotune(False)
    kappa = S.grf_kappa(n, 60 + J)
    k = dev(kappa, torch.float32)
    a = ctx.starlet_forward(k, J)
    b = plain.starlet_forward(k, J)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    if n <= 1024:
        _, g1, g2 = S.shear_map(n, 70 + J, 71 + J)
        t1, t2 = dev(g1, torch.float32), dev(g2, torch.float32)
        sa, _ = ctx.noise_maps(t1, t2, J, 40, 9, want_snr=False)
        sb, _ = plain.noise_maps(t1, t2, J, 40, 9, want_snr=False)
        torch.cuda.synchronize()
        assert float((sa.double() - sb.double()).abs().max()) <= 1e-6 * float(sb.double().abs().max())
    plain.close()


def test_schedules_round_trip_and_validation(ctx):
    # schedules read from one context and loaded into another reproduce its
    # results bit for bit; invalid schedules are refused and load nothing
    n, J, R, seed = 256, 6, 12, 5
    _, g1, g2 = S.shear_map(n, 61, 62)
    t1, t2 = dev(g1, torch.float32), dev(g2, torch.float32)
    sa, _ = ctx.noise_maps(t1, t2, J, R, seed, want_snr=False)
    plans = [p for p in ctx.plans() if p["logn"] == 8 and p["J"] == J]
    assert plans and any(p["noise"] for p in plans)
    other = amap.Context(0)
    other.plans_load(plans)
    got = [p for p in other.plans() if p["logn"] == 8 and p["J"] == J]
    assert sorted(map(str, got)) == sorted(map(str, plans))
    sb, _ = other.noise_maps(t1, t2, J, R, seed, want_snr=False)
    torch.cuda.synchronize()
    assert torch.equal(sa, sb)
    before = other.plans()
    bad = [dict(plans[0]), ]
    bad[0]["stages"] = [list(st) for st in plans[0]["stages"]]
    bad[0]["stages"][0][2] = 48                      # no such tile width
    for broken in (bad, '[{"mode": 1, "elem": 4}]', '[{"mode": 1, "elem": 4, "logn": 8, "J": 6, '
                   '"noise": 1, "batch": 12, "stages": [[1, 2, 64, 32, 1, 0], [4, 2, 64, 32, 1, 0]]}]'):
        with pytest.raises(amap.AmapError):
            other.plans_load(broken)
    assert other.plans() == before
    other.close()


def test_run_path_calls_back_to_back_on_a_stream(ctx):
    # two calls queued back to back on a non-default stream, with no
    # synchronisation between them (the second reuses the context's
    # workspace), give each call's results bit for bit
    n, J, R = 256, 6, 8
    side = torch.cuda.Stream()
    maps = []
    for k in range(2):
        _, g1, g2 = S.shear_map(n, 900 + k, 950 + k)
        maps.append((dev(g1, torch.float32), dev(g2, torch.float32)))
    def kb():
        return {"kappa_b": torch.full((n, n), float("nan"), device="cuda")}
    alone = []
    for g1, g2 in maps:
        alone.append(ctx.run_path(g1, g2, J, R, 31, 2.5, out=kb()))
        torch.cuda.synchronize()
    with torch.cuda.stream(side):
        outs = [ctx.run_path(g1, g2, J, R, 31, 2.5, out=kb()) for g1, g2 in maps]
    side.synchronize()
    for got, ref in zip(outs, alone):
        for key in ("kappa_e", "kappa_b", "planes", "sigma", "snr", "peaks"):
            assert torch.equal(got[key], ref[key]), key

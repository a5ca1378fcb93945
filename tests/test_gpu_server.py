"""The request loop (amap_server_*): continuous batching of independent jobs.

A job's results must be the same alone and in the mix.  Each job's kernels
read only its own inputs and workspace, so the comparison is bit for bit
against the same job run alone on the default stream.  Admission respects
the memory budget, over-budget jobs are rejected and a full queue reports
busy.
"""
import numpy as np
import pytest
import torch

import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = amap.Context(0)
    yield c
    c.close()


def make_job(n, seed, n_real, dtype=torch.float32):
    J = max(2, min(9, n.bit_length() - 1 - 2))
    _, g1, g2 = S.shear_map(n, seed, seed + 1)
    job = {"g1": torch.tensor(g1, dtype=dtype, device="cuda"),
           "g2": torch.tensor(g2, dtype=dtype, device="cuda"),
           "planes": torch.full((J, n, n), float("nan"), dtype=dtype, device="cuda")}
    if n_real:
        job.update({"n_real": n_real, "seed": seed + 7, "threshold": 2.5,
                    "sigma": torch.full((J - 1, n, n), float("nan"), dtype=dtype, device="cuda"),
                    "snr": torch.full((J - 1, n, n), float("nan"), dtype=dtype, device="cuda"),
                    "peaks": torch.full((J - 1,), -1, dtype=torch.int64, device="cuda")})
    return job


def run_alone(ctx, job):
    J = job["planes"].shape[0]
    if job.get("n_real", 0):
        return ctx.run_path(job["g1"], job["g2"], J, job["n_real"], job["seed"], job["threshold"])
    k, _ = ctx.ks_invert(job["g1"], job["g2"])
    return {"planes": ctx.starlet_forward(k, J)}


def test_results_same_alone_and_in_the_mix(ctx):
    rng = np.random.default_rng(5)
    sides = [64, 128, 256, 512, 64, 256, 128, 512, 64, 128, 256, 64]
    jobs = [make_job(int(n), 100 + 3 * i, int(rng.choice([0, 4, 8]))) for i, n in enumerate(sides)]
    print("server mix: %s" % [(j["g1"].shape[0], j.get("n_real", 0)) for j in jobs], flush=True)
    # each job alone first (into buffers of its own): this also settles the
    # context's tile schedules, so that no admission in the mix stops to tune
    refs = [run_alone(ctx, j) for j in jobs]
    torch.cuda.synchronize()
    srv = amap.Server(ctx, mem_budget=1 << 30, max_inflight=4)
    # a few milliseconds of matrix products ahead on the submitting stream:
    # every job waits for its submit point, so the first ones are admitted
    # together and are on the device at once however fast each one runs
    m = torch.randn((4096, 4096), device="cuda") * 1e-2
    for _ in range(8):
        m = m @ m.clamp(-1.0, 1.0)
    tickets = [srv.submit(j) for j in jobs]
    saw_overlap = srv.stats()["inflight"] > 1
    pending = set(tickets)
    while pending:
        for t in list(pending):
            if srv.poll(t):
                pending.discard(t)
        saw_overlap = saw_overlap or srv.stats()["inflight"] > 1
    assert saw_overlap, "the mix never had two jobs on the device at once"
    srv.close()
    torch.cuda.synchronize()
    for j, ref in zip(jobs, refs):
        keys = ("planes", "sigma", "snr", "peaks") if j.get("n_real", 0) else ("planes",)
        for key in keys:
            assert torch.equal(j[key], ref[key]), "n=%d %s differs alone vs mix" % (
                j["g1"].shape[0], key)


def test_job_waits_for_its_submitting_stream(ctx):
    # the inputs are written on a side stream behind a long queue of work and
    # the job is submitted on that stream: it must see the written inputs,
    # not the zeros they held before
    job = make_job(256, 700, 8)
    src1, src2 = job["g1"].clone(), job["g2"].clone()
    job["g1"].zero_()
    job["g2"].zero_()
    a = torch.randn(2048, 2048, device="cuda")
    torch.cuda.synchronize()
    srv = amap.Server(ctx, mem_budget=1 << 30, max_inflight=2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for _ in range(40):
            a = torch.tanh(a @ a)  # keeps the stream busy for a while
        job["g1"].copy_(src1)
        job["g2"].copy_(src2)
        t = srv.submit(job)
    srv.wait(t)
    srv.close()
    torch.cuda.synchronize()
    ref = run_alone(ctx, job)
    torch.cuda.synchronize()
    for key in ("planes", "sigma", "snr", "peaks"):
        assert torch.equal(job[key], ref[key]), key


def test_admission_respects_the_budget(ctx):
    jobs = [make_job(256, 400 + i, 8) for i in range(4)]
    fp = amap.job_footprint_bytes(amap.F32, 256, jobs[0]["planes"].shape[0], 8)
    srv = amap.Server(ctx, mem_budget=fp + fp // 2, max_inflight=4)   # room for one at a time
    tickets = [srv.submit(j) for j in jobs]
    peak = srv.stats()["inflight"]
    while not all(srv.poll(t) for t in tickets):
        st = srv.stats()
        peak = max(peak, st["inflight"])
        assert st["mem_in_use"] <= fp + fp // 2
    assert peak == 1
    for j in jobs:
        ref = run_alone(ctx, j)
        torch.cuda.synchronize()
        assert torch.equal(j["sigma"], ref["sigma"])
    srv.close()


def test_over_budget_and_busy(ctx):
    job = make_job(128, 500, 4)
    srv = amap.Server(ctx, mem_budget=1024, max_inflight=2)
    with pytest.raises(amap.AmapError) as e:
        srv.submit(job)
    assert e.value.status == amap.E_NOMEM
    srv.close()
    # a one-slot, one-deep queue: the first job is admitted at once, the
    # second waits, the third finds the queue full (the first takes far
    # longer on the GPU than the two submit calls that follow it)
    small = [make_job(512, 600 + i, 8) for i in range(3)]
    srv = amap.Server(ctx, mem_budget=8 << 30, max_inflight=1, max_queued=1)
    t0 = srv.submit(small[0])
    t1 = srv.submit(small[1])
    busy = False
    try:
        srv.submit(small[2])
    except amap.AmapError as err:
        busy = err.status == amap.E_BUSY
    srv.wait(t0)
    srv.wait(t1)
    assert busy, "a third job was queued behind a full one-deep queue"
    srv.close()

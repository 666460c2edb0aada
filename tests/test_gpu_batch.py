"""Batched form: one persistent, graph-replayed launch over many uneven requests.

Each request's result must equal the single-request path bit for bit (same
device functions, same summation order), for graph replays with eager work in
between, for direct launches, and with invalid requests mixed in.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_17263_amd import scenes as S
from tests import parity as PT

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2211_17263_amd import native as NV
    ctx = NV.Context(0)
    jobs = S.batch_jobs(seed=44, n_jobs=10, max_side=128, max_tris=20000)
    scenes, refs = [], []
    for j in jobs:
        sc = NV.prdpt_scene_create(ctx, j["scene"])
        scenes.append(sc)
        refs.append(NV.prdpt_render_reference(sc, j["theta_ref"], 3))
    torch.cuda.synchronize()
    yield ctx, jobs, scenes, refs
    for sc in scenes:
        sc.destroy()
    ctx.close()


def _alone(NV, sc, ref, j, seed):
    return NV.prdpt_grad_estimate(sc, ref, j["theta0"], j["sigma"], j["N"], seed, j["est"])


def _batch(NV, ctx, jobs, scenes, refs, idx, seeds):
    reqs = [NV.BatchRequest(scenes[i], refs[i], jobs[i]["theta0"], jobs[i]["sigma"], jobs[i]["N"],
                            seeds[i], jobs[i]["est"]) for i in idx]
    NV.prdpt_batch_estimate(ctx, reqs)
    return reqs


@pytest.mark.parametrize("use_graph,bpc,tpi", [(True, 4, 2), (False, 4, 2), (True, 0, 1)])
def test_batch_equals_alone_bitwise(setup, use_graph, bpc, tpi):
    # bpc 0: the default, as many work-groups as the compute units hold at once
    import torch
    from paper_2211_17263_amd import native as NV
    ctx, jobs, scenes, refs = setup
    say("batch-vs-alone", "graph" if use_graph else "direct", bpc, tpi,
        [j["scene"].width for j in jobs])
    NV.prdpt_batch_config(ctx, bpc, tpi, use_graph)
    rng = np.random.default_rng(0)
    for rep in range(3):   # graph replays with eager single-request work in between
        idx = list(range(len(jobs))) if rep == 0 else sorted(rng.choice(len(jobs), 6, replace=False))
        seeds = {i: 1000 * rep + 17 * i + 1 for i in idx}
        reqs = _batch(NV, ctx, jobs, scenes, refs, idx, seeds)
        for i, q in zip(idx, reqs):
            a = _alone(NV, scenes[i], refs[i], jobs[i], seeds[i])
            torch.cuda.synchronize()
            assert q.status == 0
            d = scenes[i].d
            assert np.array_equal(q.grad[:d], a["grad"]), (rep, i)
            assert np.array_equal(q.losses[: jobs[i]["N"]], a["losses"]), (rep, i)
            assert q.loss[0] == a["loss"]


def test_batch_with_rotated_instances(setup):
    # a scene with a rotated, rotation-bound box next to scenes without
    # rotations: the batch takes the rotating variant of the render when any
    # request needs it (the captured graph is replaced when that changes), and
    # every request still equals its single-request result bit for bit
    import torch
    from paper_2211_17263_amd import native as NV
    ctx, jobs, scenes, refs = setup
    pr = S.cornell_problem(seed=2, rotation=True, width=48, height=40, spp=2, ico_level=2)
    say("batch-rotation")
    rs = NV.prdpt_scene_create(ctx, pr["scene"])
    try:
        rjob = dict(theta0=pr["theta0"], sigma=pr["sigma"], N=8, est=NV.PRDPT_EST_IS)
        js, ss = [jobs[0], jobs[1], rjob], [scenes[0], scenes[1], rs]
        rf = [refs[0], refs[1], NV.prdpt_render_reference(rs, pr["theta_ref"], 3)]
        NV.prdpt_batch_config(ctx, 4, 2, True)
        for rep, idx in enumerate([[2, 0], [0, 1], [1, 2], [2]]):
            seeds = {i: 500 * rep + 3 * i + 1 for i in idx}
            reqs = _batch(NV, ctx, js, ss, rf, idx, seeds)
            for i, q in zip(idx, reqs):
                a = _alone(NV, ss[i], rf[i], js[i], seeds[i])
                torch.cuda.synchronize()
                assert q.status == 0
                assert np.array_equal(q.grad[: ss[i].d], a["grad"]), (rep, i)
                assert np.array_equal(q.losses[: js[i]["N"]], a["losses"]), (rep, i)
    finally:
        rs.destroy()


def test_batch_with_many_samples(setup):
    # a scene with more samples per pixel than one chunk (the chunked render)
    # beside the setup's scenes, bit-equal to the single-request path
    import torch
    from paper_2211_17263_amd import native as NV
    ctx, jobs, scenes, refs = setup
    say("batch-two-chunks")
    sc = S.toy_scene(width=27, height=19, spp=80, bounces=1)
    gs = NV.prdpt_scene_create(ctx, sc)
    try:
        job = dict(theta0=np.array([0.2, -0.1], np.float32), sigma=np.full(2, 0.3, np.float32),
                   N=4, est=NV.PRDPT_EST_IS)
        js, ss = [job, jobs[0]], [gs, scenes[0]]
        rf = [NV.prdpt_render_reference(gs, np.zeros(2, np.float32), 3), refs[0]]
        NV.prdpt_batch_config(ctx, 4, 2, True)
        for rep in range(2):
            seeds = {0: 11 + rep, 1: 23 + rep}
            reqs = _batch(NV, ctx, js, ss, rf, [0, 1], seeds)
            for i, q in zip([0, 1], reqs):
                a = _alone(NV, ss[i], rf[i], js[i], seeds[i])
                torch.cuda.synchronize()
                assert q.status == 0
                assert np.array_equal(q.grad[: ss[i].d], a["grad"]), (rep, i)
                assert np.array_equal(q.losses[: js[i]["N"]], a["losses"]), (rep, i)
    finally:
        gs.destroy()


def test_batch_isolates_invalid_requests(setup):
    from paper_2211_17263_amd import native as NV
    ctx, jobs, scenes, refs = setup
    say("batch-invalid")
    NV.prdpt_batch_config(ctx, 4, 1, True)
    good = NV.BatchRequest(scenes[0], refs[0], jobs[0]["theta0"], jobs[0]["sigma"], jobs[0]["N"], 5,
                           jobs[0]["est"])
    odd = NV.BatchRequest(scenes[1], refs[1], jobs[1]["theta0"], jobs[1]["sigma"], 3, 5, jobs[1]["est"])
    bad_sigma = NV.BatchRequest(scenes[2], refs[2], jobs[2]["theta0"], np.zeros_like(jobs[2]["sigma"]),
                                jobs[2]["N"], 5, jobs[2]["est"])
    bad_est = NV.BatchRequest(scenes[3], refs[3], jobs[3]["theta0"], jobs[3]["sigma"], jobs[3]["N"], 5, 9)
    # a wide request (d = 150, 75 spheres) in the same batch is valid
    srt = S.sort_problem(width=16, height=16, spp=1)
    wide_sc = NV.prdpt_scene_create(ctx, srt["scene"])
    wide_ref = NV.prdpt_render_reference(wide_sc, srt["theta_ref"], 1)
    wide = NV.BatchRequest(wide_sc, wide_ref, srt["theta0"], srt["sigma"], 4, 5, 1)
    NV.prdpt_batch_estimate(ctx, [odd, good, bad_sigma, bad_est, wide])
    assert [r.status for r in (odd, good, bad_sigma, bad_est, wide)] == [
        NV.PRDPT_E_ARG, 0, NV.PRDPT_E_ARG, NV.PRDPT_E_ARG, 0]
    a = _alone(NV, scenes[0], refs[0], jobs[0], 5)
    assert np.array_equal(good.grad[: scenes[0].d], a["grad"])
    w = NV.prdpt_grad_estimate(wide_sc, wide_ref, srt["theta0"], srt["sigma"], 4, 5, 1)
    assert np.array_equal(wide.grad[:150], w["grad"]) and wide.loss[0] == w["loss"]
    wide_sc.destroy()


def test_batch_against_oracle(setup):
    import torch
    from paper_2211_17263_amd import native as NV
    ctx, jobs, scenes, refs = setup
    i = min(range(len(jobs)), key=lambda t: jobs[t]["scene"].width * jobs[t]["scene"].spp)
    j = jobs[i]
    say("batch-oracle", j["scene"].width, j["scene"].spp, j["N"])
    osc = O.OracleScene(j["scene"])
    ref = osc.reference(j["theta_ref"], seed=8)
    ref_d = torch.from_numpy(ref).cuda()
    q = NV.BatchRequest(scenes[i], ref_d, j["theta0"], j["sigma"], j["N"], 77, j["est"])
    NV.prdpt_batch_estimate(ctx, [q])
    o = osc.grad_estimate(ref, j["theta0"], j["sigma"], j["N"], 77, j["est"])
    _, c = O.draw_tau(j["est"], j["sigma"], j["N"] // 2, 77)
    PT.assert_losses_match(q.losses[: j["N"]], o["losses"], "batch")
    PT.assert_grad_match(q.grad[: scenes[i].d], o["grad"], c, o["losses"], "batch")


def test_autotune_writes_and_reads_cache(setup, tmp_path):
    from paper_2211_17263_amd import native as NV
    ctx, jobs, scenes, refs = setup
    say("autotune")
    reqs = [NV.BatchRequest(scenes[i], refs[i], jobs[i]["theta0"], jobs[i]["sigma"], jobs[i]["N"], 9,
                            jobs[i]["est"]) for i in range(len(jobs))]
    cache = str(tmp_path / "tune.jsonl")
    b, t, ms = NV.prdpt_batch_autotune(ctx, reqs, cache)
    assert b >= 1 and t >= 1 and ms > 0
    assert os.path.exists(cache) and '"blocks_per_cu": %d' % b in open(cache).read()
    b2, t2, ms2 = NV.prdpt_batch_autotune(ctx, reqs, cache)
    assert (b2, t2) == (b, t) and ms2 == pytest.approx(ms, rel=1e-6)
    NV.prdpt_batch_estimate(ctx, reqs)
    assert all(r.status == 0 for r in reqs)


def test_batch_large_scene_against_oracle():
    # a batched request on a scene of the batched workload's largest size
    # (512x512, about 120k triangles) beside a small one: losses and gradient
    # against the oracle's estimate
    import torch
    from paper_2211_17263_amd import native as NV
    rng = np.random.default_rng(61)
    cases = []
    for side, n_tris, N, est, d in ((512, 120000, 4, O.IS, 6), (64, 2000, 8, O.GAUSS, 3)):
        sc, fields = S.random_job_scene(rng, side, n_tris, 4, 2)
        for idx in rng.permutation(len(fields))[:d]:
            sc.bind(*fields[idx])
        cases.append((sc, N, est, d))
    ctx = NV.Context(0)
    try:
        reqs, want = [], []
        for k, (sc, N, est, d) in enumerate(cases):
            say("batch-large-oracle", sc.width, sc.n_tris, N)
            th_ref = np.zeros(d, np.float32)
            th0 = np.full(d, 0.1, np.float32)
            sg = np.full(d, 0.3, np.float32)
            osc = O.OracleScene(sc)
            ref = osc.reference(th_ref, seed=5 + k)
            gs = NV.prdpt_scene_create(ctx, sc)
            reqs.append((gs, NV.BatchRequest(gs, torch.from_numpy(ref).cuda(), th0, sg, N, 70 + k,
                                             est)))
            want.append((osc.grad_estimate(ref, th0, sg, N, 70 + k, est), sg, N, est))
        NV.prdpt_batch_estimate(ctx, [q for _, q in reqs])
        for (gs, q), (o, sg, N, est) in zip(reqs, want):
            assert q.status == 0
            _, c = O.draw_tau(est, sg, N // 2, q.seed)
            PT.assert_losses_match(q.losses[:N], o["losses"], "batch-large")
            PT.assert_grad_match(q.grad[: gs.d], o["grad"], c, o["losses"], "batch-large")
            gs.destroy()
    finally:
        ctx.close()

"""Continuous-batching server: results in the mix equal each request alone,
admission by HBM footprint with LRU eviction, cancellation, stats."""
import sys
import time

import numpy as np
import pytest

from paper_2211_17263_amd import scenes as S

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def drain(sv, n, timeout=120.0):
    got = []
    t0 = time.time()
    while len(got) < n and time.time() - t0 < timeout:
        got += sv.poll(timeout_ms=100)
    assert len(got) == n, (len(got), n)
    return {c["ticket"]: c for c in got}


def test_mix_equals_alone_with_evictions():
    import torch
    from paper_2211_17263_amd import native as NV
    jobs = S.batch_jobs(seed=55, n_jobs=6, max_side=128, max_tris=30000)
    say("serve-mix", [j["scene"].n_tris for j in jobs])
    ctx = NV.Context(0)
    # references rendered on the device once
    refs = []
    alone_scenes = []
    for j in jobs:
        sc = NV.prdpt_scene_create(ctx, j["scene"])
        alone_scenes.append(sc)
        refs.append(NV.prdpt_render_reference(sc, j["theta_ref"], 2).cpu().numpy())
    need = [sc.footprint + j["scene"].width * j["scene"].height * 12
            for sc, j in zip(alone_scenes, jobs)]
    # room for the largest job and a little more: requests for other jobs evict
    budget = int(1.2 * max(need))
    sv = NV.Server(ctx, hbm_budget=budget, max_batch=4)
    try:
        ids = [sv.add_job(j["scene"], r) for j, r in zip(jobs, refs)]
        rng = np.random.default_rng(1)
        subs = []
        for i in range(30):
            k = int(rng.integers(len(jobs)))
            th = (jobs[k]["theta0"] + rng.normal(0, 0.05, jobs[k]["scene"].d)).astype(np.float32)
            seed = 500 + i
            t = sv.submit(ids[k], th, jobs[k]["sigma"], jobs[k]["N"], seed, jobs[k]["est"])
            subs.append((t, k, th, seed))
            if i % 7 == 0:
                time.sleep(0.002)
        res = drain(sv, len(subs))
        st = sv.stats()
    finally:
        sv.stop()
    assert st["completed"] == 30 and st["evictions"] > 0, st
    for t, k, th, seed in subs:
        c = res[t]
        assert c["status"] == 0
        a = NV.prdpt_grad_estimate(alone_scenes[k], torch.from_numpy(refs[k]).cuda(), th,
                                   jobs[k]["sigma"], jobs[k]["N"], seed, jobs[k]["est"])
        assert np.array_equal(c["grad"], a["grad"]), (t, k)
        assert c["loss"] == a["loss"]
        assert c["t_submit"] <= c["t_start"] <= c["t_done"]
    for sc in alone_scenes:
        sc.destroy()
    ctx.close()


def test_admission_refusal_and_cancel():
    from paper_2211_17263_amd import native as NV
    say("serve-admission-cancel")
    ctx = NV.Context(0)
    big = S.cornell_problem(seed=2)          # 256x256, 16 spp: tens of ms per request
    sv = NV.Server(ctx, hbm_budget=3_000_000, max_batch=1)
    try:
        ref = np.zeros((256, 256, 3), np.float32)
        j_big = sv.add_job(big["scene"], ref)
        huge = S.caustic_problem(seed=3, width=64, height=64, spp=1)   # 50k-triangle occluder
        j_huge = sv.add_job(huge["scene"], np.zeros((64, 64, 3), np.float32))
        t_refused = sv.submit(j_huge, huge["theta0"], huge["sigma"], 4, 1, 0)
        tickets = [sv.submit(j_big, big["theta0"], big["sigma"], 16, 10 + i, big["est"]) for i in range(6)]
        sv.cancel(tickets[-1])
        res = drain(sv, 7)
    finally:
        sv.stop()
    assert res[t_refused]["status"] == NV.PRDPT_E_ADMISSION
    assert res[tickets[-1]]["status"] == NV.PRDPT_E_CANCELLED
    assert all(res[t]["status"] == 0 for t in tickets[:-1])
    ctx.close()


def test_served_results_against_oracle():
    # completions of the server on small jobs equal the oracle's estimates
    # within the parity bar (not only the HIP single-request path)
    from oracle import oracle as O
    from paper_2211_17263_amd import native as NV
    from tests import parity as PT
    jobs = S.batch_jobs(seed=77, n_jobs=3, max_side=64, max_tris=5000)
    say("serve-oracle", [(j["scene"].width, j["scene"].n_tris, j["N"]) for j in jobs])
    ctx = NV.Context(0)
    orcs = [O.OracleScene(j["scene"]) for j in jobs]
    refs = [o.reference(j["theta_ref"], seed=4) for o, j in zip(orcs, jobs)]
    sv = NV.Server(ctx, max_batch=4)
    try:
        ids = [sv.add_job(j["scene"], r) for j, r in zip(jobs, refs)]
        subs = []
        for i in range(6):
            k = i % len(jobs)
            t = sv.submit(ids[k], jobs[k]["theta0"], jobs[k]["sigma"], jobs[k]["N"], 900 + i,
                          jobs[k]["est"])
            subs.append((t, k, 900 + i))
        res = drain(sv, len(subs))
    finally:
        sv.stop()
    for t, k, seed in subs:
        j = jobs[k]
        c = res[t]
        assert c["status"] == 0
        o = orcs[k].grad_estimate(refs[k], j["theta0"], j["sigma"], j["N"], seed, j["est"])
        _, w = O.draw_tau(j["est"], j["sigma"], j["N"] // 2, seed)
        PT.assert_grad_match(c["grad"], o["grad"], w, o["losses"], "served")
        assert abs(c["loss"] - o["loss"]) <= PT.LOSS_REL * abs(o["loss"])
    ctx.close()


def test_high_dimensional_job_batched_and_served():
    # the 150-parameter object-sorting scene (75 spheres: a larger dynamic LDS
    # and fewer resident work-groups) through the batched and the served
    # forms: both equal the single-request estimate bit for bit
    import torch
    from paper_2211_17263_amd import native as NV
    pr = S.sort_problem(width=24, height=16, spp=1)
    d = pr["scene"].d
    say("serve-150d", d)
    assert d == 150
    ctx = NV.Context(0)
    sc = NV.prdpt_scene_create(ctx, pr["scene"])
    try:
        ref = NV.prdpt_render_reference(sc, pr["theta_ref"], 2)
        a = NV.prdpt_grad_estimate(sc, ref, pr["theta0"], pr["sigma"], 8, 77, pr["est"])
        torch.cuda.synchronize()
        q = NV.BatchRequest(sc, ref, pr["theta0"], pr["sigma"], 8, 77, pr["est"])
        NV.prdpt_batch_estimate(ctx, [q])
        assert q.status == 0
        assert np.array_equal(q.grad[:d], a["grad"]) and q.loss[0] == a["loss"]
        sv = NV.Server(ctx)
        try:
            j = sv.add_job(pr["scene"], ref.cpu().numpy())
            t = sv.submit(j, pr["theta0"], pr["sigma"], 8, 77, pr["est"])
            c = drain(sv, 1)[t]
        finally:
            sv.stop()
        assert c["status"] == 0
        assert np.array_equal(c["grad"], a["grad"]) and c["loss"] == a["loss"]
    finally:
        sc.destroy()
        ctx.close()

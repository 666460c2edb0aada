"""Error paths of the C ABI, forced from the host: allocation failures
(prdpt_debug_fail_allocations), per-request deadlines of the server, a served
job whose upload fails, and the combine call at large d (autograd backward of a
150-parameter scene).  No kernel is made to fault or wait: every failure is
decided on the host before or after a normal launch."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
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


@pytest.fixture
def no_fault_injection():
    from paper_2211_17263_amd import native as NV
    NV.prdpt_debug_fail_allocations(-1)
    yield
    NV.prdpt_debug_fail_allocations(-1)


def test_scene_create_allocation_failure(no_fault_injection):
    from paper_2211_17263_amd import native as NV
    pr = S.cornell_problem(seed=2, width=32, height=24, spp=1, ico_level=1)
    say("alloc-fail scene_create")
    ctx = NV.Context(0)
    try:
        for after in range(6):  # each of the scene's six device arrays fails in turn
            NV.prdpt_debug_fail_allocations(after)
            with pytest.raises(NV.PrdptError) as e:
                NV.prdpt_scene_create(ctx, pr["scene"])
            assert e.value.code == NV.PRDPT_E_NOMEM
            assert ctx.resident_bytes() == 0
        NV.prdpt_debug_fail_allocations(-1)
        sc = NV.prdpt_scene_create(ctx, pr["scene"])
        assert ctx.resident_bytes() == sc.footprint
        sc.destroy()
    finally:
        ctx.close()


def test_estimate_allocation_failure_then_recovery(no_fault_injection):
    import torch
    from paper_2211_17263_amd import native as NV
    pr = S.cornell_problem(seed=2, width=40, height=24, spp=2, ico_level=1)
    say("alloc-fail estimate")
    osc = O.OracleScene(pr["scene"])
    ref = torch.from_numpy(osc.reference(pr["theta_ref"], seed=3)).cuda()
    ctx0 = NV.Context(0)
    sc0 = NV.prdpt_scene_create(ctx0, pr["scene"])
    want = NV.prdpt_grad_estimate(sc0, ref, pr["theta0"], pr["sigma"], 8, 5, pr["est"])
    sc0.destroy()
    ctx0.close()
    ctx = NV.Context(0)
    sc = NV.prdpt_scene_create(ctx, pr["scene"])
    try:
        failures = 0
        for after in range(40):  # fail the k-th scratch allocation of a fresh context
            NV.prdpt_debug_fail_allocations(after)
            try:
                got = NV.prdpt_grad_estimate(sc, ref, pr["theta0"], pr["sigma"], 8, 5, pr["est"])
            except NV.PrdptError as e:
                assert e.code == NV.PRDPT_E_NOMEM
                failures += 1
                continue
            break
        NV.prdpt_debug_fail_allocations(-1)
        assert failures >= 3        # several scratch arrays, each failed once
        np.testing.assert_array_equal(got["grad"], want["grad"])
        np.testing.assert_array_equal(got["losses"], want["losses"])
    finally:
        NV.prdpt_debug_fail_allocations(-1)
        sc.destroy()
        ctx.close()


def test_server_deadlines_leave_other_requests_alone():
    import torch
    from paper_2211_17263_amd import native as NV
    say("serve-deadline")
    small = S.cornell_problem(seed=2, width=48, height=32, spp=2, ico_level=1)
    big = S.cornell_problem(seed=2)                     # 256x256, 16 spp: >= 10 ms per estimate
    ctx = NV.Context(0)
    sc_small = NV.prdpt_scene_create(ctx, small["scene"])
    ref_small = NV.prdpt_render_reference(sc_small, small["theta_ref"], 2).cpu().numpy()
    sv = NV.Server(ctx, max_batch=8, max_inflight=1)
    try:
        j_small = sv.add_job(small["scene"], ref_small)
        j_big = sv.add_job(big["scene"], np.zeros((256, 256, 3), np.float32))
        # the big request runs for many milliseconds: its 1 ms deadline passes
        # while it is queued or running
        t_big = sv.submit(j_big, big["theta0"], big["sigma"], 16, 7, big["est"], timeout_s=1e-3)
        t_ok = [sv.submit(j_small, small["theta0"], small["sigma"], 8, 20 + i, small["est"])
                for i in range(3)]
        t_late = sv.submit(j_small, small["theta0"], small["sigma"], 8, 30, small["est"],
                           timeout_s=1e-9)              # expired on arrival
        t_slack = sv.submit(j_small, small["theta0"], small["sigma"], 8, 31, small["est"],
                            timeout_s=600.0)
        res = drain(sv, 6)
    finally:
        sv.stop()
    assert res[t_big]["status"] == NV.PRDPT_E_TIMEOUT
    assert res[t_late]["status"] == NV.PRDPT_E_TIMEOUT
    with pytest.raises(NV.PrdptError):
        sv_bad = NV.Server(ctx)
        try:
            sv_bad.submit(sv_bad.add_job(small["scene"], ref_small), small["theta0"],
                          small["sigma"], 8, 1, small["est"], timeout_s=-1.0)
        finally:
            sv_bad.stop()
    ref_d = torch.from_numpy(ref_small).cuda()
    for t, seed in zip(t_ok + [t_slack], [20, 21, 22, 31]):
        c = res[t]
        assert c["status"] == 0, c
        a = NV.prdpt_grad_estimate(sc_small, ref_d, small["theta0"], small["sigma"], 8, seed,
                                   small["est"])
        assert np.array_equal(c["grad"], a["grad"]) and c["loss"] == a["loss"]
    sc_small.destroy()
    ctx.close()


def test_server_upload_failure_fails_the_request_and_stops(no_fault_injection):
    from paper_2211_17263_amd import native as NV
    say("serve-upload-failure")
    pr = S.cornell_problem(seed=2, width=32, height=24, spp=1, ico_level=1)
    ref = np.zeros((24, 32, 3), np.float32)
    # the context's own budget is smaller than the server's: the upload of the
    # job fails with the context's admission error, not a wait for memory
    ctx = NV.Context(0, hbm_budget=1000)
    sv = NV.Server(ctx, hbm_budget=1 << 30)
    try:
        j = sv.add_job(pr["scene"], ref)
        tickets = [sv.submit(j, pr["theta0"], pr["sigma"], 4, 1 + i, pr["est"]) for i in range(3)]
        res = drain(sv, 3, timeout=30.0)
    finally:
        t0 = time.time()
        sv.stop()
        assert time.time() - t0 < 10.0
    assert all(res[t]["status"] == NV.PRDPT_E_ADMISSION for t in tickets)
    ctx.close()
    # device memory running out during an upload: that request fails with
    # PRDPT_E_NOMEM, later ones (memory back) run normally
    ctx = NV.Context(0)
    sv = NV.Server(ctx, max_inflight=1)
    try:
        j = sv.add_job(pr["scene"], ref)
        NV.prdpt_debug_fail_allocations(0)
        t_fail = sv.submit(j, pr["theta0"], pr["sigma"], 4, 1, pr["est"])
        r1 = drain(sv, 1, timeout=30.0)
        NV.prdpt_debug_fail_allocations(-1)
        t_ok = sv.submit(j, pr["theta0"], pr["sigma"], 4, 2, pr["est"])
        r2 = drain(sv, 1, timeout=30.0)
    finally:
        NV.prdpt_debug_fail_allocations(-1)
        sv.stop()
    assert r1[t_fail]["status"] == NV.PRDPT_E_NOMEM
    assert r2[t_ok]["status"] == 0
    ctx.close()


def test_autograd_backward_at_150_parameters():
    # the combine call takes any d up to the parameter limit: backward of the
    # 150-D problem equals the C ABI's gradient bit for bit
    import torch
    from paper_2211_17263_amd import native as NV
    from paper_2211_17263_amd.autograd import smoothed_loss
    pr = S.sort_problem(width=32, height=32, spp=1)
    say("autograd d=150")
    ref = O.OracleScene(pr["scene"]).reference(pr["theta_ref"], seed=3)
    ctx = NV.Context(0)
    sc = NV.prdpt_scene_create(ctx, pr["scene"])
    try:
        ref_d = torch.from_numpy(ref).cuda()
        for est in (NV.PRDPT_EST_GAUSS, NV.PRDPT_EST_IS):
            theta = torch.tensor(pr["theta0"], device="cuda", requires_grad=True)
            q = smoothed_loss(theta, sc, ref_d, pr["sigma"], 8, 17, est)
            q.backward()
            r = NV.prdpt_grad_estimate(sc, ref_d, pr["theta0"], pr["sigma"], 8, 17, est)
            assert theta.grad.numel() == 150
            np.testing.assert_array_equal(theta.grad.cpu().numpy(), r["grad"].astype(np.float32))
        with pytest.raises(NV.PrdptError) as e:
            c = torch.zeros(4, 257, dtype=torch.float64, device="cuda")
            NV.prdpt_combine_async(ctx, 4, 257, c, torch.zeros(8, dtype=torch.float64, device="cuda"),
                                   None, torch.zeros(257, dtype=torch.float64, device="cuda"))
        assert e.value.code == NV.PRDPT_E_ARG
    finally:
        sc.destroy()
        ctx.close()

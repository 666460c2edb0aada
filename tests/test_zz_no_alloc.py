"""The allocation-free estimate (prdpt_grad_estimate_noalloc) against the
stream-ordered estimate it mirrors (prdpt_grad_estimate_async), through the C
ABI: equal bit for bit on two calls in a row, the second smaller; with every
library allocation made to fail it still runs; requests beyond its scratch
are refused before anything is enqueued."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_17263_amd import scenes as S

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _both(NV, sc, ref, theta, sigma, N, seed, est, with_outputs):
    import torch
    d = sc.d
    rows = N if est & NV.PRDPT_EST_INDEPENDENT else N // 2
    out = []
    for fn in (NV.prdpt_grad_estimate_async, NV.prdpt_grad_estimate_noalloc):
        g = torch.full((d,), float("nan"), dtype=torch.float64, device="cuda")
        q = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        L = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda") if with_outputs else None
        c = (torch.full((rows, d), float("nan"), dtype=torch.float64, device="cuda")
             if with_outputs else None)
        fn(sc, ref, torch.tensor(theta, device="cuda"), torch.tensor(sigma, device="cuda"), N,
           seed, est, g, q, L, c)
        torch.cuda.synchronize()
        out.append((g.cpu().numpy(), q.cpu().numpy(),
                    None if L is None else L.cpu().numpy(), None if c is None else c.cpu().numpy()))
    return out


def test_noalloc_equals_async_twice_then_smaller():
    import torch
    from paper_2211_17263_amd import native as NV
    ctx = NV.Context(0)
    big = S.cornell_problem(seed=2, width=96, height=64, spp=4, ico_level=3)
    small = S.toy_problem(seed=3)
    scenes = []
    try:
        for pr, N, seed, est, outs in ((big, 16, 5, NV.PRDPT_EST_IS, True),
                                       (small, 4, 6, NV.PRDPT_EST_GAUSS, False),
                                       (small, 6, 7, NV.PRDPT_EST_IS | NV.PRDPT_EST_INDEPENDENT, True)):
            sc_desc = pr["scene"]
            say("noalloc", sc_desc.width, sc_desc.height, sc_desc.spp, N, est)
            ref = torch.from_numpy(O.OracleScene(sc_desc).reference(pr["theta_ref"], seed=2)).cuda()
            sc = NV.prdpt_scene_create(ctx, sc_desc)
            scenes.append(sc)
            (ga, qa, La, ca), (gn, qn, Ln, cn) = _both(NV, sc, ref, pr["theta0"], pr["sigma"], N,
                                                       seed, est, outs)
            assert np.all(np.isfinite(gn)) and np.array_equal(ga, gn)
            assert np.array_equal(qa, qn)
            if outs:
                assert np.array_equal(La, Ln) and np.array_equal(ca, cn)
    finally:
        for sc in scenes:
            sc.destroy()
        ctx.close()


def test_noalloc_needs_no_allocation_and_refuses_large_requests():
    import torch
    from paper_2211_17263_amd import native as NV
    pr = S.toy_problem(seed=4)
    ctx = NV.Context(0)
    sc = NV.prdpt_scene_create(ctx, pr["scene"])
    big = NV.prdpt_scene_create(ctx, S.toy_scene(width=4096, height=4096))
    ref = torch.from_numpy(O.OracleScene(pr["scene"]).reference(pr["theta_ref"], seed=2)).cuda()
    th = torch.tensor(pr["theta0"], device="cuda")
    sg = torch.tensor(pr["sigma"], device="cuda")
    try:
        g = torch.zeros(2, dtype=torch.float64, device="cuda")
        q = torch.zeros(1, dtype=torch.float64, device="cuda")
        say("noalloc with every allocation failing")
        NV.prdpt_debug_fail_allocations(0)
        try:
            NV.prdpt_grad_estimate_noalloc(sc, ref, th, sg, 8, 9, NV.PRDPT_EST_GAUSS, g, q)
            torch.cuda.synchronize()
            # the allocating form needs its scratch on this fresh context
            with pytest.raises(NV.PrdptError) as e:
                NV.prdpt_grad_estimate_async(sc, ref, th, sg, 8, 9, NV.PRDPT_EST_GAUSS,
                                             torch.zeros_like(g), torch.zeros_like(q))
            assert e.value.code == NV.PRDPT_E_NOMEM
        finally:
            NV.prdpt_debug_fail_allocations(-1)
        want = NV.prdpt_grad_estimate(sc, ref, pr["theta0"], pr["sigma"], 8, 9, NV.PRDPT_EST_GAUSS)
        assert np.array_equal(g.cpu().numpy(), want["grad"])
        # 4096 x 4096 image, N = 64: 64 x 262144 tile losses exceed the scratch
        say("noalloc over the limit")
        with pytest.raises(NV.PrdptError) as e:
            NV.prdpt_grad_estimate_noalloc(big, ref, th, sg, 64, 1, NV.PRDPT_EST_GAUSS, g, q)
        assert e.value.code == NV.PRDPT_E_ARG
    finally:
        sc.destroy()
        big.destroy()
        ctx.close()

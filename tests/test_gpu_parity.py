"""HIP path vs CPU oracle, element by element, through the C ABI (needs a GPU).

Every case prints its name, shapes and seed before touching the GPU so that a
failing run names the case.
"""
import math
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
def ctx():
    import torch
    from paper_2211_17263_amd import native as NV
    assert torch.cuda.is_available()
    c = NV.Context(0)
    yield c
    c.synchronize()


def gpu_scene(ctx, scene):
    from paper_2211_17263_amd import native as NV
    return NV.prdpt_scene_create(ctx, scene)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS, O.IS_PERDIM, O.IS | O.INDEPENDENT,
                                  O.GAUSS | O.INDEPENDENT,
                                  O.IS | O.INDEPENDENT | O.STRATIFIED,
                                  O.GAUSS | O.INDEPENDENT | O.STRATIFIED,
                                  O.IS_PERDIM | O.INDEPENDENT | O.STRATIFIED])
@pytest.mark.parametrize("d", [1, 2, 3, 6, 12, 32, 33, 150, 256])
def test_perturbation_draw_bit_exact(ctx, mode, d):
    from paper_2211_17263_amd import native as NV
    say("draw_tau", mode, d)
    sigma = np.linspace(0.05, 1.5, d).astype(np.float32)
    tg, cg = NV.prdpt_draw_tau(ctx, mode, sigma, 777, 0x1234_5678_9ABC)
    to, co = O.draw_tau(mode, sigma, 777, 0x1234_5678_9ABC)
    assert np.array_equal(tg.view(np.uint32), to.view(np.uint32))
    assert np.array_equal(cg.view(np.uint64), co.view(np.uint64))


def _full_parity(ctx, pr, seed, what, N=None, est=None, check_images=True):
    scene = pr["scene"]
    N = N or pr["N"]
    est = pr["est"] if est is None else est
    say(what, f"{scene.width}x{scene.height} spp={scene.spp} B={scene.max_bounces}",
        f"tris={scene.n_tris} N={N} est={est} seed={seed}")
    from paper_2211_17263_amd import native as NV
    osc = O.OracleScene(scene)
    ref = osc.reference(pr["theta_ref"], seed=seed + 1)
    gs = gpu_scene(ctx, scene)
    try:
        if check_images:
            imgs, tau = NV.prdpt_render_perturbed(gs, pr["theta0"], pr["sigma"], N, seed, est)
            oimgs, otau = osc.render_perturbed(pr["theta0"], pr["sigma"], N, seed, est)
            assert np.array_equal(tau, otau)
            gi = imgs.cpu().numpy()
            for k in range(N):
                PT.assert_images_match(gi[k], oimgs[k], f"{what} image {k}")
        r = NV.prdpt_grad_estimate(gs, to_dev(ref), pr["theta0"], pr["sigma"], N, seed, est)
        o = osc.grad_estimate(ref, pr["theta0"], pr["sigma"], N, seed, est)
        _, c = O.draw_tau(est, pr["sigma"], N if est & O.INDEPENDENT else N // 2, seed)
        PT.assert_losses_match(r["losses"], o["losses"], what)
        PT.assert_grad_match(r["grad"], o["grad"], c, o["losses"], what)
        assert abs(r["loss"] - o["loss"]) <= PT.LOSS_REL * abs(o["loss"])
        return r, o
    finally:
        gs.destroy()


def test_toy_workload_full(ctx):
    pr = S.toy_problem(seed=1)
    r, o = _full_parity(ctx, pr, 11, "toy")
    assert np.any(r["grad"] != 0)


@pytest.mark.parametrize("seed", [3, 4])
def test_toy_workload_is_mode(ctx, seed):
    pr = S.toy_problem(seed=seed)
    _full_parity(ctx, pr, seed, "toy-is", est=O.IS, N=8)


@pytest.mark.parametrize("est", [O.GAUSS | O.INDEPENDENT, O.IS | O.INDEPENDENT,
                                 O.IS | O.INDEPENDENT | O.STRATIFIED])
def test_independent_perturbations_toy(ctx, est):
    # the noAT arm: N independent draws, one render each with its own paths
    pr = S.toy_problem(seed=2)
    r, o = _full_parity(ctx, pr, 13, "toy-independent", est=est, N=6)
    assert np.any(r["grad"] != 0)


def test_independent_perturbations_cornell_reduced(ctx):
    pr = S.cornell_problem(seed=2, width=64, height=48, spp=4, ico_level=3)
    _full_parity(ctx, pr, 8, "cornell-reduced-independent", est=O.IS | O.INDEPENDENT, N=6)


def test_colour_bindings_cornell_reduced(ctx):
    # light position, sphere translation and the left wall's albedo (d = 9)
    pr = S.cornell_problem(seed=2, colour=True, width=64, height=48, spp=4, ico_level=3)
    r, o = _full_parity(ctx, pr, 7, "cornell-reduced-colour")
    assert np.all(r["grad"][6:] != 0)


@pytest.mark.parametrize("est", [O.GAUSS, O.IS_PERDIM])
def test_emission_and_albedo_bindings(ctx, est):
    # the area light's radiance (emissive branch) and one wall channel
    sc = S.cornell_scene(width=40, height=36, spp=3, bounces=3, ico_level=2)
    sc.bindings = []
    light = [i for i, t in enumerate(sc.mat_type) if t == S.EMISSIVE][0]
    for c in range(3):
        sc.bind(S.BIND_ALBEDO, light, c)
    sc.bind(S.BIND_ALBEDO, 1, 0)
    pr = dict(scene=sc, theta_ref=np.array([-3.0, 2.0, 0.0, 0.2], np.float32),
              theta0=np.zeros(4, np.float32), sigma=np.array([2.0, 2.0, 2.0, 0.2], np.float32),
              N=8, est=est)
    r, o = _full_parity(ctx, pr, 12, "emission-albedo")
    assert np.any(r["grad"] != 0)


def test_rotation_bindings_cornell_reduced(ctx):
    # light position, sphere translation, wall colour and the tall box's turn
    # about the vertical axis (d = 10)
    pr = S.cornell_problem(seed=2, colour=True, rotation=True, width=64, height=48, spp=4,
                           ico_level=3)
    r, o = _full_parity(ctx, pr, 15, "cornell-reduced-rotation")
    assert r["grad"][9] != 0


@pytest.mark.parametrize("est", [O.GAUSS, O.IS])
def test_rotation_all_axes(ctx, est):
    # a random-triangle cloud turned about all three axes and moved, beside a
    # rotated mesh whose angles are not bound
    rng = np.random.default_rng(21)
    sc = S.toy_scene(width=48, height=40, spp=2, bounces=2)
    sc.bindings = []
    v, f = S.random_triangles(rng, 3000, (-0.5, -0.5, -0.3), (0.5, 0.5, 0.3), 0.08)
    m = sc.mesh(v, f, 0, translation=(0.2, 0.1, 0.6), rotation=(0.3, -0.2, 0.8))
    vb, fb = S.box_tris((0.0, 0.0, 0.0), (0.4, 0.3, 0.2), 0.0)
    sc.mesh(vb, fb, 0, translation=(-0.8, -0.6, 0.2), rotation=(0.0, 0.4, 1.0))
    for c in range(3):
        sc.bind(S.BIND_MESH_ROT, m, c)
    sc.bind(S.BIND_MESH, m, 0)
    pr = dict(scene=sc, theta_ref=np.array([0.1, 0.2, -0.3, 0.05], np.float32),
              theta0=np.array([-0.2, 0.1, 0.2, -0.1], np.float32),
              sigma=np.full(4, 0.2, np.float32), N=8, est=est)
    r, o = _full_parity(ctx, pr, 16, "rotation-all-axes")
    assert np.all(r["grad"] != 0)


@pytest.mark.parametrize("est", [O.IS, O.GAUSS, O.IS_PERDIM])
def test_many_objects_reduced(ctx, est):
    # 75 spheres, each moved in x and z: d = 150
    pr = S.sort_problem(width=48, height=40, spp=2)
    r, o = _full_parity(ctx, pr, 17, "sort-reduced", est=est, N=8)
    assert np.count_nonzero(r["grad"]) > 100


def test_cornell_reduced(ctx):
    pr = S.cornell_problem(seed=2, width=64, height=48, spp=4, ico_level=3)
    _full_parity(ctx, pr, 5, "cornell-reduced")


def test_caustic_reduced(ctx):
    pr = S.caustic_problem(seed=3, width=96, height=72, spp=4, n_occluders=5000)
    _full_parity(ctx, pr, 6, "caustic-reduced", N=8)


def test_ragged_tiny_and_degenerate(ctx):
    # ragged tile tail, N = 2 (one pair), d = 1, pixel-centre sampling, odd spp
    sc = S.toy_scene(width=37, height=23, spp=3, pixel_center=0, bounces=2)
    sc.bindings = sc.bindings[:1]
    pr = dict(scene=sc, theta_ref=np.zeros(1, np.float32), theta0=np.array([0.4], np.float32),
              sigma=np.array([0.25], np.float32), N=2, est=O.IS)
    _full_parity(ctx, pr, 9, "ragged")
    sc2 = S.toy_scene(width=1, height=1, spp=1, pixel_center=1)
    pr2 = dict(scene=sc2, theta_ref=np.zeros(2, np.float32), theta0=np.array([0.1, 0.2], np.float32),
               sigma=np.array([0.3, 0.3], np.float32), N=2, est=O.GAUSS)
    _full_parity(ctx, pr2, 10, "one-pixel")


def test_more_samples_than_one_wave(ctx):
    # more samples per pixel (80) than lanes in a wave, several paths of the
    # same pixel finishing in one iteration; a small image with at least 16
    # samples per pixel renders in 4x4 tiles, here with ragged edges
    # (21 x 13: 80 x 16 jobs per full tile)
    sc = S.toy_scene(width=21, height=13, spp=80, bounces=1)
    pr = dict(scene=sc, theta_ref=np.zeros(2, np.float32), theta0=np.array([0.3, -0.2], np.float32),
              sigma=np.full(2, 0.3, np.float32), N=4, est=O.IS)
    _full_parity(ctx, pr, 19, "spp-80")


def test_exact_ties_take_the_smaller_id(ctx):
    # two identical static icospheres (one BVH): every hit on them is an exact
    # tie in t between a triangle and its twin, which the closest-hit rule
    # breaks by the smaller primitive id, i.e. the first (green) copy; shadow
    # rays meet the same twin occluders
    sc = S.toy_scene(width=40, height=32, spp=2, bounces=2)
    green = sc.material(S.DIFFUSE, (0.1, 0.8, 0.1))
    blue = sc.material(S.DIFFUSE, (0.1, 0.1, 0.8))
    v, f = S.icosphere(2)
    v = (v * 0.45 + np.array([-0.9, 0.3, 0.6])).astype(np.float32)
    sc.mesh(v, f, green)
    sc.mesh(v.copy(), f.copy(), blue)
    pr = dict(scene=sc, theta_ref=np.zeros(2, np.float32), theta0=np.array([0.2, -0.1], np.float32),
              sigma=np.full(2, 0.3, np.float32), N=4, est=O.IS)
    _full_parity(ctx, pr, 23, "exact-ties")
    img = O.OracleScene(sc).reference(pr["theta_ref"], seed=5)
    g, b = img[..., 1], img[..., 2]
    assert np.count_nonzero(g > 2.0 * b + 1e-3) > 20   # the green copy is what shows
    assert np.count_nonzero(b > 2.0 * g + 1e-3) == 0


def test_zero_normal_component_picks_the_same_frame(ctx):
    # an icosphere has faces whose edge cross product has a z component of
    # -0; the world normal (the zero-angle rotation applied to it) has +0
    # there, and the sign of that zero selects the tangent frame of a bounce,
    # so both sides must carry it the same way (camera paths reach such faces)
    sc = S.toy_scene(width=40, height=32, spp=2, bounces=2)
    green = sc.material(S.DIFFUSE, (0.1, 0.8, 0.1))
    v, f = S.icosphere(2)
    v = (v * 0.45 + np.array([-0.9, 0.3, 0.6])).astype(np.float32)
    e1, e2 = v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]]
    nz = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    assert np.any((nz == 0) & np.signbit(nz))
    sc.mesh(v, f, green)
    pr = dict(scene=sc, theta_ref=np.zeros(2, np.float32), theta0=np.array([0.2, -0.1], np.float32),
              sigma=np.full(2, 0.3, np.float32), N=4, est=O.IS)
    _full_parity(ctx, pr, 23, "zero-normal-component")


@pytest.mark.parametrize("seed", range(16))
def test_random_scenes(ctx, seed):
    # small scenes mixing every primitive, material and parameter kind
    sc, theta_ref, theta0, sigma = S.random_scene(seed)
    est = [O.IS, O.GAUSS, O.IS_PERDIM, O.IS | O.INDEPENDENT][seed % 4]
    pr = dict(scene=sc, theta_ref=theta_ref, theta0=theta0, sigma=sigma, N=4, est=est)
    _full_parity(ctx, pr, 40 + seed, f"random-{seed}")


def test_work_counts(ctx):
    # the counting kernel sees every camera path once and whole loops
    from paper_2211_17263_amd import native as NV
    pr = S.cornell_problem(seed=2, width=40, height=24, spp=3, ico_level=2)
    sc = pr["scene"]
    say("work-counts")
    gs = gpu_scene(ctx, sc)
    try:
        c = NV.prdpt_traversal_counts(gs, pr["theta0"], pr["sigma"], 8, 3, O.IS)
    finally:
        gs.destroy()
    assert c["paths"] == 8 * sc.width * sc.height * sc.spp
    assert c["rays"] >= c["paths"]
    for loop, work in (("wave_node_iters", "nodes"), ("wave_tri_iters", "tris"), ("wave_ray_iters", "rays")):
        assert 0 < c[work] <= 64 * c[loop]
    assert 0 <= c["idle_lane_iters"] <= 64 * c["wave_ray_iters"]


def test_environment_and_glass(ctx):
    from paper_2211_17263_amd import native as NV
    for glass in (False, True):
        sc = S.furnace_scene(glass=glass, bounces=6, spp=8, width=40, height=40)
        sc.plight((2.0, 2.0, 2.0), (5.0, 5.0, 5.0))
        sc.bind(S.BIND_SPHERE, 0, 0)
        say("furnace", glass)
        gs = gpu_scene(ctx, sc)
        try:
            X = np.array([0.15], np.float32)
            img = NV.prdpt_render_reference(gs, X, 21).cpu().numpy()
            oimg = O.OracleScene(sc).reference(X, seed=21)
            PT.assert_images_match(img, oimg, f"furnace glass={glass}")
        finally:
            gs.destroy()


def test_smoothed_loss_and_reference(ctx):
    from paper_2211_17263_amd import native as NV
    pr = S.cornell_problem(seed=2, width=40, height=40, spp=2, ico_level=2)
    say("smoothed-loss")
    osc = O.OracleScene(pr["scene"])
    gs = gpu_scene(ctx, pr["scene"])
    try:
        ref_gpu = NV.prdpt_render_reference(gs, pr["theta_ref"], 4).cpu().numpy()
        ref = osc.reference(pr["theta_ref"], seed=4)
        PT.assert_images_match(ref_gpu, ref, "reference")
        q = NV.prdpt_smoothed_loss(gs, to_dev(ref), pr["theta0"], pr["sigma"], 6, 12)
        qo = osc.smoothed_loss(ref, pr["theta0"], pr["sigma"], 6, 12)
        assert abs(q - qo) <= 1e-4 * qo
    finally:
        gs.destroy()


def test_bitwise_reproducible(ctx):
    from paper_2211_17263_amd import native as NV
    pr = S.cornell_problem(seed=2, width=48, height=32, spp=2, ico_level=2)
    say("reproducible")
    ref = O.OracleScene(pr["scene"]).reference(pr["theta_ref"], seed=1)
    gs = gpu_scene(ctx, pr["scene"])
    try:
        a = NV.prdpt_grad_estimate(gs, to_dev(ref), pr["theta0"], pr["sigma"], 8, 99, O.IS)
        b = NV.prdpt_grad_estimate(gs, to_dev(ref), pr["theta0"], pr["sigma"], 8, 99, O.IS)
        assert np.array_equal(a["grad"], b["grad"]) and np.array_equal(a["losses"], b["losses"])
    finally:
        gs.destroy()


def test_async_and_combine(ctx):
    import torch
    from paper_2211_17263_amd import native as NV
    pr = S.toy_problem(seed=5)
    say("async")
    ref = O.OracleScene(pr["scene"]).reference(pr["theta_ref"], seed=2)
    gs = gpu_scene(ctx, pr["scene"])
    try:
        N, d = 6, 2
        sync = NV.prdpt_grad_estimate(gs, to_dev(ref), pr["theta0"], pr["sigma"], N, 7, O.GAUSS)
        g = torch.zeros(d, dtype=torch.float64, device="cuda")
        q = torch.zeros(1, dtype=torch.float64, device="cuda")
        L = torch.zeros(N, dtype=torch.float64, device="cuda")
        c = torch.zeros(N // 2, d, dtype=torch.float64, device="cuda")
        NV.prdpt_grad_estimate_async(gs, to_dev(ref), to_dev(pr["theta0"]), to_dev(pr["sigma"]),
                                     N, 7, O.GAUSS, g, q, L, c)
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy(), sync["grad"])
        assert np.array_equal(L.cpu().numpy(), sync["losses"])
        g2 = torch.zeros(d, dtype=torch.float64, device="cuda")
        scale = torch.tensor([2.5], dtype=torch.float64, device="cuda")
        NV.prdpt_combine_async(ctx, N // 2, d, c, L, scale, g2, O.GAUSS)
        torch.cuda.synchronize()
        np.testing.assert_allclose(g2.cpu().numpy(), 2.5 * sync["grad"], rtol=1e-15)
        # the same with independent perturbations (one weight row per render)
        est = O.GAUSS | O.INDEPENDENT
        sync = NV.prdpt_grad_estimate(gs, to_dev(ref), pr["theta0"], pr["sigma"], N, 9, est)
        c = torch.zeros(N, d, dtype=torch.float64, device="cuda")
        NV.prdpt_grad_estimate_async(gs, to_dev(ref), to_dev(pr["theta0"]), to_dev(pr["sigma"]),
                                     N, 9, est, g, q, L, c)
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy(), sync["grad"])
        NV.prdpt_combine_async(ctx, N, d, c, L, scale, g2, est)
        torch.cuda.synchronize()
        np.testing.assert_allclose(g2.cpu().numpy(), 2.5 * sync["grad"], rtol=1e-15)
    finally:
        gs.destroy()


def test_error_codes(ctx):
    from paper_2211_17263_amd import native as NV
    pr = S.toy_problem(seed=1)
    say("errors")
    gs = gpu_scene(ctx, pr["scene"])
    ref = to_dev(np.zeros((64, 64, 3), np.float32))
    try:
        for N, sigma, est in [(3, pr["sigma"], 0), (0, pr["sigma"], 0),
                              (4, np.array([0.5, 0.0], np.float32), 0), (4, pr["sigma"], 7),
                              (4, pr["sigma"], NV.PRDPT_EST_IS | NV.PRDPT_EST_STRATIFIED)]:
            with pytest.raises(NV.PrdptError) as e:
                NV.prdpt_grad_estimate(gs, ref, pr["theta0"], sigma, N, 1, est)
            assert e.value.code == NV.PRDPT_E_ARG
        bad = S.toy_scene()
        bad.bind(S.BIND_SPHERE, 5, 0)
        with pytest.raises(NV.PrdptError) as e:
            gpu_scene(ctx, bad)
        assert e.value.code == NV.PRDPT_E_SCENE
        bad2 = S.toy_scene()
        bad2.quad_mat[0] = bad2.material(S.DIELECTRIC, ior=1.5)
        with pytest.raises(NV.PrdptError) as e:
            gpu_scene(ctx, bad2)
        assert e.value.code == NV.PRDPT_E_SCENE
        # at most PRDPT_MAX_PARAMS parameters
        many = S.sort_scene(n_objects=128)       # 128 spheres (the most), 256 parameters
        many.bind(S.BIND_QUAD, 0, 1)
        with pytest.raises(NV.PrdptError) as e:
            gpu_scene(ctx, many)
        assert e.value.code == NV.PRDPT_E_SCENE
        # rotation bindings: mesh index in range; angles finite
        bad4 = S.toy_scene()
        bad4.bind(S.BIND_MESH_ROT, 0, 1)          # the toy scene has no mesh
        with pytest.raises(NV.PrdptError) as e:
            gpu_scene(ctx, bad4)
        assert e.value.code == NV.PRDPT_E_SCENE
        bad5 = S.toy_scene()
        vb, fb = S.box_tris((0.0, 0.0, 0.0), (0.4, 0.3, 0.2), 0.0)
        bad5.mesh(vb, fb, 0, rotation=(0.0, float("nan"), 0.0))
        with pytest.raises(NV.PrdptError) as e:
            gpu_scene(ctx, bad5)
        assert e.value.code == NV.PRDPT_E_SCENE
        # colour bindings: material index in range, and no dielectric
        for idx in (len(S.toy_scene().mat_type), None):
            bad3 = S.toy_scene()
            if idx is None:
                idx = bad3.material(S.DIELECTRIC, ior=1.5)
            bad3.bind(S.BIND_ALBEDO, idx, 0)
            with pytest.raises(NV.PrdptError) as e:
                gpu_scene(ctx, bad3)
            assert e.value.code == NV.PRDPT_E_SCENE
    finally:
        gs.destroy()


def test_admission_budget():
    from paper_2211_17263_amd import native as NV
    say("admission")
    small = NV.Context(0, hbm_budget=200_000)
    pr = S.cornell_problem(seed=2, width=32, height=32, spp=1, ico_level=4)
    with pytest.raises(NV.PrdptError) as e:
        NV.prdpt_scene_create(small, pr["scene"])
    assert e.value.code == NV.PRDPT_E_ADMISSION
    ok = NV.prdpt_scene_create(small, S.toy_scene())
    assert small.resident_bytes() == ok.footprint
    ok.destroy()
    assert small.resident_bytes() == 0
    small.close()


def test_cornell_full_size(ctx):
    # the full global-illumination workload: 256x256, 16 spp, 4 bounces, N = 16,
    # IS; all 16 images pixel by pixel, the losses and the gradient
    pr = S.cornell_problem(seed=2)
    _full_parity(ctx, pr, 2024, "cornell-full")


def test_caustic_full_size_estimate(ctx):
    # one whole estimate of the caustic workload (512x512, 64 spp, 8 bounces,
    # 50k occluders, N = 32, IS, sigma 1.0 of step 0) against the oracle's:
    # every per-image loss and the gradient
    pr = S.caustic_problem(seed=3)
    _full_parity(ctx, pr, 4242, "caustic-full-estimate", check_images=False)


def test_deep_stack_uses_private_part(ctx):
    # long thin triangles overlapping across the view: a ray's traversal
    # stack outgrows its LDS part into the private entries (host tests show
    # this tree's bound is above the LDS part and within the private one);
    # the estimate still equals the oracle's
    from paper_2211_17263_amd import native as NV
    sc = S.deep_stack_scene()
    pr = dict(scene=sc, theta_ref=np.array([0.05, -0.03], np.float32),
              theta0=np.array([-0.04, 0.06], np.float32), sigma=np.full(2, 0.05, np.float32),
              N=4, est=O.IS)
    gs = gpu_scene(ctx, sc)
    try:
        say("deep-stack counts", sc.n_tris)
        c = NV.prdpt_traversal_counts(gs, pr["theta0"], pr["sigma"], 4, 3, O.IS)
    finally:
        gs.destroy()
    assert c["deepest_stack"] > 23 and c["overflow_pushes"] > 0, c  # LDS part: 13 entries
    _full_parity(ctx, pr, 3, "deep-stack")


@pytest.mark.parametrize("step", [0, 100, 199])
def test_caustic_full_size_sampled(ctx, step):
    # full caustic workload: 512x512, 64 spp, 8 bounces, 50k occluders, N = 32,
    # at the bandwidth of annealing steps 0, 100 and 199 of 200 (sigma 1.0 ->
    # 0.05); the oracle re-renders 256 sampled pixels of three perturbed images
    from paper_2211_17263_amd import native as NV
    pr = S.caustic_problem(seed=3)
    sigma = np.array([O.sigma_schedule(a, b, step, 200) for a, b in
                      zip(pr["sigma"], np.full_like(pr["sigma"], pr["sigma_end"]))], np.float32)
    seed, N = 31 + step, 32
    say("caustic-full", "512x512 spp=64 B=8 N=32 step", step, "sigma", float(sigma[0]))
    osc = O.OracleScene(pr["scene"])
    gs = gpu_scene(ctx, pr["scene"])
    try:
        imgs, tau = NV.prdpt_render_perturbed(gs, pr["theta0"], sigma, N, seed, O.IS)
        otau, _ = O.draw_tau(O.IS, sigma, N // 2, seed)
        assert np.array_equal(tau, otau)
        rng = np.random.default_rng(0)
        pix = rng.choice(512 * 512, 256, replace=False).astype(np.int32)
        for k in (0, 1, N - 1):
            p = k // 2
            X = (pr["theta0"] + tau[p]) if k % 2 == 0 else (pr["theta0"] - tau[p])
            X = X.astype(np.float32)
            ov = osc.render_pixels(X, pix, tag=O.TAG_PATH, pair=p, seed=seed)
            gv = imgs[k].reshape(-1, 3)[pix].cpu().numpy()
            PT.assert_images_match(gv, ov, f"caustic-full k={k}")
    finally:
        gs.destroy()

"""Pins of the oracle's path tracer: closed forms, analytic geometry, brute force,
and the end-to-end estimator against quadrature plus finite differences."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_17263_amd import scenes as S


def camera_rays_f64(sc):
    """Pixel-centre camera rays in binary64 from the scene's binary32 camera vectors."""
    W, H = sc.width, sc.height
    x, y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    sx = 2.0 * x / W - 1.0
    sy = 1.0 - 2.0 * y / H
    f, r, u = (np.asarray(v, np.float64) for v in (sc.fwd, sc.right, sc.up))
    d = f[None, None, :] + sx[..., None] * r[None, None, :] + sy[..., None] * u[None, None, :]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.asarray(sc.eye, np.float64), d


def ray_sphere(o, d, c, r):
    oc = o - c
    b = (oc * d).sum(-1)
    cc = (oc * oc).sum() - r * r
    disc = b * b - cc
    t = np.where(disc >= 0, -b - np.sqrt(np.maximum(disc, 0)), np.inf)
    return t, disc


@pytest.mark.parametrize("albedo", [0.25, 0.6, 0.9])
def test_white_furnace(albedo):
    # convex diffuse sphere under unit environment: sphere pixels equal the
    # albedo, background pixels equal 1, with zero variance
    sc = S.furnace_scene(albedo=albedo, spp=3, bounces=3)
    sc.pixel_center = 1
    img = O.OracleScene(sc).render([], seed=9)
    o, d = camera_rays_f64(sc)
    t, disc = ray_sphere(o, d, np.zeros(3), 0.8)
    hit = disc > 1e-4
    miss = disc < -1e-4
    a32 = np.float32(albedo)
    assert np.all(img[hit] == a32)
    assert np.all(img[miss] == 1.0)
    assert hit.sum() > 50 and miss.sum() > 50


def test_lambertian_plane_point_light():
    # radiance = (rho/pi) I h / r^3 for pixel-centre rays, direct lighting only
    sc = S.plane_scene()
    img = O.OracleScene(sc).render([])
    o, d = camera_rays_f64(sc)
    t = -o[2] / d[..., 2]
    p = o[None, None, :] + t[..., None] * d
    lpos = np.array(sc.plights[0][:3], np.float64)
    I = sc.plights[0][3]
    rho = sc.mat_rgb[0][0]
    v = lpos[None, None, :] - p
    r = np.linalg.norm(v, axis=-1)
    L = rho / math.pi * I * lpos[2] / r**3
    np.testing.assert_allclose(img[..., 0], L, rtol=2e-5)
    np.testing.assert_allclose(img[..., 1], img[..., 0], rtol=0)


def plane_irradiance_over_pi(sc):
    """I h / (pi r^3) at each pixel-centre hit of the plane scene (binary64)."""
    o, d = camera_rays_f64(sc)
    t = -o[2] / d[..., 2]
    p = o[None, None, :] + t[..., None] * d
    lpos = np.array(sc.plights[0][:3], np.float64)
    r = np.linalg.norm(lpos[None, None, :] - p, axis=-1)
    return sc.plights[0][3] / math.pi * lpos[2] / r**3


def test_albedo_binding_plane_closed_form():
    # a colour binding offsets one channel of the material's albedo, which the
    # Lambertian shading multiplies: channel c reads (rho_c + x_c) I h / (pi r^3)
    sc = S.plane_scene()
    sc.bind(S.BIND_ALBEDO, 0, 0)
    sc.bind(S.BIND_ALBEDO, 0, 2)
    img = O.OracleScene(sc).render(np.array([0.25, -0.125], np.float32))
    A = plane_irradiance_over_pi(sc)
    rho = sc.mat_rgb[0][0]
    np.testing.assert_allclose(img[..., 0], (rho + 0.25) * A, rtol=2e-5)
    np.testing.assert_allclose(img[..., 1], rho * A, rtol=2e-5)
    np.testing.assert_allclose(img[..., 2], (rho - 0.125) * A, rtol=2e-5)


@pytest.mark.parametrize("mode", [O.GAUSS, O.IS, O.GAUSS | O.INDEPENDENT])
def test_albedo_gradient_of_quadratic_loss(mode):
    # with albedo offsets x the plane's image is (rho + x) A per channel, so the
    # loss is a quadratic in x: an antithetic difference is exactly 2 grad L . tau,
    # and an independent draw's loss is L(theta) + grad L . tau + tau^T H tau / 2
    sc = S.plane_scene()
    sc.bind(S.BIND_ALBEDO, 0, 0)
    sc.bind(S.BIND_ALBEDO, 0, 2)
    osc = O.OracleScene(sc)
    x_ref = np.array([0.1, -0.05], np.float32)
    ref = osc.reference(x_ref)
    theta = np.zeros(2, np.float32)
    sigma = np.array([0.05, 0.08], np.float32)
    N, seed = 8, 21
    r = osc.grad_estimate(ref, theta, sigma, N, seed, mode)
    A2 = (plane_irradiance_over_pi(sc) ** 2).mean()
    grad = 2.0 / 3.0 * A2 * (theta - x_ref.astype(np.float64))   # mean over 3 channels
    H = 2.0 / 3.0 * A2
    tau = r["tau"].astype(np.float64)
    if mode & O.INDEPENDENT:
        # single-sample Gaussian weight tau / sigma^2 on L(theta + tau)
        L0 = (2.0 / 3.0) * A2 * 0.5 * float(((theta - x_ref) ** 2).sum())
        Li = L0 + tau @ grad + 0.5 * H * (tau ** 2).sum(1)
        np.testing.assert_allclose(r["losses"], Li, rtol=1e-4)
        want = ((tau / sigma.astype(np.float64) ** 2) * Li[:, None]).mean(0)
    else:
        if mode == O.GAUSS:
            c = tau / (2.0 * sigma.astype(np.float64) ** 2)
        else:
            _, c = O.draw_tau(mode, sigma, N // 2, seed)
        want = (c * (2.0 * (tau @ grad))[:, None]).mean(0)
    np.testing.assert_allclose(r["grad"], want, rtol=2e-4)


def test_emission_binding_is_linear_in_radiance():
    # every contribution of a path carries one emitted radiance, and sampling
    # does not depend on it: with the light's channel bound, that channel of
    # the image scales by (Le + x) / Le at a fixed seed, the others are unchanged
    sc = S.cornell_scene(width=24, height=20, spp=2, bounces=3, ico_level=1)
    sc.bindings = []
    light = [i for i, t in enumerate(sc.mat_type) if t == S.EMISSIVE][0]
    sc.bind(S.BIND_ALBEDO, light, 1)
    osc = O.OracleScene(sc)
    a = osc.render(np.zeros(1, np.float32), seed=4)
    b = osc.render(np.array([-6.0], np.float32), seed=4)
    le = sc.mat_rgb[light][1]
    np.testing.assert_array_equal(a[..., [0, 2]], b[..., [0, 2]])
    np.testing.assert_allclose(b[..., 1], a[..., 1] * (le - 6.0) / le, rtol=1e-5, atol=1e-7)
    assert a[..., 1].mean() > 0.05


def test_shadow_boundary_against_analytic_geometry():
    # toy scene at a fixed sphere position, pixel-centre rays, direct light only:
    # every pixel classified analytically (binary64) as sphere / lit plane /
    # shadowed plane must agree with the render, except within a thin margin
    sc = S.toy_scene(pixel_center=1)
    X = np.array([0.35, -0.25], np.float32)
    img = O.OracleScene(sc).render(X)
    o, d = camera_rays_f64(sc)
    c = np.array([0.35, -0.25, 0.5], np.float64)
    r = 0.5
    t_s, disc = ray_sphere(o, d, c, r)
    lpos = np.array(sc.plights[0][:3], np.float64)
    on_sphere = disc > 1e-3
    on_plane = disc < -1e-3
    tp = -o[2] / d[..., 2]
    p = o[None, None, :] + tp[..., None] * d
    # segment plane point -> light against the sphere
    L = lpos[None, None, :] - p
    dist = np.linalg.norm(L, axis=-1)
    Ld = L / dist[..., None]
    oc = p - c
    b = (oc * Ld).sum(-1)
    cc = (oc * oc).sum(-1) - r * r
    disc2 = b * b - cc
    shadowed = (disc2 > 1e-3) & (-b - np.sqrt(np.maximum(disc2, 0)) > 0)
    lit = (disc2 < -1e-3) | ((disc2 > 1e-3) & (-b + np.sqrt(np.maximum(disc2, 0)) < 0))
    v = img[..., 0]
    assert np.all(v[on_plane & shadowed] == 0.0)
    assert np.all(v[on_plane & lit] > 0.0)
    # sphere points facing the light are lit
    ps = o[None, None, :] + t_s[..., None] * d
    n = (ps - c) / r
    facing = ((lpos[None, None, :] - ps) * n).sum(-1)
    assert np.all(v[on_sphere & (facing > 1e-3)] > 0.0)
    assert np.all(v[on_sphere & (facing < -1e-3)] == 0.0)
    assert (on_plane & shadowed).sum() > 20


def test_bvh_closest_hit_equals_brute_force():
    rng = np.random.default_rng(3)
    sc = S.toy_scene()
    v, f = S.random_triangles(rng, 3000, (-1, -1, 0.2), (1, 1, 1.5), 0.08)
    m = sc.mesh(v, f, 0, translation=(0.1, -0.05, 0.0))
    sc.bind(S.BIND_MESH, m, 2)
    X = np.array([0.2, 0.1, 0.05], np.float32)
    fast = O.OracleScene(sc)
    slow = O.OracleScene(sc, brute_force=True)
    n = 20000
    o = np.tile(np.array([0.0, 0.0, 5.0], np.float32), (n, 1)) + rng.normal(0, 0.3, (n, 3)).astype(np.float32)
    tgt = rng.uniform(-1.2, 1.2, (n, 3)).astype(np.float32)
    tgt[:, 2] = rng.uniform(0, 1.5, n)
    d = (tgt - o)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t1, i1 = fast.trace(X, o, d.astype(np.float32))
    t2, i2 = slow.trace(X, o, d.astype(np.float32))
    assert np.array_equal(i1, i2)
    assert np.array_equal(t1, t2)
    assert (i1 >= 3).sum() > 1000          # many triangle hits (ids after sphere and quad)


def _twin_scenes():
    sc = S.toy_scene(width=40, height=32, spp=2, bounces=2)
    green = sc.material(S.DIFFUSE, (0.1, 0.8, 0.1))
    blue = sc.material(S.DIFFUSE, (0.1, 0.1, 0.8))
    v, f = S.icosphere(2)
    v = (v * 0.45 + np.array([-0.9, 0.3, 0.6])).astype(np.float32)
    single = S.toy_scene(width=40, height=32, spp=2, bounces=2)
    single.material(S.DIFFUSE, (0.1, 0.8, 0.1))
    single.material(S.DIFFUSE, (0.1, 0.1, 0.8))
    sc.mesh(v, f, green)
    sc.mesh(v.copy(), f.copy(), blue)
    single.mesh(v.copy(), f.copy(), green)
    return sc, single, len(f)


def test_exact_ties_resolve_to_the_smaller_id():
    # a mesh and its exact twin: every hit on them ties in t, and the closest-hit
    # rule (t, then primitive id) must take the first copy, in the BVH and by
    # brute force alike; the rendered image is then the twin-free scene's
    sc, single, nf = _twin_scenes()
    rng = np.random.default_rng(8)
    X = np.zeros(2, np.float32)
    n = 4000
    o = np.tile(np.array([0.0, 0.0, 5.0], np.float32), (n, 1))
    tgt = np.array([-0.9, 0.3, 0.6]) + rng.uniform(-0.5, 0.5, (n, 3))
    d = (tgt - o) / np.linalg.norm(tgt - o, axis=1, keepdims=True)
    first = 1 + 1  # ids: the sphere, the ground quad, then the triangles
    for brute in (False, True):
        t, i = O.OracleScene(sc, brute_force=brute).trace(X, o, d.astype(np.float32))
        assert np.count_nonzero((i >= first) & (i < first + nf)) > 1000
        assert np.count_nonzero(i >= first + nf) == 0
    theta = np.array([0.2, -0.1], np.float32)
    a = O.OracleScene(sc).reference(theta, seed=5)
    b = O.OracleScene(single).reference(theta, seed=5)
    assert np.array_equal(a, b)


def test_many_spheres_closest_hit_analytic():
    # 75 bound spheres, each moved by its two parameters: the closest hit of a
    # ray is the nearest intersected sphere in binary64 (rays whose two nearest
    # candidates are within 1e-4 of each other, or that graze a sphere, are
    # left out)
    pr = S.sort_problem(width=8, height=8, spp=1)
    sc = pr["scene"]
    X = pr["theta0"]
    rng = np.random.default_rng(12)
    n = 20000
    o = np.tile(np.array(sc.eye, np.float32), (n, 1))
    tgt = np.stack([rng.uniform(-1.6, 1.6, n), np.full(n, 0.1), rng.uniform(-1.6, 1.6, n)], 1)
    d = tgt - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    t, ids = O.OracleScene(sc).trace(X, o, d)
    cen = np.array([s[:3] for s in sc.spheres], np.float64)
    for j, (kind, idx, comp) in enumerate(sc.bindings):
        cen[idx, comp] = np.float32(np.float32(sc.spheres[idx][comp]) + X[j])
    r = np.array([s[3] for s in sc.spheres], np.float64)
    oc = o[:, None, :].astype(np.float64) - cen[None]
    dd = d.astype(np.float64)
    b = (oc * dd[:, None, :]).sum(-1)
    disc = b * b - ((oc * oc).sum(-1) - r[None] ** 2)
    th = np.where(disc > 0, -b - np.sqrt(np.maximum(disc, 0)), np.inf)
    srt = np.sort(th, axis=1)
    gap = np.where(np.isfinite(srt[:, 1]), srt[:, 1] - np.where(np.isfinite(srt[:, 0]), srt[:, 0], 0),
                   np.inf)
    clear = (np.abs(disc) > 1e-4).all(1) & (gap > 1e-4)
    want = np.where(np.isfinite(srt[:, 0]), np.argmin(th, axis=1), -1)
    sph_hit = want >= 0
    assert (clear & sph_hit).sum() > 2000
    assert np.array_equal(ids[clear & sph_hit], want[clear & sph_hit])
    # (binary32 intersection: the error grows as a ray nears grazing)
    np.testing.assert_allclose(t[clear & sph_hit], srt[clear & sph_hit, 0], rtol=2e-4)
    assert (clear & ~sph_hit).sum() > 2000
    assert np.all(ids[clear & ~sph_hit] >= len(sc.spheres))    # the floor, or a miss


def _euler_scipy(a, b, c):
    # extrinsic rotations about x, then y, then z: Rz(c) Ry(b) Rx(a)
    from scipy.spatial.transform import Rotation
    return Rotation.from_euler("xyz", [a, b, c]).as_matrix()


@pytest.mark.parametrize("angles", [(0.0, 0.0, math.pi / 2), (0.4, -0.7, 1.1), (-2.5, 0.3, 0.05)])
def test_mesh_rotation_equals_rotated_vertices(angles):
    # an instance rotated by (a, b, c) and translated by t must hit what the
    # static mesh with vertices R x + t (binary64, then rounded) hits; part of
    # each angle comes from a rotation binding
    rng = np.random.default_rng(7)
    v, f = S.random_triangles(rng, 400, (-0.6, -0.6, -0.6), (0.6, 0.6, 0.6), 0.15)
    t = np.array([0.2, -0.1, 0.3])
    base = np.array(angles, np.float32) - np.float32(0.25)
    X = np.full(3, 0.25, np.float32)
    ang = (base + X).astype(np.float64)       # the binary32 sums the renderer forms
    inst = S.toy_scene()
    inst.bindings = []
    m = inst.mesh(v, f, 0, translation=t, rotation=base)
    for c in range(3):
        inst.bind(S.BIND_MESH_ROT, m, c)
    R = _euler_scipy(*ang)
    flat = S.toy_scene()
    flat.bindings = []
    flat.mesh((v.astype(np.float64) @ R.T + t).astype(np.float32), f, 0)
    n = 20000
    o = np.tile(np.array([0.3, 0.2, 5.0], np.float32), (n, 1)) + rng.normal(0, 0.2, (n, 3)).astype(np.float32)
    tgt = rng.uniform(-0.9, 0.9, (n, 3)) + t
    d = tgt - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    t1, i1 = O.OracleScene(inst).trace(X, o, d)
    t2, i2 = O.OracleScene(flat).trace(np.zeros(0, np.float32), o, d)
    same = i1 == i2
    assert same.mean() > 0.995, same.mean()      # ids differ only for rays grazing an edge
    hit = same & (i1 >= 2)
    assert hit.sum() > 3000
    np.testing.assert_allclose(t1[hit], t2[hit], rtol=2e-5)


def test_rotated_plane_lambertian_closed_form():
    # a mesh square in its own z = 0 plane, rotated by a about x (through a
    # binding): the plane is n . x = 0 with n = (0, -sin a, cos a), and the
    # direct radiance is (rho / pi) I |n . (l - p)| / |l - p|^3
    sc = S.plane_scene()
    sc.quads, sc.quad_mat = [], []
    v, f = S.quad_tris((-50.0, -50.0, 0.0), (100.0, 0.0, 0.0), (0.0, 100.0, 0.0))
    m = sc.mesh(v, f, 0, rotation=(0.2, 0.0, 0.0))
    sc.bind(S.BIND_MESH_ROT, m, 0)
    X = np.array([0.15], np.float32)
    a = float(np.float32(0.2) + X[0])
    img = O.OracleScene(sc).render(X)
    o, d = camera_rays_f64(sc)
    nrm = np.array([0.0, -math.sin(a), math.cos(a)])
    tt = -(o @ nrm) / (d @ nrm)
    p = o[None, None, :] + tt[..., None] * d
    lpos = np.array(sc.plights[0][:3], np.float64)
    lv = lpos[None, None, :] - p
    r = np.linalg.norm(lv, axis=-1)
    L = sc.mat_rgb[0][0] / math.pi * sc.plights[0][3] * np.abs(lv @ nrm) / r**3
    np.testing.assert_allclose(img[..., 0], L, rtol=5e-5)
    # the same plane without the rotation is lit differently
    assert np.abs(img[..., 0] - O.OracleScene(S.plane_scene()).render([])[..., 0]).max() > 1e-2


def test_fresnel_special_values():
    n = 1.5
    assert abs(O.fresnel(1.0, 1.0, n) - ((n - 1) / (n + 1)) ** 2) < 1e-7          # 0.04
    thb = math.atan(n)                                                              # Brewster
    rs2 = ((n * n - 1) / (n * n + 1)) ** 2
    assert abs(O.fresnel(math.cos(thb), 1.0, n) - 0.5 * rs2) < 2e-6
    crit = math.asin(1 / n)
    assert O.fresnel(math.cos(crit + 0.01), n, 1.0) == 1.0                          # TIR
    assert O.fresnel(math.cos(crit - 0.05), n, 1.0) < 1.0
    assert abs(O.fresnel(1e-6, 1.0, n) - 1.0) < 1e-4                                # grazing


def test_glass_furnace_energy():
    # a dielectric sphere under unit environment neither absorbs nor emits: every
    # path that escapes within the bounce cap returns 1
    sc = S.furnace_scene(glass=True, bounces=12, spp=32, width=24, height=24)
    img = O.OracleScene(sc).render([], seed=4)
    assert img.max() <= 1.0
    assert img.mean() > 1.0 - 2e-3


def test_render_is_deterministic_and_thread_independent():
    pr = S.cornell_problem(width=48, height=48, spp=2, ico_level=2)
    sc = O.OracleScene(pr["scene"])
    a = sc.render(pr["theta0"], seed=5, nthreads=1)
    b = sc.render(pr["theta0"], seed=5, nthreads=4)
    assert np.array_equal(a, b)
    c = sc.render(pr["theta0"], seed=5, pair=1)
    assert not np.array_equal(a, c)
    r = sc.reference(pr["theta0"], seed=5)
    assert not np.array_equal(a, r)
    pix = np.array([0, 17, 48 * 20 + 7, 48 * 48 - 1], np.int32)
    np.testing.assert_array_equal(sc.render_pixels(pr["theta0"], pix, seed=5), a.reshape(-1, 3)[pix])


def _one_parameter_scene(kind):
    sc = S.toy_scene(width=32, height=32, pixel_center=1)
    if kind == "sphere-x":
        sc.bindings = sc.bindings[:1]
        return sc, 0.45, 0.3
    # the sphere replaced by a box turning about the viewing axis
    sc.bindings = []
    sc.spheres, sc.sphere_mat = [], []
    v, f = S.box_tris((0.0, 0.0, 0.0), (1.2, 0.5, 0.5), 0.0)
    m = sc.mesh(v, f, 0, translation=(0.0, 0.0, 0.35), rotation=(0.0, 0.0, 0.3))
    sc.bind(S.BIND_MESH_ROT, m, 2)
    return sc, 0.5, 0.35


@pytest.mark.parametrize("kind", ["sphere-x", "box-rotation-z"])
def test_estimator_against_quadrature_and_finite_differences(kind):
    # One-parameter toy scene (sphere x, or a box's rotation angle), pixel-centre
    # rays, direct light: the render is deterministic, so
    # Q(theta) = int kappa(x - theta) L(x) dx.  Q is evaluated by a trapezoid
    # rule on a fixed x grid, its derivative by central differences (h = 1e-3);
    # the estimator mean must match within 4 SE plus the quadrature error.
    sc, theta, sigma = _one_parameter_scene(kind)
    osc = O.OracleScene(sc)
    ref = osc.render(np.array([0.0], np.float32))

    def dQ(dx):
        xs = np.arange(theta - 6 * sigma, theta + 6 * sigma + dx / 2, dx).astype(np.float32)
        L = np.array([O.mse(osc.render(np.array([x], np.float32)), ref) for x in xs])
        x64 = xs.astype(np.float64)

        def Q(th):
            k = np.exp(-0.5 * ((x64 - th) / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
            return np.trapezoid(k * L, x64)
        h = 1e-3
        return (Q(theta + h) - Q(theta - h)) / (2 * h)

    fine, coarse = dQ(1e-3), dQ(2e-3)
    quad_err = abs(fine - coarse)
    sig32 = np.array([sigma], np.float32)
    th32 = np.array([theta], np.float32)
    for mode in (O.IS, O.GAUSS):
        P = 3000
        r = osc.grad_estimate(ref, th32, sig32, 2 * P, 77, mode)
        _, c = O.draw_tau(mode, sig32, P, 77)
        terms = c[:, 0] * (r["losses"][0::2] - r["losses"][1::2])
        se = terms.std(ddof=1) / math.sqrt(P)
        assert abs(r["grad"][0] - terms.mean()) < 1e-12
        assert abs(r["grad"][0] - fine) <= 4 * se + quad_err, (mode, r["grad"], fine, se, quad_err)
        assert abs(fine) > 6 * se     # the check has power: the gradient is not ~0

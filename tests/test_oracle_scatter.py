"""Pins of the oracle renderer's three sampling steps that a furnace cannot see:
next-event estimation of a parallelogram area light, the cosine-weighted
diffuse bounce, and refraction at a dielectric interface.  Each is checked
against closed-form optics (Lambert's polygon form factor, the cosine law's
distribution, Snell's law and the paraxial focus of a ball lens), not against
a retyped copy of the oracle's formula.  The renderer estimates the pixel
integral of Sec. 2.1 (Eq. 1-3); these are its conventions R5-R7."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2211_17263_amd import scenes as S
from tests import analytic as AN


# ---------------------------------------------------------------------------
# area light: radiance of a Lambertian point lit by a uniform parallelogram of
# radiance Le is rho Le F, with F Lambert's point-to-polygon form factor
# ---------------------------------------------------------------------------
AREA_LIGHTS = {
    "tilted": ((0.9, -0.3, 1.2), (0.0, 0.6, 0.1), (0.5, 0.0, 0.2)),
    "steep": ((-1.6, 0.2, 0.4), (0.0, 0.8, 0.0), (0.3, 0.0, 0.9)),
}


@pytest.mark.parametrize("light", sorted(AREA_LIGHTS))
def test_area_light_form_factor(light):
    o, e1, e2 = AREA_LIGHTS[light]
    sc = S.area_light_plane_scene(spp=256, light=(o, e1, e2))
    n_l = np.cross(e1, e2)
    assert n_l[2] < 0  # emits downwards, towards the plane
    osc = O.OracleScene(sc)
    K = 16
    imgs = np.stack([osc.render([], seed=100 + s)[..., 0] for s in range(K)]).astype(np.float64)
    mean = imgs.mean(0)
    se = imgs.std(0, ddof=1) / math.sqrt(K)
    pts = AN.plane_hits(sc)
    verts = AN.parallelogram(o, e1, e2)
    want = np.array([[0.7 * 5.0 * AN.polygon_form_factor(p, (0, 0, 1), verts) for p in row]
                     for row in pts], np.float64)
    # the rendered value estimates the closed form within 4 standard errors
    z = np.abs(mean - want) / np.maximum(se, 1e-12)
    assert np.all(z <= 4.0), (z.max(), mean.ravel()[:4], want.ravel()[:4])
    assert want.max() > 0.1 and np.median(se / want) < 0.02  # a sharp test


# ---------------------------------------------------------------------------
# cosine-weighted bounce: density cos(theta) / pi about the normal
# ---------------------------------------------------------------------------
def _frame(n):
    n = np.asarray(n, np.float64)
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t = np.cross(n, a)
    t /= np.linalg.norm(t)
    return t, np.cross(n, t)


@pytest.mark.parametrize("normal", [(0.0, 0.0, 1.0), (0.0, 0.0, -1.0), (0.48, -0.6, 0.64),
                                    (-0.36, 0.0, -0.8), (1.0, 0.0, 0.0)])
def test_cosine_bounce_distribution(normal):
    # under the cosine law cos^2(theta) is uniform on (0, 1) and the azimuth is
    # uniform on the circle, independently of the normal's orientation
    n = np.asarray(normal, np.float64)
    n /= np.linalg.norm(n)
    n32 = n.astype(np.float32)
    rng = np.random.default_rng(7)
    u = rng.random((4000, 2)).astype(np.float32)
    dirs = np.array([O.cosine_direction(n32, a, b) for a, b in u], np.float64)
    np.testing.assert_allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-6)
    c = dirs @ n
    assert np.all(c >= 0.0)
    assert stats.kstest(c ** 2, "uniform").pvalue > 1e-3
    t, b = _frame(n)
    phi = np.arctan2(dirs @ b, dirs @ t)
    assert stats.kstest((phi + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
    # mean cosine of the cosine law is 2/3
    assert abs(c.mean() - 2.0 / 3.0) < 4 * math.sqrt(1.0 / 18.0 / len(c))


@pytest.mark.parametrize("blocker", [((-0.3, -0.8, 1.0), (1.1, 0.0, 0.0), (0.0, 1.3, 0.0)),
                                     ((0.2, -0.1, 0.7), (2.0, 0.0, 0.0), (0.0, 0.6, 0.0))])
def test_cosine_bounce_form_factor(blocker):
    # a path escapes to the unit environment unless its bounce meets the black
    # rectangle, which a cosine-distributed bounce does with probability F:
    # pixel = rho (1 - F), a binomial mean with known standard error
    spp, rho = 2048, 0.6
    sc = S.occluded_sky_scene(spp=spp, albedo=rho, blocker=blocker)
    img = O.OracleScene(sc).render([], seed=3)[..., 0].astype(np.float64)
    verts = AN.parallelogram(*blocker)
    F = np.array([[AN.polygon_form_factor(p, (0, 0, 1), verts) for p in row]
                  for row in AN.plane_hits(sc)])
    want = np.float32(rho) * (1.0 - F)
    se = rho * np.sqrt(F * (1.0 - F) / spp)
    assert np.all(np.abs(img - want) <= 4.0 * se + 1e-6), np.abs(img - want).max()
    assert F.min() > 0.05 and F.max() < 0.95


# ---------------------------------------------------------------------------
# dielectric interface: Snell's law, mirror reflection, total internal reflection
# ---------------------------------------------------------------------------
def _random_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("ior", [1.5, 1.33, 2.4])
def test_refraction_obeys_snell(ior):
    rng = np.random.default_rng(11)
    d = _random_unit(rng, 500).astype(np.float32)
    n = _random_unit(rng, 500).astype(np.float32)
    u_refract = np.float32(1.0 - 2.0 ** -24)  # above every F < 1: refract unless TIR
    n_tested = n_tir = 0
    for di, ni in zip(d.astype(np.float64), n.astype(np.float64)):
        cos_i = -float(di @ ni)
        if abs(cos_i) < 1e-3:
            continue
        entering = cos_i > 0
        m = ni if entering else -ni             # normal against the ray
        ei, et = (1.0, ior) if entering else (ior, 1.0)
        out, side = O.dielectric_scatter(di, ni, ior, u_refract)
        out = out.astype(np.float64)
        sin_i = np.linalg.norm(np.cross(di, m))
        assert abs(np.linalg.norm(out) - 1.0) < 1e-6
        if ei * sin_i / et >= 1.0 + 1e-6:       # total internal reflection
            n_tir += 1
            np.testing.assert_allclose(out, di - 2.0 * (di @ m) * m, atol=2e-6)
            np.testing.assert_allclose(side, m, atol=1e-7)
            continue
        if ei * sin_i / et > 1.0 - 1e-4:
            continue
        n_tested += 1
        sin_t = np.linalg.norm(np.cross(out, m))
        assert abs(ei * sin_i - et * sin_t) <= 2e-6 * max(1.0, ior)     # Snell
        assert out @ m < 0                                              # crosses over
        assert abs(np.linalg.det(np.stack([di, m, out]))) < 2e-6        # plane of incidence
        # the tangential component keeps its direction
        tan_in = di - (di @ m) * m
        tan_out = out - (out @ m) * m
        if sin_i > 1e-3:
            assert tan_in @ tan_out > 0
        np.testing.assert_allclose(side, -m, atol=1e-7)
    assert n_tested > 200 and n_tir > 20


def test_reflection_branch_mirrors():
    rng = np.random.default_rng(12)
    for di, ni in zip(_random_unit(rng, 200), _random_unit(rng, 200)):
        if abs(di @ ni) < 1e-3:
            continue
        m = ni if di @ ni < 0 else -ni
        out, side = O.dielectric_scatter(di, ni, 1.5, 0.0)  # u = 0 < F: reflect
        np.testing.assert_allclose(out, di - 2.0 * (di @ m) * m, atol=2e-6)
        np.testing.assert_allclose(side, m, atol=1e-7)


def test_ball_lens_paraxial_focus():
    # rays parallel to the axis through a glass ball (n = 1.5, R = 0.5) meet
    # the axis behind it; as the ray height h -> 0 the crossing tends to the
    # paraxial focus n R / (2 (n - 1)) = 0.75 from the centre.  The rays are
    # traced with the oracle's own intersection and interface steps.
    ior, R = 1.5, 0.5
    osc = O.OracleScene(S.lens_scene(ior=ior, radius=R))
    u_refract = 1.0 - 2.0 ** -24
    hs = np.array([0.02, 0.04, 0.06, 0.08, 0.10])
    cross = []
    for h in hs:
        o = np.array([h, 0.0, 3.0])
        d = np.array([0.0, 0.0, -1.0])
        for _ in range(2):  # enter, then leave
            t, ids = osc.trace([], o.astype(np.float32), d.astype(np.float32))
            assert ids[0] == 0
            p = o + float(t[0]) * d
            ng = p / np.linalg.norm(p)
            nd, side = O.dielectric_scatter(d, ng, ior, u_refract)
            d = nd.astype(np.float64)
            o = p + side.astype(np.float64) * 1e-4
        assert d[0] < 0  # converging towards the axis
        s = -o[0] / d[0]
        cross.append(-(o[2] + s * d[2]))  # distance behind the centre
    cross = np.array(cross)
    A = np.stack([np.ones_like(hs), hs ** 2], 1)
    f0, c2 = np.linalg.lstsq(A, cross, rcond=None)[0]
    assert abs(f0 - ior * R / (2.0 * (ior - 1.0))) < 1e-3, cross
    assert c2 < 0  # marginal rays focus nearer (spherical aberration)

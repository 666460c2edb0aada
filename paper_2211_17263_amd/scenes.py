"""Seeded synthetic scene generators (inputs only).

This module builds scene descriptions as plain numpy arrays: geometry, materials,
lights, camera basis and parameter bindings.  It contains none of the estimator's
or the renderer's arithmetic; both the HIP library and the CPU oracle receive the
same arrays from here.  Random draws use numpy's PCG64 generator seeded per scene.

The paper's scenes (Cup, Shadows, Occlusion, GI, Sort, Caustic; Sec. 4.1) are not
available, so these generators are synthetic stand-ins with the sizes of the
workloads the paper's timing and hyper-parameter tables describe (Tab. 3, Tab. S1).

Conventions shared by every consumer of a scene:
  * material types: DIFFUSE (albedo rgb), DIELECTRIC (index of refraction),
    EMISSIVE (radiance rgb; only quads may be emissive, they are the area lights)
  * primitive ids: spheres first, then quads, then triangles in mesh order
  * camera: pinhole at ``eye``; ray direction before normalisation is
    fwd + sx*right + sy*up with sx, sy in [-1, 1]; ``right`` and ``up`` are
    pre-scaled by tan(fov/2)*aspect and tan(fov/2)
  * parameter binding (kind, index, component): the bound field equals its base
    value plus the parameter value.  kinds: 0 sphere centre, 1 quad origin,
    2 mesh translation, 3 point-light position, 4 material colour channel,
    5 mesh rotation angle about the x, y or z axis (radians)
  * a mesh's vertex x is placed at Rz(c) Ry(b) Rx(a) x + translation, with
    (a, b, c) its rotation angles
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

DIFFUSE, DIELECTRIC, EMISSIVE = 0, 1, 2
BIND_SPHERE, BIND_QUAD, BIND_MESH, BIND_PLIGHT, BIND_ALBEDO, BIND_MESH_ROT = 0, 1, 2, 3, 4, 5
EST_GAUSS, EST_IS, EST_IS_PERDIM = 0, 1, 2


@dataclasses.dataclass
class Mesh:
    verts: np.ndarray        # float32 [V][3]
    faces: np.ndarray        # int32 [T][3]
    material: int
    translation: np.ndarray  # float32 [3]
    rotation: np.ndarray     # float32 [3] angles (a, b, c): x -> Rz(c) Ry(b) Rx(a) x + translation


@dataclasses.dataclass
class Scene:
    width: int
    height: int
    spp: int
    max_bounces: int
    eye: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    pixel_center: int = 0
    env: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3, np.float32))
    mat_type: List[int] = dataclasses.field(default_factory=list)
    mat_rgb: List[List[float]] = dataclasses.field(default_factory=list)
    mat_ior: List[float] = dataclasses.field(default_factory=list)
    spheres: List[List[float]] = dataclasses.field(default_factory=list)   # cx cy cz r
    sphere_mat: List[int] = dataclasses.field(default_factory=list)
    quads: List[List[float]] = dataclasses.field(default_factory=list)     # origin e1 e2
    quad_mat: List[int] = dataclasses.field(default_factory=list)
    meshes: List[Mesh] = dataclasses.field(default_factory=list)
    plights: List[List[float]] = dataclasses.field(default_factory=list)   # pos, intensity rgb
    bindings: List[List[int]] = dataclasses.field(default_factory=list)    # kind index comp
    name: str = ""

    # ---- builders -------------------------------------------------------
    def material(self, kind: int, rgb=(0.0, 0.0, 0.0), ior: float = 1.0) -> int:
        self.mat_type.append(int(kind))
        self.mat_rgb.append([float(c) for c in rgb])
        self.mat_ior.append(float(ior))
        return len(self.mat_type) - 1

    def sphere(self, c, r, mat) -> int:
        self.spheres.append([float(c[0]), float(c[1]), float(c[2]), float(r)])
        self.sphere_mat.append(int(mat))
        return len(self.spheres) - 1

    def quad(self, o, e1, e2, mat) -> int:
        self.quads.append([float(v) for v in (*o, *e1, *e2)])
        self.quad_mat.append(int(mat))
        return len(self.quads) - 1

    def mesh(self, verts, faces, mat, translation=(0.0, 0.0, 0.0), rotation=(0.0, 0.0, 0.0)) -> int:
        self.meshes.append(Mesh(np.ascontiguousarray(verts, np.float32),
                                np.ascontiguousarray(faces, np.int32), int(mat),
                                np.asarray(translation, np.float32),
                                np.asarray(rotation, np.float32)))
        return len(self.meshes) - 1

    def plight(self, pos, intensity) -> int:
        self.plights.append([float(v) for v in (*pos, *intensity)])
        return len(self.plights) - 1

    def bind(self, kind, index, comp) -> int:
        self.bindings.append([int(kind), int(index), int(comp)])
        return len(self.bindings) - 1

    # ---- flat arrays -----------------------------------------------------
    @property
    def d(self) -> int:
        return len(self.bindings)

    @property
    def n_tris(self) -> int:
        return int(sum(m.faces.shape[0] for m in self.meshes))

    def arrays(self) -> dict:
        """Flat contiguous arrays; triangles are expanded to (v0, v1, v2) rows."""
        tri_rows, off = [], [0]
        for m in self.meshes:
            tri_rows.append(m.verts[m.faces].reshape(-1, 9))
            off.append(off[-1] + m.faces.shape[0])
        f32 = lambda a, w: np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1, w))
        i32 = lambda a, w: np.ascontiguousarray(np.asarray(a, np.int32).reshape(-1, w))
        return dict(
            mat_type=i32(self.mat_type, 1).ravel(), mat_rgb=f32(self.mat_rgb, 3),
            mat_ior=f32(self.mat_ior, 1).ravel(),
            spheres=f32(self.spheres, 4), sphere_mat=i32(self.sphere_mat, 1).ravel(),
            quads=f32(self.quads, 9), quad_mat=i32(self.quad_mat, 1).ravel(),
            tris=(np.ascontiguousarray(np.concatenate(tri_rows), np.float32)
                  if tri_rows else np.zeros((0, 9), np.float32)),
            mesh_off=np.asarray(off, np.int32),
            mesh_mat=i32([m.material for m in self.meshes], 1).ravel(),
            mesh_xlate=f32([m.translation for m in self.meshes], 3),
            mesh_rot=f32([m.rotation for m in self.meshes], 3),
            plights=f32(self.plights, 6), bindings=i32(self.bindings, 3),
        )



def camera_basis(eye, look, up, vfov_deg, width, height):
    """Pinhole camera vectors, computed in float64 and stored as float32."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(look, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(vfov_deg) * 0.5)
    aspect = width / height
    return (eye.astype(np.float32), f.astype(np.float32),
            (r * th * aspect).astype(np.float32), (u * th).astype(np.float32))


def _new_scene(name, width, height, spp, bounces, eye, look, up=(0, 1, 0), fov=40.0, **kw):
    e, f, r, u = camera_basis(eye, look, up, fov, width, height)
    return Scene(width=width, height=height, spp=spp, max_bounces=bounces,
                 eye=e, fwd=f, right=r, up=u, name=name, **kw)


# ---------------------------------------------------------------------------
# geometry helpers
# ---------------------------------------------------------------------------
def icosphere(level: int):
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache, nf = {}, []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return np.array(v, np.float64), np.array(f, np.int32)


def jittered_icosphere(rng, level, radius, center, jitter=0.15):
    v, f = icosphere(level)
    s = 1.0 + rng.uniform(-jitter, jitter, size=(v.shape[0], 1))
    return (v * s * radius + np.asarray(center, np.float64)).astype(np.float32), f


def quad_tris(o, e1, e2):
    o, e1, e2 = (np.asarray(x, np.float64) for x in (o, e1, e2))
    v = np.stack([o, o + e1, o + e1 + e2, o + e2]).astype(np.float32)
    return v, np.array([[0, 1, 2], [0, 2, 3]], np.int32)


def box_tris(center, size, rot_y_deg):
    c, h = np.asarray(center, np.float64), np.asarray(size, np.float64) * 0.5
    a = math.radians(rot_y_deg)
    R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                       np.float64) * h
    v = (corners @ R.T + c).astype(np.float32)
    # outward winding is irrelevant (diffuse surfaces are two-sided)
    f = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                  [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]], np.int32)
    return v, f


def random_triangles(rng, n, lo, hi, half_extent):
    c = rng.uniform(lo, hi, size=(n, 1, 3))
    v = c + rng.uniform(-half_extent, half_extent, size=(n, 3, 3))
    return v.reshape(-1, 3).astype(np.float32), np.arange(3 * n, dtype=np.int32).reshape(n, 3)


# ---------------------------------------------------------------------------
# workload 1: toy direct-light scene (sphere position over a plane, point light)
# ---------------------------------------------------------------------------
def toy_scene(width=64, height=64, spp=1, light=(1.5, 1.5, 3.0), pixel_center=0,
              bounces=0, intensity=10.0):
    s = _new_scene("toy", width, height, spp, bounces, eye=(0, 0, 5), look=(0, 0, 0),
                   up=(0, 1, 0), fov=40.0, pixel_center=pixel_center)
    ground = s.material(DIFFUSE, (0.8, 0.8, 0.8))
    red = s.material(DIFFUSE, (0.8, 0.3, 0.2))
    sph = s.sphere((0.0, 0.0, 0.5), 0.5, red)
    s.quad((-10.0, -10.0, 0.0), (20.0, 0.0, 0.0), (0.0, 20.0, 0.0), ground)
    s.plight(light, (intensity,) * 3)
    s.bind(BIND_SPHERE, sph, 0)
    s.bind(BIND_SPHERE, sph, 1)
    return s


def plateau_scene(width=64, height=64, spp=1, fov=60.0):
    """The circle-position plateau of Sec. 2.1: the toy camera and sphere
    (theta = sphere (x, y)), no ground and no lights, so the sphere renders
    black over a constant unit environment and its appearance does not depend
    on its position.  Moving it without overlapping its reference position
    leaves the image loss unchanged.  The 60 degree field of view is the wider
    view the paper's bandwidth study uses so that perturbed positions stay in
    the frame (with 40 degrees, leaving the frame also lowers the loss)."""
    s = _new_scene("plateau", width, height, spp, 0, eye=(0, 0, 5), look=(0, 0, 0),
                   up=(0, 1, 0), fov=fov, env=np.ones(3, np.float32))
    dark = s.material(DIFFUSE, (0.8, 0.3, 0.2))
    sph = s.sphere((0.0, 0.0, 0.5), 0.5, dark)
    s.bind(BIND_SPHERE, sph, 0)
    s.bind(BIND_SPHERE, sph, 1)
    return s


def toy_problem(seed=1, **kw):
    """Toy workload: theta = sphere (x, y); theta_ref = (0, 0); theta_0 ~ U[-1,1]^2."""
    rng = np.random.default_rng(seed)
    return dict(scene=toy_scene(**kw), theta_ref=np.zeros(2, np.float32),
                theta0=rng.uniform(-1, 1, 2).astype(np.float32),
                sigma=np.full(2, 0.5, np.float32), N=4, est=EST_GAUSS)


# ---------------------------------------------------------------------------
# workload 2: Cornell-style box, movable area light + two jittered icospheres
# ---------------------------------------------------------------------------
def cornell_scene(seed=2, width=256, height=256, spp=16, bounces=4, ico_level=4, colour=False,
                  rotation=False):
    """Cornell box; binds the area light's position (3) and the yellow sphere's
    translation (3), with colour=True also the left wall's albedo (3), and with
    rotation=True the tall box's turn about the vertical axis (1; the box is
    then an instance built around its own centre)."""
    rng = np.random.default_rng(seed)
    s = _new_scene("cornell", width, height, spp, bounces, eye=(0, 0, 3.4), look=(0, 0, 0))
    white = s.material(DIFFUSE, (0.73, 0.73, 0.73))
    red = s.material(DIFFUSE, (0.63, 0.065, 0.05))
    green = s.material(DIFFUSE, (0.14, 0.45, 0.091))
    yellow = s.material(DIFFUSE, (0.8, 0.75, 0.2))
    blue = s.material(DIFFUSE, (0.2, 0.45, 0.8))
    light = s.material(EMISSIVE, (15.0, 15.0, 15.0))
    # area light: 0.5 x 0.5 below the ceiling, facing down (e1 x e2 = -y)
    lq = s.quad((-0.25, 0.99, -0.25), (0.5, 0.0, 0.0), (0.0, 0.0, 0.5), light)
    walls = [((-1, -1, -1), (2, 0, 0), (0, 0, 2), white),   # floor
             ((-1, 1, -1), (2, 0, 0), (0, 0, 2), white),    # ceiling
             ((-1, -1, -1), (2, 0, 0), (0, 2, 0), white),   # back
             ((-1, -1, -1), (0, 0, 2), (0, 2, 0), red),     # left
             ((1, -1, -1), (0, 0, 2), (0, 2, 0), green)]    # right
    for o, e1, e2, m in walls:
        v, f = quad_tris(o, e1, e2)
        s.mesh(v, f, m)
    if rotation:
        v, f = box_tris((0.0, 0.0, 0.0), (0.55, 0.6, 0.55), 0.0)
        box = s.mesh(v, f, white, translation=(0.35, -0.7, 0.25),
                     rotation=(0.0, math.radians(18.0), 0.0))
    else:
        v, f = box_tris((0.35, -0.7, 0.25), (0.55, 0.6, 0.55), 18.0)
        s.mesh(v, f, white)
    va, fa = jittered_icosphere(rng, ico_level, 0.2, (-0.45, -0.55, -0.15))
    mesh_a = s.mesh(va, fa, yellow)
    vb, fb = jittered_icosphere(rng, ico_level, 0.2, (0.35, -0.15, 0.25))
    s.mesh(vb, fb, blue)
    for c in range(3):
        s.bind(BIND_QUAD, lq, c)
    for c in range(3):
        s.bind(BIND_MESH, mesh_a, c)
    if colour:
        for c in range(3):
            s.bind(BIND_ALBEDO, red, c)
    if rotation:
        s.bind(BIND_MESH_ROT, box, 1)
    return s


def cornell_problem(seed=2, colour=False, rotation=False, **kw):
    """Geometry (light position, sphere translation); with colour=True the left
    wall's colour as offsets from its initial albedo (theta_0's); with
    rotation=True the tall box's turn (radians) about the vertical axis."""
    rng = np.random.default_rng(seed + 1000)
    scene = cornell_scene(seed=seed, colour=colour, rotation=rotation, **kw)
    theta_ref = np.array([rng.uniform(-0.3, 0.3), -0.02, rng.uniform(-0.3, 0.3),
                          rng.uniform(-0.2, 0.2), 0.0, rng.uniform(-0.2, 0.2)], np.float32)
    offs = rng.uniform(-0.5, 0.5, 6)
    offs[1] = -abs(offs[1]) * 0.6      # keep the light below the ceiling at theta_0
    theta0 = (theta_ref + offs).astype(np.float32)
    sigma = np.full(6, 0.3, np.float32)
    if colour:
        base = np.array(scene.mat_rgb[1], np.float64)       # the red wall
        target = rng.uniform(0.1, 0.9, 3)
        theta_ref = np.concatenate([theta_ref, target - base]).astype(np.float32)
        theta0 = np.concatenate([theta0, np.zeros(3)]).astype(np.float32)
        sigma = np.concatenate([sigma, np.full(3, 0.2)]).astype(np.float32)
    if rotation:
        theta_ref = np.append(theta_ref, rng.uniform(-0.5, 0.5)).astype(np.float32)
        theta0 = np.append(theta0, 0.0).astype(np.float32)
        sigma = np.append(sigma, 0.3).astype(np.float32)
    return dict(scene=scene, theta_ref=theta_ref, theta0=theta0, sigma=sigma, N=16, est=EST_IS)


# ---------------------------------------------------------------------------
# workload 3: caustic scene (glass sphere, area light, random-triangle occluder)
# ---------------------------------------------------------------------------
def caustic_scene(seed=3, width=512, height=512, spp=64, bounces=8, n_occluders=50000):
    rng = np.random.default_rng(seed)
    s = _new_scene("caustic", width, height, spp, bounces, eye=(0.0, 2.6, 3.6),
                   look=(0.0, 0.2, 0.0))
    floor = s.material(DIFFUSE, (0.8, 0.8, 0.8))
    glass = s.material(DIELECTRIC, ior=1.5)
    occl = s.material(DIFFUSE, (0.5, 0.5, 0.5))
    light = s.material(EMISSIVE, (40.0, 40.0, 40.0))
    sph = s.sphere((0.0, 0.0, 0.0), 0.5, glass)
    s.quad((-4.0, 0.0, -4.0), (0.0, 0.0, 8.0), (8.0, 0.0, 0.0), floor)
    # light centred at (-1.5, 2.5, 0), tilted to face the sphere
    n = np.array([1.5, -2.0, 0.0])
    n /= np.linalg.norm(n)
    e1 = np.array([0.0, 0.0, 0.5])
    e2 = np.cross(n, e1)             # so that e1 x e2 points along n
    e2 = e2 / np.linalg.norm(e2) * 0.5
    o = np.array([-1.5, 2.5, 0.0]) - 0.5 * e1 - 0.5 * e2
    if np.dot(np.cross(e1, e2), n) < 0:
        e1, e2 = e2, e1
        o = np.array([-1.5, 2.5, 0.0]) - 0.5 * e1 - 0.5 * e2
    s.quad(o, e1, e2, light)
    if n_occluders:
        v, f = random_triangles(rng, n_occluders, (-3.0, 1.2, -1.6), (-1.1, 1.9, 1.6), 0.03)
        s.mesh(v, f, occl)
    for c in range(3):
        s.bind(BIND_SPHERE, sph, c)
    return s


def caustic_problem(seed=3, **kw):
    rng = np.random.default_rng(seed + 1000)
    scene = caustic_scene(seed=seed, **kw)
    theta_ref = np.array([0.3, 0.5, 0.2], np.float32)
    theta0 = (theta_ref + np.array([rng.uniform(-0.8, 0.8), rng.uniform(0.0, 0.4),
                                    rng.uniform(-0.8, 0.8)])).astype(np.float32)
    return dict(scene=scene, theta_ref=theta_ref, theta0=theta0,
                sigma=np.full(3, 1.0, np.float32), N=32, est=EST_IS,
                sigma_end=0.05, steps=200, lr=0.01)


# ---------------------------------------------------------------------------
# many objects: Sort-like stand-in (75 objects, two coordinates each)
# ---------------------------------------------------------------------------
def sort_scene(n_objects=75, width=128, height=128, spp=4, bounces=2, radius=0.1, spacing=0.33,
               n_colours=15, seed=5):
    """n_objects coloured diffuse spheres on a floor on a square grid, lit by an
    area light, seen from above at an angle; binds each sphere's x and z (the
    floor-plane coordinates), so d = 2 n_objects (150 for the default 75)."""
    rng = np.random.default_rng(seed)
    s = _new_scene("sort", width, height, spp, bounces, eye=(0.0, 4.2, 2.6), look=(0, 0, 0),
                   fov=45.0)
    floor = s.material(DIFFUSE, (0.7, 0.7, 0.7))
    light = s.material(EMISSIVE, (12.0, 12.0, 12.0))
    colours = [s.material(DIFFUSE, tuple(rng.uniform(0.1, 0.9, 3))) for _ in range(n_colours)]
    s.quad((-4.0, 0.0, -4.0), (0.0, 0.0, 8.0), (8.0, 0.0, 0.0), floor)
    s.quad((-0.75, 3.0, -0.75), (1.5, 0.0, 0.0), (0.0, 0.0, 1.5), light)
    side = int(math.ceil(math.sqrt(n_objects)))
    spheres = []
    for i in range(n_objects):
        gx, gz = i % side, i // side
        x = (gx - 0.5 * (side - 1)) * spacing
        z = (gz - 0.5 * (side - 1)) * spacing
        spheres.append(s.sphere((x, radius, z), radius, colours[i % n_colours]))
    for i in spheres:
        s.bind(BIND_SPHERE, i, 0)
        s.bind(BIND_SPHERE, i, 2)
    return s


def sort_problem(seed=5, n_objects=75, offset=0.12, **kw):
    """Recover every object's floor position from offsets of up to `offset` in
    each coordinate (d = 2 n_objects)."""
    rng = np.random.default_rng(seed + 1000)
    scene = sort_scene(n_objects=n_objects, seed=seed, **kw)
    d = scene.d
    theta_ref = np.zeros(d, np.float32)
    theta0 = rng.uniform(-offset, offset, d).astype(np.float32)
    return dict(scene=scene, theta_ref=theta_ref, theta0=theta0,
                sigma=np.full(d, 0.05, np.float32), N=16, est=EST_IS)


# ---------------------------------------------------------------------------
# workload 4: many uneven scenes (batched estimation)
# ---------------------------------------------------------------------------
def random_job_scene(rng, side, n_tris, spp, bounces):
    s = _new_scene("job", side, side, spp, bounces, eye=(0.0, 2.0, 4.0), look=(0, 0.3, 0),
                   fov=45.0)
    floor = s.material(DIFFUSE, (0.75, 0.75, 0.75))
    red = s.material(DIFFUSE, tuple(rng.uniform(0.2, 0.9, 3)))
    occl = s.material(DIFFUSE, (0.5, 0.5, 0.5))
    ico_m = s.material(DIFFUSE, tuple(rng.uniform(0.2, 0.9, 3)))
    light = s.material(EMISSIVE, (30.0, 30.0, 30.0))
    sph = s.sphere((rng.uniform(-0.5, 0.5), 0.4, rng.uniform(-0.5, 0.5)), 0.4, red)
    s.quad((-4.0, 0.0, -4.0), (0.0, 0.0, 8.0), (8.0, 0.0, 0.0), floor)
    lq = s.quad((-0.3, 2.5, -0.3), (0.6, 0.0, 0.0), (0.0, 0.0, 0.6), light)
    n_ico = 1280 if n_tris >= 2560 else 320
    level = 3 if n_ico == 1280 else 2
    n_rand = max(0, n_tris - n_ico)
    v, f = random_triangles(rng, n_rand, (-1.5, 1.3, -1.5), (1.5, 1.8, 1.5), 0.03)
    occ_mesh = s.mesh(v, f, occl)
    vi, fi = jittered_icosphere(rng, level, 0.3, (rng.uniform(-1, 1), 0.3, rng.uniform(-1, 1)))
    ico_mesh = s.mesh(vi, fi, ico_m)
    fields = ([(BIND_SPHERE, sph, c) for c in range(3)] + [(BIND_QUAD, lq, c) for c in range(3)]
              + [(BIND_MESH, occ_mesh, c) for c in range(3)]
              + [(BIND_MESH, ico_mesh, c) for c in range(3)])
    return s, fields


def batch_jobs(seed=4, n_jobs=64, max_side=512, max_tris=200000):
    """Uneven jobs: side in {64..512}, 1k-200k triangles (log-uniform), d in [2, 12],
    N in {4, 8, 16, 32}, spp in {1, 4, 16}, bounces in {1, 2, 4}, sigma ~ U[0.1, 0.5]."""
    rng = np.random.default_rng(seed)
    sides = [s for s in (64, 128, 256, 512) if s <= max_side]
    jobs = []
    for j in range(n_jobs):
        side = int(rng.choice(sides))
        n_tris = int(round(math.exp(rng.uniform(math.log(1000), math.log(max_tris)))))
        spp = int(rng.choice([1, 4, 16]))
        bounces = int(rng.choice([1, 2, 4]))
        scene, fields = random_job_scene(rng, side, n_tris, spp, bounces)
        d = int(rng.integers(2, 13))
        order = rng.permutation(len(fields))[:d]
        for idx in order:
            scene.bind(*fields[idx])
        sig = float(rng.uniform(0.1, 0.5))
        theta_ref = np.zeros(d, np.float32)
        theta0 = rng.uniform(-0.3, 0.3, d).astype(np.float32)
        jobs.append(dict(scene=scene, theta_ref=theta_ref, theta0=theta0,
                         sigma=np.full(d, sig, np.float32),
                         N=int(rng.choice([4, 8, 16, 32])),
                         est=int(rng.choice([EST_GAUSS, EST_IS])), seed=int(rng.integers(1, 2**62))))
    return jobs


# ---------------------------------------------------------------------------
# randomised small scenes (every primitive, material and parameter kind)
# ---------------------------------------------------------------------------
def random_scene(seed):
    """A small scene drawn from seed: a floor, 0-3 spheres (diffuse or glass),
    0-1 area light, 0-2 point lights, 1-2 meshes (triangle cloud or box, turned
    and moved), a random environment, and 1-8 parameters of random kinds
    (sphere centre, quad origin, mesh translation, mesh angle, point-light
    position, material colour).  Returns (scene, theta_ref, theta0, sigma)."""
    rng = np.random.default_rng(seed)
    W, H = int(rng.integers(5, 41)), int(rng.integers(5, 41))
    s = _new_scene("random", W, H, int(rng.integers(1, 5)), int(rng.integers(0, 4)),
                   eye=(0.3, 1.6, 3.2), look=(0.0, 0.2, 0.0), fov=float(rng.uniform(35, 60)),
                   pixel_center=int(rng.integers(0, 2)))
    s.env = np.asarray(rng.uniform(0.0, 0.3, 3), np.float32)
    floor = s.material(DIFFUSE, tuple(rng.uniform(0.2, 0.9, 3)))
    s.quad((-3.0, 0.0, -3.0), (0.0, 0.0, 6.0), (6.0, 0.0, 0.0), floor)
    fields = []
    for _ in range(int(rng.integers(0, 4))):
        glass = rng.random() < 0.3
        m = s.material(DIELECTRIC, ior=1.5) if glass else s.material(DIFFUSE, tuple(rng.uniform(0.1, 0.9, 3)))
        i = s.sphere(tuple(rng.uniform([-1.0, 0.2, -1.0], [1.0, 0.8, 1.0])), float(rng.uniform(0.1, 0.4)), m)
        fields += [(BIND_SPHERE, i, c) for c in range(3)]
        if not glass:
            fields.append((BIND_ALBEDO, m, int(rng.integers(0, 3))))
    if rng.random() < 0.7:
        lm = s.material(EMISSIVE, tuple(rng.uniform(5.0, 20.0, 3)))
        lq = s.quad((-0.4, 2.2, -0.4), (0.8, 0.0, 0.0), (0.0, 0.0, 0.8), lm)
        fields += [(BIND_QUAD, lq, c) for c in range(3)] + [(BIND_ALBEDO, lm, 1)]
    for _ in range(int(rng.integers(0, 3))):
        pl = s.plight(tuple(rng.uniform([-1.5, 1.0, -1.5], [1.5, 2.5, 1.5])), tuple(rng.uniform(2.0, 8.0, 3)))
        fields += [(BIND_PLIGHT, pl, c) for c in range(3)]
    for _ in range(int(rng.integers(1, 3))):
        mm = s.material(DIFFUSE, tuple(rng.uniform(0.1, 0.9, 3)))
        if rng.random() < 0.5:
            v, f = random_triangles(rng, int(rng.integers(20, 400)), (-0.4, -0.3, -0.4), (0.4, 0.3, 0.4), 0.08)
        else:
            v, f = box_tris((0.0, 0.0, 0.0), tuple(rng.uniform(0.2, 0.6, 3)), 0.0)
        mesh = s.mesh(v, f, mm, translation=tuple(rng.uniform([-1.0, 0.3, -1.0], [1.0, 0.7, 1.0])),
                      rotation=tuple(rng.uniform(-1.0, 1.0, 3)) if rng.random() < 0.6 else (0.0, 0.0, 0.0))
        fields += [(BIND_MESH, mesh, c) for c in range(3)] + [(BIND_MESH_ROT, mesh, c) for c in range(3)]
    if not fields:
        fields.append((BIND_ALBEDO, floor, 0))
    order = rng.permutation(len(fields))[: int(rng.integers(1, min(8, len(fields)) + 1))]
    for idx in order:
        s.bind(*fields[idx])
    d = s.d
    theta_ref = np.zeros(d, np.float32)
    theta0 = rng.uniform(-0.15, 0.15, d).astype(np.float32)
    sigma = rng.uniform(0.05, 0.3, d).astype(np.float32)
    return s, theta_ref, theta0, sigma


# ---------------------------------------------------------------------------
# scenes used by closed-form checks
# ---------------------------------------------------------------------------
def furnace_scene(albedo=0.6, width=32, height=32, spp=4, bounces=2, glass=False):
    """Convex sphere under constant unit environment radiance, no lights."""
    s = _new_scene("furnace", width, height, spp, bounces, eye=(0, 0, 3), look=(0, 0, 0),
                   env=np.ones(3, np.float32))
    m = s.material(DIELECTRIC, ior=1.5) if glass else s.material(DIFFUSE, (albedo,) * 3)
    s.sphere((0.0, 0.0, 0.0), 0.8, m)
    return s


def plane_scene(width=32, height=32, light=(0.3, -0.2, 2.0), intensity=7.0, albedo=0.5):
    """Lambertian plane z=0 lit by one point light, pixel-centre rays, direct only."""
    s = _new_scene("plane", width, height, 1, 0, eye=(0.2, 0.1, 4.0), look=(0, 0, 0),
                   pixel_center=1)
    m = s.material(DIFFUSE, (albedo,) * 3)
    s.quad((-50.0, -50.0, 0.0), (100.0, 0.0, 0.0), (0.0, 100.0, 0.0), m)
    s.plight(light, (intensity,) * 3)
    return s


def area_light_plane_scene(width=8, height=8, spp=256, albedo=0.7, radiance=5.0,
                           light=((0.9, -0.3, 1.2), (0.0, 0.6, 0.1), (0.5, 0.0, 0.2))):
    """Lambertian plane z=0 lit by one tilted parallelogram emitter (origin,
    edge1, edge2; it emits along edge1 x edge2, downwards) outside the camera's
    view; pixel-centre rays, direct lighting only."""
    s = _new_scene("area-plane", width, height, spp, 0, eye=(0.0, 0.0, 3.0), look=(0, 0, 0),
                   pixel_center=1)
    m = s.material(DIFFUSE, (albedo,) * 3)
    s.quad((-10.0, -10.0, 0.0), (20.0, 0.0, 0.0), (0.0, 20.0, 0.0), m)
    e = s.material(EMISSIVE, (radiance,) * 3)
    s.quad(light[0], light[1], light[2], e)
    return s


def occluded_sky_scene(width=8, height=8, spp=2048, albedo=0.6,
                       blocker=((-0.3, -0.8, 1.0), (1.1, 0.0, 0.0), (0.0, 1.3, 0.0))):
    """Lambertian plane z=0 under a constant unit environment with a black
    (albedo 0) rectangle above it; one bounce, no lights.  A camera below the
    rectangle looks straight down, so a pixel-centre path returns the albedo
    when its bounce escapes and 0 when the bounce meets the rectangle."""
    s = _new_scene("occluded-sky", width, height, spp, 1, eye=(0.0, 0.0, 0.6), look=(0, 0, 0),
                   fov=30.0, pixel_center=1, env=np.ones(3, np.float32))
    m = s.material(DIFFUSE, (albedo,) * 3)
    s.quad((-10.0, -10.0, 0.0), (20.0, 0.0, 0.0), (0.0, 20.0, 0.0), m)
    k = s.material(DIFFUSE, (0.0, 0.0, 0.0))
    s.quad(blocker[0], blocker[1], blocker[2], k)
    return s


def lens_scene(ior=1.5, radius=0.5):
    """A glass sphere at the origin (for tracing rays through it)."""
    s = _new_scene("lens", 8, 8, 1, 8, eye=(0.0, 0.0, 3.0), look=(0, 0, 0))
    m = s.material(DIELECTRIC, ior=ior)
    s.sphere((0.0, 0.0, 0.0), radius, m)
    return s


def deep_stack_scene(seed=6, n_tris=524288, width=48, height=40, spp=2, bounces=1):
    """Many long, thin triangles overlapping across the whole view in a slab
    (z in [-0.5, 0.5]): their BVH is deep and a ray meets most boxes, so
    traversal keeps up to three siblings per level on its stack.  A diffuse
    floor below and a point light; the parameters translate the mesh in x, y."""
    rng = np.random.default_rng(seed)
    s = _new_scene("deep-stack", width, height, spp, bounces, eye=(0.0, 0.0, 3.0), look=(0, 0, 0))
    floor = s.material(DIFFUSE, (0.7, 0.7, 0.7))
    m = s.material(DIFFUSE, (0.6, 0.4, 0.3))
    s.quad((-10.0, -10.0, -1.0), (20.0, 0.0, 0.0), (0.0, 20.0, 0.0), floor)
    z = rng.uniform(-0.5, 0.5, n_tris)
    x, y = rng.uniform(-1, 1, n_tris), rng.uniform(-1, 1, n_tris)
    dx, dy = rng.uniform(-1, 1, n_tris), rng.uniform(-1, 1, n_tris)
    v = np.stack([np.stack([x - dx, y - dy, z], 1), np.stack([x + dx, y + dy, z + 0.001], 1),
                  np.stack([x + 0.002, y, z], 1)], 1).astype(np.float32)
    s.mesh(v.reshape(-1, 3), np.arange(3 * n_tris, dtype=np.int32).reshape(-1, 3), m)
    s.plight((0.5, 0.8, 2.5), (6.0, 6.0, 6.0))
    s.bind(BIND_MESH, 0, 0)
    s.bind(BIND_MESH, 0, 1)
    return s


def dp_scene(width=32, height=32, spp=1, eye=(0.0, 0.0, 5.0), look=(0.0, 0.0, 0.0), fov=40.0,
             sphere=(0.0, 0.0, 0.5), radius=0.5, albedo=(0.8, 0.3, 0.2), light=(1.5, 1.5, 3.0),
             ground=((-10.0, -10.0, 0.0), (20.0, 0.0, 0.0), (0.0, 20.0, 0.0)), env=(0.0, 0.0, 0.0),
             pixel_center=0):
    """The toy workload's kind of scene for the differentiable renderer: one
    diffuse sphere whose centre (x, y) are the parameters, one diffuse ground
    quad, one point light, direct light only; camera, sphere colour, light,
    ground placement and environment are arguments (the renderer's tests use
    them to isolate its interior, silhouette and shadow terms)."""
    s = _new_scene("dp", width, height, spp, 0, eye=eye, look=look, up=(0, 1, 0), fov=fov,
                   pixel_center=pixel_center, env=np.asarray(env, np.float32))
    g = s.material(DIFFUSE, (0.8, 0.8, 0.8))
    m = s.material(DIFFUSE, albedo)
    sph = s.sphere(sphere, radius, m)
    s.quad(ground[0], ground[1], ground[2], g)
    s.plight(light, (10.0, 10.0, 10.0))
    s.bind(BIND_SPHERE, sph, 0)
    s.bind(BIND_SPHERE, sph, 1)
    return s

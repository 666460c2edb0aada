"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark import
this module.  It marshals scene arrays from the shared input generators into the
oracle's own C structure and calls the oracle; it contains no renderer or
estimator arithmetic of its own.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PRDPT_ORACLE_LIB names another build of oracle.c (the mutation checks of the
# pins load deliberately broken copies this way, each in its own process)
LIB_PATH = os.environ.get("PRDPT_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

GAUSS, IS, IS_PERDIM = 0, 1, 2
INDEPENDENT = 0x100          # or-ed into a mode: no antithetic partners (noAT)
STRATIFIED = 0x200           # or-ed into an independent mode: stratified first uniforms
TAG_TAU, TAG_PATH, TAG_REF = 1, 2, 3

_lib = None


def use_library(path):
    """Load the oracle from another build of oracle.c (e.g. the host-tuned one
    the benchmark times); only before the oracle has been used."""
    global LIB_PATH
    if _lib is not None and path != LIB_PATH:
        raise RuntimeError("the oracle library is already loaded")
    LIB_PATH = path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b  # noqa: WPS433
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")


class SceneIn(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("fwd", C.c_float * 3), ("right", C.c_float * 3),
                ("up", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32), ("spp", C.c_int32),
                ("max_bounces", C.c_int32), ("pixel_center", C.c_int32),
                ("env", C.c_float * 3),
                ("n_mat", C.c_int32), ("mat_type", C.c_void_p), ("mat_rgb", C.c_void_p),
                ("mat_ior", C.c_void_p),
                ("n_sph", C.c_int32), ("sph", C.c_void_p), ("sph_mat", C.c_void_p),
                ("n_quad", C.c_int32), ("quad", C.c_void_p), ("quad_mat", C.c_void_p),
                ("n_mesh", C.c_int32), ("mesh_off", C.c_void_p), ("mesh_mat", C.c_void_p),
                ("mesh_xlate", C.c_void_p),
                ("n_tri", C.c_int32), ("tri", C.c_void_p),
                ("n_plight", C.c_int32), ("plight", C.c_void_p),
                ("n_param", C.c_int32), ("binding", C.c_void_p), ("mesh_rot", C.c_void_p)]


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_u01.argtypes = [C.c_uint32]
    L.orc_u01.restype = C.c_float
    L.orc_ln.argtypes = [C.c_float]
    L.orc_ln.restype = C.c_float
    L.orc_sincos_2pi.argtypes = [C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.orc_chi_mean.argtypes = [C.c_int]
    L.orc_chi_mean.restype = C.c_double
    L.orc_draw_tau.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, _f32p, _f32p, _f64p]
    L.orc_combine.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p, C.POINTER(C.c_double)]
    L.orc_combine_independent.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p,
                                          C.POINTER(C.c_double)]
    L.orc_scene_new.argtypes = [C.POINTER(SceneIn)]
    L.orc_scene_new.restype = C.c_void_p
    L.orc_scene_free.argtypes = [C.c_void_p]
    L.orc_set_brute_force.argtypes = [C.c_void_p, C.c_int]
    L.orc_trace.argtypes = [C.c_void_p, _f32p, C.c_int, _f32p, _f32p, _f32p, _i32p]
    L.orc_render.argtypes = [C.c_void_p, _f32p, C.c_int, C.c_int, C.c_uint64, C.c_int, _f32p]
    L.orc_render_pixels.argtypes = [C.c_void_p, _f32p, C.c_int, C.c_int, C.c_uint64, C.c_int,
                                    _i32p, C.c_int, _f32p]
    L.orc_mse.argtypes = [_f32p, _f32p, C.c_int]
    L.orc_mse.restype = C.c_double
    L.orc_grad_estimate.argtypes = [C.c_void_p, _f32p, _f32p, _f32p, C.c_int, C.c_uint64,
                                    C.c_int, C.c_int, _f64p, C.POINTER(C.c_double), _f64p,
                                    _f32p]
    L.orc_smoothed_loss.argtypes = [C.c_void_p, _f32p, _f32p, _f32p, C.c_int, C.c_uint64,
                                    C.c_int, C.POINTER(C.c_double)]
    L.orc_render_perturbed.argtypes = [C.c_void_p, _f32p, _f32p, C.c_int, C.c_uint64, C.c_int,
                                       C.c_int, _f32p, _f32p]
    L.orc_fresnel.argtypes = [C.c_float, C.c_float, C.c_float]
    L.orc_fresnel.restype = C.c_float
    L.orc_cosine_direction.argtypes = [_f32p, C.c_float, C.c_float, _f32p]
    L.orc_dielectric_scatter.argtypes = [_f32p, _f32p, C.c_float, C.c_float, _f32p, _f32p]
    L.orc_dp_image_derivative.argtypes = [C.c_void_p, _f32p, C.c_int, C.c_uint64, C.c_int, C.c_int,
                                          C.c_int, _f64p]
    L.orc_dp_grad_estimate.argtypes = [C.c_void_p, _f32p, _f32p, _f32p, C.c_int, C.c_uint64,
                                       C.c_int, C.c_int, _f64p, C.POINTER(C.c_double), _f64p]
    L.orc_sigma_schedule.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
    L.orc_sigma_schedule.restype = C.c_double
    L.orc_adam_step.argtypes = [C.c_int, _f64p, _f64p, _f64p, _f64p, C.c_int, C.c_double,
                                C.c_double, C.c_double, C.c_double]


def _f32(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, np.float32))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


# --- generator and sample transforms ------------------------------------------
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def u01(x):
    return lib().orc_u01(int(x))


def ln(x):
    return lib().orc_ln(float(x))


def sincos_2pi(u):
    s, c = C.c_float(), C.c_float()
    lib().orc_sincos_2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def chi_mean(d):
    return lib().orc_chi_mean(int(d))


def fresnel(cos_i, eta_i, eta_t):
    return lib().orc_fresnel(float(cos_i), float(eta_i), float(eta_t))


def cosine_direction(n, u1, u2):
    """The renderer's cosine-weighted bounce direction about unit normal n."""
    out = np.zeros(3, np.float32)
    lib().orc_cosine_direction(_f32(n, 3), float(u1), float(u2), out)
    return out


def dielectric_scatter(d, ng, ior, u):
    """The renderer's dielectric interface step: (new direction, offset side)."""
    out = np.zeros(3, np.float32)
    side = np.zeros(3, np.float32)
    lib().orc_dielectric_scatter(_f32(d, 3), _f32(ng, 3), float(ior), float(u), out, side)
    return out, side


def draw_tau(mode, sigma, P, seed):
    sigma = _f32(sigma)
    d = sigma.size
    tau = np.zeros((P, d), np.float32)
    c = np.zeros((P, d), np.float64)
    rc = lib().orc_draw_tau(int(mode), d, int(P), int(seed), sigma, tau, c)
    if rc:
        raise ValueError("invalid draw_tau arguments")
    return tau, c


def combine(c, L):
    c = np.ascontiguousarray(c, np.float64)
    L = np.ascontiguousarray(L, np.float64)
    P, d = c.shape
    g = np.zeros(d, np.float64)
    q = C.c_double()
    lib().orc_combine(P, d, c, L, g, C.byref(q))
    return g, q.value


def combine_independent(c, L):
    c = np.ascontiguousarray(c, np.float64)
    L = np.ascontiguousarray(L, np.float64)
    N, d = c.shape
    g = np.zeros(d, np.float64)
    q = C.c_double()
    lib().orc_combine_independent(N, d, c, L, g, C.byref(q))
    return g, q.value


def sigma_schedule(sigma0, sigma_end, t, T):
    return lib().orc_sigma_schedule(sigma0, sigma_end, t, T)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    lib().orc_adam_step(theta.size, theta, np.ascontiguousarray(g, np.float64), m, v, int(t),
                        lr, b1, b2, eps)


# --- scenes --------------------------------------------------------------------
class OracleScene:
    """Oracle-side copy of a scene built by the shared input generators."""

    def __init__(self, scene, brute_force=False):
        self.scene = scene
        a = scene.arrays()
        self._keep = a
        st = SceneIn()
        for nm in ("eye", "fwd", "right", "up"):
            getattr(st, nm)[:] = [float(v) for v in getattr(scene, nm)]
        st.env[:] = [float(v) for v in scene.env]
        st.width, st.height, st.spp = scene.width, scene.height, scene.spp
        st.max_bounces, st.pixel_center = scene.max_bounces, scene.pixel_center
        ptr = lambda x: x.ctypes.data if x.size else None
        st.n_mat = a["mat_type"].size
        st.mat_type, st.mat_rgb, st.mat_ior = ptr(a["mat_type"]), ptr(a["mat_rgb"]), ptr(a["mat_ior"])
        st.n_sph = a["spheres"].shape[0]
        st.sph, st.sph_mat = ptr(a["spheres"]), ptr(a["sphere_mat"])
        st.n_quad = a["quads"].shape[0]
        st.quad, st.quad_mat = ptr(a["quads"]), ptr(a["quad_mat"])
        st.n_mesh = a["mesh_mat"].size
        st.mesh_off, st.mesh_mat, st.mesh_xlate = (ptr(a["mesh_off"]), ptr(a["mesh_mat"]),
                                                   ptr(a["mesh_xlate"]))
        st.n_tri = a["tris"].shape[0]
        st.tri = ptr(a["tris"])
        st.n_plight = a["plights"].shape[0]
        st.plight = ptr(a["plights"])
        st.n_param = a["bindings"].shape[0]
        st.binding = ptr(a["bindings"])
        st.mesh_rot = ptr(a["mesh_rot"])
        self.h = lib().orc_scene_new(C.byref(st))
        lib().orc_set_brute_force(self.h, 1 if brute_force else 0)
        self.d = st.n_param
        self.W, self.H = scene.width, scene.height

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_scene_free(self.h)
            self.h = None

    def set_brute_force(self, on):
        lib().orc_set_brute_force(self.h, 1 if on else 0)

    def trace(self, X, o, d):
        o, d = _f32(o).reshape(-1, 3), _f32(d).reshape(-1, 3)
        n = o.shape[0]
        t = np.zeros(n, np.float32)
        ids = np.zeros(n, np.int32)
        lib().orc_trace(self.h, _f32(X if len(X) else [0.0]), n, o, d, t, ids)
        return t, ids

    def render(self, X, tag=TAG_PATH, pair=0, seed=0, nthreads=0):
        img = np.zeros((self.H, self.W, 3), np.float32)
        lib().orc_render(self.h, _f32(X if len(X) else [0.0]), tag, pair, int(seed), nthreads, img)
        return img

    def render_pixels(self, X, pix, tag=TAG_PATH, pair=0, seed=0, nthreads=0):
        pix = np.ascontiguousarray(pix, np.int32)
        out = np.zeros((pix.size, 3), np.float32)
        lib().orc_render_pixels(self.h, _f32(X if len(X) else [0.0]), tag, pair, int(seed),
                                pix.size, pix, nthreads, out)
        return out

    def reference(self, theta_ref, seed=0, nthreads=0):
        """Reference image rendered at theta_ref with the REF stream."""
        return self.render(theta_ref, tag=TAG_REF, pair=0, seed=seed, nthreads=nthreads)

    def grad_estimate(self, ref, theta, sigma, N, seed, mode, nthreads=0):
        d = self.d
        g = np.zeros(d, np.float64)
        q = C.c_double()
        L = np.zeros(N, np.float64)
        tau = np.zeros((N if int(mode) & INDEPENDENT else N // 2, d), np.float32)
        rc = lib().orc_grad_estimate(self.h, _f32(ref), _f32(theta, d), _f32(sigma, d), int(N),
                                     int(seed), int(mode), nthreads, g, C.byref(q), L, tau)
        if rc:
            raise ValueError("invalid estimator arguments")
        return dict(grad=g, loss=q.value, losses=L, tau=tau)

    def smoothed_loss(self, ref, theta, sigma, N, seed, nthreads=0):
        q = C.c_double()
        rc = lib().orc_smoothed_loss(self.h, _f32(ref), _f32(theta, self.d), _f32(sigma, self.d),
                                     int(N), int(seed), nthreads, C.byref(q))
        if rc:
            raise ValueError("invalid estimator arguments")
        return q.value

    def dp_image_derivative(self, X, pair=0, seed=0, edge_samples=4096, mask=7, nthreads=0):
        """dI/dtheta [H, W, 3, d] of one render (Eq. 9's differentiable renderer)."""
        out = np.zeros((self.H, self.W, 3, self.d), np.float64)
        rc = lib().orc_dp_image_derivative(self.h, _f32(X, self.d), int(pair), int(seed),
                                           int(edge_samples), int(mask), nthreads, out)
        if rc:
            raise ValueError("scene or arguments not supported by the differentiable renderer")
        return out

    def dp_grad_estimate(self, ref, theta, sigma, N, seed, edge_samples=4096, nthreads=0):
        """Eq. 9 estimate: dict(grad, loss, losses)."""
        d = self.d
        g = np.zeros(d, np.float64)
        q = C.c_double()
        L = np.zeros(N, np.float64)
        rc = lib().orc_dp_grad_estimate(self.h, _f32(ref), _f32(theta, d), _f32(sigma, d), int(N),
                                        int(seed), int(edge_samples), nthreads, g, C.byref(q), L)
        if rc:
            raise ValueError("scene or arguments not supported by the differentiable renderer")
        return dict(grad=g, loss=q.value, losses=L)

    def render_perturbed(self, theta, sigma, N, seed, mode, nthreads=0):
        imgs = np.zeros((N, self.H, self.W, 3), np.float32)
        tau = np.zeros((N if int(mode) & INDEPENDENT else N // 2, self.d), np.float32)
        rc = lib().orc_render_perturbed(self.h, _f32(theta, self.d), _f32(sigma, self.d), int(N),
                                        int(seed), int(mode), nthreads, imgs, tau)
        if rc:
            raise ValueError("invalid estimator arguments")
        return imgs, tau


def mse(img, ref):
    img, ref = _f32(img), _f32(ref)
    return lib().orc_mse(img, ref, img.size // 3)

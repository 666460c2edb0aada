"""Thin ctypes binding of libprdpt.so (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device buffers
are torch tensors on the context's device (torch supplies memory and streams
only); host vectors are numpy arrays.  The binding fails loudly if the HIP
library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libprdpt.so")

PRDPT_OK = 0
PRDPT_E_ARG, PRDPT_E_NOMEM, PRDPT_E_ADMISSION, PRDPT_E_HIP = -1, -2, -3, -4
PRDPT_E_SCENE, PRDPT_E_CANCELLED, PRDPT_E_TIMEOUT = -5, -6, -7
PRDPT_EST_GAUSS, PRDPT_EST_IS, PRDPT_EST_IS_PERDIM = 0, 1, 2
PRDPT_EST_INDEPENDENT = 0x100   # or-ed into a mode: no antithetic partners (noAT)
PRDPT_EST_STRATIFIED = 0x200    # or-ed into an independent mode: stratified first uniforms
PRDPT_MAX_PARAMS = 256
PRDPT_BATCH_MAX_PARAMS = PRDPT_MAX_PARAMS  # d limit of the batched and served forms

# every symbol declared in include/prdpt.h
EXPORTS = [
    "prdpt_last_error", "prdpt_ctx_create", "prdpt_ctx_destroy", "prdpt_ctx_set_stream",
    "prdpt_ctx_resident_bytes", "prdpt_ctx_synchronize", "prdpt_scene_create",
    "prdpt_scene_destroy", "prdpt_scene_info", "prdpt_draw_tau", "prdpt_render_perturbed",
    "prdpt_render_reference", "prdpt_smoothed_loss", "prdpt_grad_estimate",
    "prdpt_grad_estimate_async", "prdpt_combine_async", "prdpt_ctx_set_timing",
    "prdpt_ctx_read_timing", "prdpt_traversal_counts", "prdpt_sigma_schedule", "prdpt_adam_step",
    "prdpt_copy_probe", "prdpt_selftest_math", "prdpt_batch_estimate", "prdpt_batch_config",
    "prdpt_batch_autotune",
    "prdpt_server_start", "prdpt_server_add_job", "prdpt_server_submit", "prdpt_server_cancel",
    "prdpt_server_poll", "prdpt_server_get_stats", "prdpt_server_stop",
    "prdpt_server_submit_deadline", "prdpt_debug_fail_allocations",
    "prdpt_grad_estimate_noalloc", "prdpt_grad_estimate_dp",
]


class PrdptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"prdpt error {code}: {msg}")
        self.code = code


class SceneDesc(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("fwd", C.c_float * 3), ("right", C.c_float * 3),
                ("up", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32), ("spp", C.c_int32),
                ("max_bounces", C.c_int32), ("pixel_center", C.c_int32),
                ("env", C.c_float * 3),
                ("n_materials", C.c_int32), ("mat_type", C.c_void_p), ("mat_rgb", C.c_void_p),
                ("mat_ior", C.c_void_p),
                ("n_spheres", C.c_int32), ("spheres", C.c_void_p), ("sphere_mat", C.c_void_p),
                ("n_quads", C.c_int32), ("quads", C.c_void_p), ("quad_mat", C.c_void_p),
                ("n_meshes", C.c_int32), ("mesh_offset", C.c_void_p), ("mesh_mat", C.c_void_p),
                ("mesh_translation", C.c_void_p),
                ("n_triangles", C.c_int32), ("triangles", C.c_void_p),
                ("n_point_lights", C.c_int32), ("point_lights", C.c_void_p),
                ("n_params", C.c_int32), ("bindings", C.c_void_p),
                ("mesh_rotation", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("ref", C.c_void_p), ("theta", C.c_void_p),
                ("sigma", C.c_void_p), ("N", C.c_int32), ("est", C.c_int32),
                ("seed", C.c_uint64), ("grad_out", C.c_void_p), ("loss_out", C.c_void_p),
                ("losses_out", C.c_void_p), ("status", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_batch", C.c_int32), ("max_inflight", C.c_int32)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("job", C.c_int32), ("status", C.c_int32),
                ("loss", C.c_double), ("grad", C.c_double * PRDPT_BATCH_MAX_PARAMS), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "epochs",
                                          "admissions", "evictions", "pending",
                                          "resident_bytes")] + [("paths", C.c_double)]


_lib = None


def load():
    """Load libprdpt.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime of the process)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python -m paper_2211_17263_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, u64, sz = C.c_void_p, C.c_int, C.c_uint64, C.c_size_t
    pvp = C.POINTER(C.c_void_p)
    L.prdpt_last_error.restype = C.c_char_p
    L.prdpt_ctx_create.argtypes = [i32, vp, sz, pvp]
    L.prdpt_ctx_destroy.argtypes = [vp]
    L.prdpt_ctx_set_stream.argtypes = [vp, vp]
    L.prdpt_ctx_resident_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.prdpt_ctx_synchronize.argtypes = [vp]
    L.prdpt_scene_create.argtypes = [vp, C.POINTER(SceneDesc), pvp, C.POINTER(C.c_size_t)]
    L.prdpt_scene_destroy.argtypes = [vp]
    L.prdpt_scene_info.argtypes = [vp] + [C.POINTER(C.c_int)] * 5
    L.prdpt_draw_tau.argtypes = [vp, i32, i32, i32, u64, vp, vp, vp]
    L.prdpt_render_perturbed.argtypes = [vp, vp, vp, i32, u64, i32, vp, vp]
    L.prdpt_render_reference.argtypes = [vp, vp, u64, vp]
    L.prdpt_smoothed_loss.argtypes = [vp, vp, vp, vp, i32, u64, vp]
    L.prdpt_grad_estimate.argtypes = [vp, vp, vp, vp, i32, u64, i32, vp, vp, vp]
    L.prdpt_grad_estimate_dp.argtypes = [vp, vp, vp, vp, i32, u64, i32, vp, vp, vp]
    L.prdpt_grad_estimate_async.argtypes = [vp, vp, vp, vp, i32, u64, i32, vp, vp, vp, vp]
    L.prdpt_grad_estimate_noalloc.argtypes = [vp, vp, vp, vp, i32, u64, i32, vp, vp, vp, vp]
    L.prdpt_combine_async.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32]
    L.prdpt_ctx_set_timing.argtypes = [vp, i32]
    L.prdpt_ctx_read_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.prdpt_traversal_counts.argtypes = [vp, vp, vp, i32, u64, i32, vp]
    L.prdpt_sigma_schedule.argtypes = [C.c_double, C.c_double, i32, i32]
    dp = C.c_void_p
    L.prdpt_adam_step.argtypes = [i32, dp, dp, dp, dp, i32, C.c_double, C.c_double, C.c_double,
                                  C.c_double]
    L.prdpt_copy_probe.argtypes = [vp, vp, vp, sz, i32, C.POINTER(C.c_double)]
    L.prdpt_selftest_math.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.prdpt_batch_estimate.argtypes = [vp, C.POINTER(Request), i32]
    L.prdpt_batch_config.argtypes = [vp, i32, i32, i32]
    L.prdpt_batch_autotune.argtypes = [vp, C.POINTER(Request), i32, C.c_char_p,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_double)]
    L.prdpt_server_start.argtypes = [vp, C.POINTER(ServerConfig), pvp]
    L.prdpt_server_add_job.argtypes = [vp, C.POINTER(SceneDesc), vp, C.POINTER(C.c_int)]
    L.prdpt_server_submit.argtypes = [vp, i32, vp, vp, i32, u64, i32, C.POINTER(C.c_int64)]
    L.prdpt_server_submit_deadline.argtypes = [vp, i32, vp, vp, i32, u64, i32, C.c_double,
                                               C.POINTER(C.c_int64)]
    L.prdpt_debug_fail_allocations.argtypes = [C.c_int64]
    L.prdpt_server_cancel.argtypes = [vp, C.c_int64]
    L.prdpt_server_poll.argtypes = [vp, C.POINTER(Completion), i32, i32, C.POINTER(C.c_int)]
    L.prdpt_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    L.prdpt_server_stop.argtypes = [vp]
    for name in EXPORTS:
        if name != "prdpt_last_error":
            getattr(L, name).restype = C.c_int
    L.prdpt_sigma_schedule.restype = C.c_double
    _lib = L
    return L


def _check(rc):
    if rc != PRDPT_OK:
        raise PrdptError(rc, load().prdpt_last_error().decode())
    return rc


def _host(a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype))
    return a, a.ctypes.data_as(C.c_void_p)


def _dev(t, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


class Context:
    """prdpt_ctx: one device, one HIP stream (default: torch's current stream)."""

    def __init__(self, device=0, stream=None, hbm_budget=0):
        import torch
        L = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = C.c_void_p()
        _check(L.prdpt_ctx_create(int(device), C.c_void_p(stream.cuda_stream if stream is not None else 0),
                                  int(hbm_budget), C.byref(h)))
        self.h = h

    def resident_bytes(self):
        v = C.c_size_t()
        _check(load().prdpt_ctx_resident_bytes(self.h, C.byref(v)))
        return v.value

    def synchronize(self):
        _check(load().prdpt_ctx_synchronize(self.h))

    def set_stream(self, stream):
        _check(load().prdpt_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream if stream else 0)))
        self.stream = stream

    def close(self):
        if getattr(self, "h", None):
            _check(load().prdpt_ctx_destroy(self.h))
            self.h = None


def scene_desc(scene):
    """Fill a prdpt_scene_desc from a generator Scene; returns (desc, keep-alive)."""
    a = scene.arrays()
    d = SceneDesc()
    for nm in ("eye", "fwd", "right", "up"):
        getattr(d, nm)[:] = [float(v) for v in getattr(scene, nm)]
    d.env[:] = [float(v) for v in scene.env]
    d.width, d.height, d.spp = scene.width, scene.height, scene.spp
    d.max_bounces, d.pixel_center = scene.max_bounces, scene.pixel_center
    ptr = lambda x: x.ctypes.data if x.size else None
    d.n_materials = a["mat_type"].size
    d.mat_type, d.mat_rgb, d.mat_ior = ptr(a["mat_type"]), ptr(a["mat_rgb"]), ptr(a["mat_ior"])
    d.n_spheres = a["spheres"].shape[0]
    d.spheres, d.sphere_mat = ptr(a["spheres"]), ptr(a["sphere_mat"])
    d.n_quads = a["quads"].shape[0]
    d.quads, d.quad_mat = ptr(a["quads"]), ptr(a["quad_mat"])
    d.n_meshes = a["mesh_mat"].size
    d.mesh_offset, d.mesh_mat, d.mesh_translation = (ptr(a["mesh_off"]), ptr(a["mesh_mat"]),
                                                     ptr(a["mesh_xlate"]))
    d.n_triangles = a["tris"].shape[0]
    d.triangles = ptr(a["tris"])
    d.n_point_lights = a["plights"].shape[0]
    d.point_lights = ptr(a["plights"])
    d.n_params = a["bindings"].shape[0]
    d.bindings = ptr(a["bindings"])
    d.mesh_rotation = ptr(a["mesh_rot"])
    return d, a


class Scene:
    """prdpt_scene: resident scene handle."""

    def __init__(self, ctx, h, footprint, width, height, spp, bounces, d):
        self.ctx, self.h, self.footprint = ctx, h, footprint
        self.W, self.H, self.spp, self.B, self.d = width, height, spp, bounces, d

    def destroy(self):
        if getattr(self, "h", None):
            _check(load().prdpt_scene_destroy(self.h))
            self.h = None


def prdpt_scene_create(ctx, scene):
    desc, keep = scene_desc(scene)
    h = C.c_void_p()
    fp = C.c_size_t()
    _check(load().prdpt_scene_create(ctx.h, C.byref(desc), C.byref(h), C.byref(fp)))
    del keep
    ints = [C.c_int() for _ in range(5)]
    _check(load().prdpt_scene_info(h, *[C.byref(i) for i in ints]))
    return Scene(ctx, h, fp.value, *[i.value for i in ints])


def prdpt_scene_destroy(scene):
    scene.destroy()


def prdpt_draw_tau(ctx, est, sigma, P, seed):
    sig, sp = _host(sigma, np.float32)
    d = sig.size
    tau = np.zeros((P, d), np.float32)
    c = np.zeros((P, d), np.float64)
    _check(load().prdpt_draw_tau(ctx.h, int(est), d, int(P), int(seed), sp,
                                 tau.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p)))
    return tau, c


def prdpt_render_perturbed(scene, theta, sigma, N, seed, est, images=None):
    import torch
    th, tp = _host(theta, np.float32)
    sg, sp = _host(sigma, np.float32)
    if th.size != scene.d or sg.size != scene.d:
        raise ValueError("theta/sigma length must equal the scene's parameter count")
    if images is None:
        images = torch.empty((N, scene.H, scene.W, 3), dtype=torch.float32,
                             device=f"cuda:{scene.ctx.device}")
    rows = N if int(est) & PRDPT_EST_INDEPENDENT else N // 2
    tau = np.zeros((max(rows, 1), scene.d), np.float32)
    _check(load().prdpt_render_perturbed(scene.h, tp, sp, int(N), int(seed), int(est),
                                         _dev(images, torch.float32), tau.ctypes.data_as(C.c_void_p)))
    return images, tau


def prdpt_render_reference(scene, X, seed, image=None):
    import torch
    x, xp = _host(X, np.float32)
    if x.size != scene.d:
        raise ValueError("X length must equal the scene's parameter count")
    if image is None:
        image = torch.empty((scene.H, scene.W, 3), dtype=torch.float32,
                            device=f"cuda:{scene.ctx.device}")
    _check(load().prdpt_render_reference(scene.h, xp, int(seed), _dev(image, torch.float32)))
    return image


def prdpt_smoothed_loss(scene, ref, theta, sigma, N, seed):
    import torch
    th, tp = _host(theta, np.float32)
    sg, sp = _host(sigma, np.float32)
    if th.size != scene.d or sg.size != scene.d:
        raise ValueError("theta/sigma length must equal the scene's parameter count")
    out = C.c_double()
    _check(load().prdpt_smoothed_loss(scene.h, _dev(ref, torch.float32), tp, sp, int(N), int(seed),
                                      C.byref(out)))
    return out.value


def prdpt_grad_estimate(scene, ref, theta, sigma, N, seed, est):
    """Returns dict(grad=float64[d], loss=Q estimate, losses=float64[N])."""
    import torch
    th, tp = _host(theta, np.float32)
    sg, sp = _host(sigma, np.float32)
    if th.size != scene.d or sg.size != scene.d:
        raise ValueError("theta/sigma length must equal the scene's parameter count")
    g = np.zeros(scene.d, np.float64)
    q = C.c_double()
    L = np.zeros(max(int(N), 1), np.float64)
    _check(load().prdpt_grad_estimate(scene.h, _dev(ref, torch.float32), tp, sp, int(N), int(seed),
                                      int(est), g.ctypes.data_as(C.c_void_p), C.byref(q),
                                      L.ctypes.data_as(C.c_void_p)))
    return dict(grad=g, loss=q.value, losses=L)


def prdpt_grad_estimate_dp(scene, ref, theta, sigma, N, seed, edge_samples=4096):
    """Eq. 9 estimate: dict(grad=float64[d], loss=mean loss, losses=float64[N])."""
    import torch
    th, tp = _host(theta, np.float32)
    sg, sp = _host(sigma, np.float32)
    if th.size != scene.d or sg.size != scene.d:
        raise ValueError("theta/sigma length must equal the scene's parameter count")
    g = np.zeros(scene.d, np.float64)
    q = C.c_double()
    L = np.zeros(max(int(N), 1), np.float64)
    _check(load().prdpt_grad_estimate_dp(scene.h, _dev(ref, torch.float32), tp, sp, int(N),
                                         int(seed), int(edge_samples),
                                         g.ctypes.data_as(C.c_void_p), C.byref(q),
                                         L.ctypes.data_as(C.c_void_p)))
    return dict(grad=g, loss=q.value, losses=L)


def prdpt_grad_estimate_async(scene, ref, theta, sigma, N, seed, est, grad, loss, losses=None,
                              c=None):
    import torch
    _check(load().prdpt_grad_estimate_async(
        scene.h, _dev(ref, torch.float32), _dev(theta, torch.float32), _dev(sigma, torch.float32),
        int(N), int(seed), int(est), _dev(grad, torch.float64), _dev(loss, torch.float64),
        _dev(losses, torch.float64) if losses is not None else None,
        _dev(c, torch.float64) if c is not None else None))


def prdpt_grad_estimate_noalloc(scene, ref, theta, sigma, N, seed, est, grad, loss, losses=None,
                                c=None):
    import torch
    _check(load().prdpt_grad_estimate_noalloc(
        scene.h, _dev(ref, torch.float32), _dev(theta, torch.float32), _dev(sigma, torch.float32),
        int(N), int(seed), int(est), _dev(grad, torch.float64), _dev(loss, torch.float64),
        _dev(losses, torch.float64) if losses is not None else None,
        _dev(c, torch.float64) if c is not None else None))


def prdpt_debug_fail_allocations(after):
    """Let `after` more library allocations succeed, then fail them (< 0: off)."""
    _check(load().prdpt_debug_fail_allocations(int(after)))


def prdpt_ctx_set_timing(ctx, enable):
    _check(load().prdpt_ctx_set_timing(ctx.h, 1 if enable else 0))


def prdpt_ctx_read_timing(ctx):
    """(total render-kernel milliseconds, launches) since the last read."""
    ms, n = C.c_double(), C.c_int64()
    _check(load().prdpt_ctx_read_timing(ctx.h, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def prdpt_traversal_counts(scene, theta, sigma, N, seed, est):
    """Work counts of one estimate's render: per-lane nodes, tris, rays, paths,
    wave-level iterations of the node, triangle and ray loops, lanes idle in
    ray-loop iterations because their pixel is done, stack pushes into the
    private part and the deepest stack."""
    th, tp = _host(theta, np.float32)
    sg, sp = _host(sigma, np.float32)
    out = np.zeros(10, np.uint64)
    _check(load().prdpt_traversal_counts(scene.h, tp, sp, int(N), int(seed), int(est),
                                         out.ctypes.data_as(C.c_void_p)))
    return dict(zip(("nodes", "tris", "rays", "paths", "wave_node_iters", "wave_tri_iters",
                     "wave_ray_iters", "idle_lane_iters", "overflow_pushes", "deepest_stack"),
                    (int(x) for x in out)))


def prdpt_copy_probe(ctx, src, dst, iters=10):
    """Mean ms per copy of src into dst (device tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    ms = C.c_double()
    _check(load().prdpt_copy_probe(ctx.h, _dev(src), _dev(dst), nbytes, int(iters), C.byref(ms)))
    return ms.value


def prdpt_selftest_math(ctx):
    """Mismatch counts of the render kernel's fast correctly rounded
    reciprocal and square root over every binary32 input of their domains:
    (reciprocal, square-root core, square root)."""
    out = (C.c_uint64 * 3)()
    _check(load().prdpt_selftest_math(ctx.h, out))
    return tuple(int(v) for v in out)


def prdpt_sigma_schedule(sigma0, sigma_end, t, T):
    return load().prdpt_sigma_schedule(float(sigma0), float(sigma_end), int(t), int(T))


def prdpt_adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 numpy arrays."""
    for a in (theta, m, v):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError("theta/m/v must be contiguous float64 arrays")
    g = np.ascontiguousarray(grad, np.float64)
    _check(load().prdpt_adam_step(theta.size, theta.ctypes.data_as(C.c_void_p),
                                  g.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p),
                                  v.ctypes.data_as(C.c_void_p), int(t), float(lr), float(beta1),
                                  float(beta2), float(eps)))


def prdpt_combine_async(ctx, rows, d, c, losses, scale, grad, est=PRDPT_EST_IS):
    """rows = pairs (antithetic) or draws (est with PRDPT_EST_INDEPENDENT)."""
    import torch
    _check(load().prdpt_combine_async(ctx.h, int(rows), int(d), _dev(c, torch.float64),
                                      _dev(losses, torch.float64),
                                      _dev(scale, torch.float64) if scale is not None else None,
                                      _dev(grad, torch.float64), int(est)))


class BatchRequest:
    """Host-side holder of one prdpt_request and its output arrays."""

    def __init__(self, scene, ref, theta, sigma, N, seed, est):
        import torch
        self.scene, self.N, self.seed, self.est = scene, int(N), int(seed), int(est)
        self.ref = ref
        self.theta = np.ascontiguousarray(theta, np.float32)
        self.sigma = np.ascontiguousarray(sigma, np.float32)
        self.grad = np.zeros(max(scene.d, 1), np.float64)
        self.loss = np.zeros(1, np.float64)
        self.losses = np.zeros(max(self.N, 1), np.float64)
        self.status = None
        if not isinstance(ref, torch.Tensor):
            raise TypeError("ref must be a device tensor")

    def fill(self, r):
        r.scene = self.scene.h.value if self.scene.h is not None else None
        r.ref = self.ref.data_ptr()
        r.theta = self.theta.ctypes.data
        r.sigma = self.sigma.ctypes.data
        r.N, r.est, r.seed = self.N, self.est, self.seed
        r.grad_out = self.grad.ctypes.data
        r.loss_out = self.loss.ctypes.data
        r.losses_out = self.losses.ctypes.data
        r.status = 0


def _requests(reqs):
    arr = (Request * len(reqs))()
    for r, q in zip(arr, reqs):
        q.fill(r)
    return arr


def prdpt_batch_estimate(ctx, reqs):
    """Runs BatchRequest objects as one batch; sets .grad/.loss/.losses/.status."""
    arr = _requests(reqs)
    _check(load().prdpt_batch_estimate(ctx.h, arr, len(reqs)))
    for r, q in zip(arr, reqs):
        q.status = r.status
    return reqs


def prdpt_batch_config(ctx, blocks_per_cu, tiles_per_item, use_graph=True):
    _check(load().prdpt_batch_config(ctx.h, int(blocks_per_cu), int(tiles_per_item),
                                     1 if use_graph else 0))


def prdpt_batch_autotune(ctx, reqs, cache_path=None):
    """(blocks_per_cu, tiles_per_item, ms) chosen for batches like reqs."""
    arr = _requests(reqs)
    b, t, ms = C.c_int(), C.c_int(), C.c_double()
    _check(load().prdpt_batch_autotune(ctx.h, arr, len(reqs),
                                       cache_path.encode() if cache_path else None,
                                       C.byref(b), C.byref(t), C.byref(ms)))
    return b.value, t.value, ms.value


class Server:
    """prdpt_server: continuous-batching request loop on one context."""

    def __init__(self, ctx, hbm_budget=0, max_batch=64, max_inflight=2):
        cfg = ServerConfig(int(hbm_budget), int(max_batch), int(max_inflight))
        h = C.c_void_p()
        _check(load().prdpt_server_start(ctx.h, C.byref(cfg), C.byref(h)))
        self.h, self.ctx = h, ctx
        self.d = {}
        self._buf = (Completion * 256)()

    def add_job(self, scene, ref):
        """Register a generator Scene and its reference image (host float32 [H, W, 3])."""
        desc, keep = scene_desc(scene)
        r, rp = _host(ref, np.float32)
        jid = C.c_int()
        _check(load().prdpt_server_add_job(self.h, C.byref(desc), rp, C.byref(jid)))
        del keep
        self.d[jid.value] = scene.d
        return jid.value

    def submit(self, job, theta, sigma, N, seed, est, timeout_s=None):
        """Queue a request; with timeout_s it calls prdpt_server_submit_deadline."""
        th, tp = _host(theta, np.float32)
        sg, sp = _host(sigma, np.float32)
        if th.size != self.d[job] or sg.size != self.d[job]:
            raise ValueError("theta/sigma length must equal the job's parameter count")
        t = C.c_int64()
        if timeout_s is None:
            _check(load().prdpt_server_submit(self.h, int(job), tp, sp, int(N), int(seed),
                                              int(est), C.byref(t)))
        else:
            _check(load().prdpt_server_submit_deadline(self.h, int(job), tp, sp, int(N),
                                                       int(seed), int(est), float(timeout_s),
                                                       C.byref(t)))
        return t.value

    def cancel(self, ticket):
        _check(load().prdpt_server_cancel(self.h, int(ticket)))

    def poll(self, timeout_ms=0):
        """List of completion dicts (ticket, job, status, loss, grad, t_submit, t_start, t_done)."""
        n = C.c_int()
        _check(load().prdpt_server_poll(self.h, self._buf, len(self._buf), int(timeout_ms),
                                        C.byref(n)))
        out = []
        for c in self._buf[: n.value]:
            d = self.d.get(c.job, 0)
            out.append(dict(ticket=c.ticket, job=c.job, status=c.status, loss=c.loss,
                            grad=np.array(c.grad[:d]), t_submit=c.t_submit, t_start=c.t_start,
                            t_done=c.t_done))
        return out

    def stats(self):
        st = ServerStats()
        _check(load().prdpt_server_get_stats(self.h, C.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}

    def stop(self):
        if getattr(self, "h", None):
            _check(load().prdpt_server_stop(self.h))
            self.h = None

"""Inverse-rendering driver on top of the plateau-reduced gradient estimator.

Each iteration draws the bandwidth sigma_t from the adaptive schedule
(Sec. 3.3: linear decay from sigma_0 to the floor sigma_m; the supplement's
hyperparameter notes start the decay after about half of the iterations and
use sigma_m = 0.01), estimates the gradient of the smoothed objective with the
HIP library (Sec. 3.1 Eq. 10, Sec. 3.2), and takes the library's binary64 Adam
step on the host (Sec. 3.4: Adam with default parameters).  It records the two
metrics of Sec. 4.1: the image-space MSE that the optimisation acts on, and the
parameter-space MSE that is only evaluated.

Everything on the gradient path runs in the library; torch only holds device
memory and evaluates the recorded image MSE of the unperturbed render.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import native as NV


def sigma_at(sigma0, sigma_min, t, steps, warm_start=0.5):
    """Bandwidth of iteration t (0-based) of `steps`: sigma0 until the fraction
    `warm_start` of the iterations has passed, then linear to sigma_min at the
    last iteration (per dimension; the host schedule of the library)."""
    s0 = np.atleast_1d(np.asarray(sigma0, np.float64))
    sm = np.broadcast_to(np.asarray(sigma_min, np.float64), s0.shape)
    first = int(round(warm_start * (steps - 1))) if steps > 1 else 0
    if t <= first:
        return s0.astype(np.float32)
    span = steps - first
    return np.array([NV.prdpt_sigma_schedule(a, b, t - first, span) for a, b in zip(s0, sm)],
                    np.float32)


@dataclass
class Trace:
    """Per-iteration record of an optimisation run."""
    theta: list = field(default_factory=list)       # parameters before the step
    sigma: list = field(default_factory=list)
    q_hat: list = field(default_factory=list)       # smoothed-objective estimate
    grad: list = field(default_factory=list)
    param_mse: list = field(default_factory=list)   # mean (theta - theta_ref)^2, if known
    image_mse: list = field(default_factory=list)   # MSE of the unperturbed render, if evaluated
    step_ms: list = field(default_factory=list)     # estimate + Adam step
    final_theta: np.ndarray | None = None


def image_mse(scene, ref, theta, seed):
    """Mean squared difference over pixels and channels between the render at
    theta (reference stream, fixed seed) and ref."""
    img = NV.prdpt_render_reference(scene, np.asarray(theta, np.float32), seed)
    return float(((img - ref) ** 2).mean().item())


def optimize(scene, ref, theta0, sigma0, steps, lr, N, est=NV.PRDPT_EST_IS, seed=0,
             sigma_min=0.01, warm_start=0.5, theta_ref=None, eval_every=0, eval_seed=12345):
    """Run `steps` iterations of PRDPT + Adam from theta0; returns a Trace.

    scene: native.Scene; ref: device float32 [H, W, 3] reference image;
    sigma0: initial bandwidth (scalar or per dimension); N: renders per
    estimate (even); est: perturbation sampler; seed: iteration t uses seed + t;
    eval_every > 0 records the image MSE of the unperturbed render every that
    many iterations (and at the end)."""
    d = scene.d
    theta = np.array(theta0, np.float64).reshape(d)
    s0 = np.broadcast_to(np.asarray(sigma0, np.float64), (d,)).copy()
    m = np.zeros(d)
    v = np.zeros(d)
    tr = Trace()
    tref = None if theta_ref is None else np.asarray(theta_ref, np.float64).reshape(d)
    for t in range(steps):
        sig = sigma_at(s0, sigma_min, t, steps, warm_start)
        th32 = theta.astype(np.float32)
        t0 = time.perf_counter()
        r = NV.prdpt_grad_estimate(scene, ref, th32, sig, N, seed + t, est)
        tr.theta.append(theta.copy())
        NV.prdpt_adam_step(theta, r["grad"], m, v, t + 1, lr)
        tr.step_ms.append(1e3 * (time.perf_counter() - t0))
        tr.sigma.append(sig.copy())
        tr.q_hat.append(r["loss"])
        tr.grad.append(r["grad"].copy())
        if tref is not None:
            tr.param_mse.append(float(np.mean((tr.theta[-1] - tref) ** 2)))
        if eval_every and (t % eval_every == 0):
            tr.image_mse.append((t, image_mse(scene, ref, th32, eval_seed)))
    tr.final_theta = theta.copy()
    if tref is not None:
        tr.param_mse.append(float(np.mean((theta - tref) ** 2)))
    if eval_every:
        tr.image_mse.append((steps, image_mse(scene, ref, theta.astype(np.float32), eval_seed)))
    return tr

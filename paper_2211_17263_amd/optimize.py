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

import os
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
    state: object = None                            # DriverState after the last iteration


@dataclass
class DriverState:
    """Everything the optimisation loop carries from one iteration to the next
    (the parameters, Adam's moments and the next iteration index) and the
    settings that define the rest of the run (bandwidth schedule, learning
    rate, renders per estimate, sampler, seed base).  Resuming from it
    continues the run exactly: iteration t always uses seed + t and the
    schedule's sigma_t."""
    theta: np.ndarray
    m: np.ndarray
    v: np.ndarray
    t: int
    steps: int
    sigma0: np.ndarray
    sigma_min: float
    warm_start: float
    lr: float
    N: int
    est: int
    seed: int


def save_state(path, st):
    """Write a DriverState as an .npz of plain arrays (no pickled objects),
    atomically: a crash mid-write leaves the previous checkpoint intact."""
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, theta=st.theta, m=st.m, v=st.v, t=np.int64(st.t), steps=np.int64(st.steps),
                 sigma0=np.asarray(st.sigma0, np.float64), sigma_min=np.float64(st.sigma_min),
                 warm_start=np.float64(st.warm_start), lr=np.float64(st.lr), N=np.int64(st.N),
                 est=np.int64(st.est), seed=np.int64(st.seed))
    os.replace(tmp, path)


def load_state(path):
    """Read a checkpoint written by save_state."""
    with np.load(path, allow_pickle=False) as z:
        return DriverState(theta=z["theta"].copy(), m=z["m"].copy(), v=z["v"].copy(),
                           t=int(z["t"]), steps=int(z["steps"]), sigma0=z["sigma0"].copy(),
                           sigma_min=float(z["sigma_min"]), warm_start=float(z["warm_start"]),
                           lr=float(z["lr"]), N=int(z["N"]), est=int(z["est"]), seed=int(z["seed"]))


def image_mse(scene, ref, theta, seed):
    """Mean squared difference over pixels and channels between the render at
    theta (reference stream, fixed seed) and ref."""
    img = NV.prdpt_render_reference(scene, np.asarray(theta, np.float32), seed)
    return float(((img - ref) ** 2).mean().item())


def optimize(scene, ref, theta0, sigma0, steps, lr, N, est=NV.PRDPT_EST_IS, seed=0,
             sigma_min=0.01, warm_start=0.5, theta_ref=None, eval_every=0, eval_seed=12345,
             resume=None, checkpoint_path=None, checkpoint_every=0, stop_after=None):
    """Run `steps` iterations of PRDPT + Adam from theta0; returns a Trace.

    scene: native.Scene; ref: device float32 [H, W, 3] reference image;
    sigma0: initial bandwidth (scalar or per dimension); N: renders per
    estimate (even); est: perturbation sampler; seed: iteration t uses seed + t;
    eval_every > 0 records the image MSE of the unperturbed render every that
    many iterations (and at the end).
    Checkpoints: with checkpoint_path and checkpoint_every > 0 the DriverState
    is written after every checkpoint_every-th iteration (and when the loop
    stops); resume (a DriverState, e.g. load_state(path)) continues that run
    from its next iteration, its settings taking the place of the arguments;
    stop_after ends the loop after that many iterations of this call (an
    interrupted run, for tests).  The trace covers this call's iterations."""
    d = scene.d
    if resume is not None:
        st = resume
        theta, m, v = st.theta.astype(np.float64).copy(), st.m.copy(), st.v.copy()
        steps, lr, N, est, seed = st.steps, st.lr, st.N, st.est, st.seed
        s0, sigma_min, warm_start = np.asarray(st.sigma0, np.float64), st.sigma_min, st.warm_start
        t_first = st.t
    else:
        theta = np.array(theta0, np.float64).reshape(d)
        s0 = np.broadcast_to(np.asarray(sigma0, np.float64), (d,)).copy()
        m = np.zeros(d)
        v = np.zeros(d)
        t_first = 0
    tr = Trace()
    tref = None if theta_ref is None else np.asarray(theta_ref, np.float64).reshape(d)

    def state(t_next):
        return DriverState(theta=theta.copy(), m=m.copy(), v=v.copy(), t=t_next, steps=steps,
                           sigma0=s0.copy(), sigma_min=float(sigma_min),
                           warm_start=float(warm_start), lr=float(lr), N=int(N), est=int(est),
                           seed=int(seed))

    t_end = steps if stop_after is None else min(steps, t_first + int(stop_after))
    for t in range(t_first, t_end):
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
        if checkpoint_path and checkpoint_every > 0 and (t + 1) % checkpoint_every == 0:
            save_state(checkpoint_path, state(t + 1))
    if checkpoint_path:
        save_state(checkpoint_path, state(t_end))
    tr.final_theta = theta.copy()
    tr.state = state(t_end)
    if tref is not None:
        tr.param_mse.append(float(np.mean((theta - tref) ** 2)))
    if eval_every:
        tr.image_mse.append((t_end, image_mse(scene, ref, theta.astype(np.float32), eval_seed)))
    return tr

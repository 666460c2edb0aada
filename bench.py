#!/usr/bin/env python3
"""Throughput of the plateau-reduced gradient estimator on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
draw the antithetic perturbations, path-trace every perturbed scene, reduce each
image's squared error against the reference, combine the losses with the kernel
weights in binary64, then the host-side bandwidth schedule and Adam step.  The
default workload is the caustic scene (512x512, 64 spp, 8 bounces, a glass
sphere focusing an area light past a 50000-triangle occluder, 3 parameters,
N = 32 importance-sampled perturbations, bandwidth annealed 1.0 -> 0.05); the
global-illumination scene (256x256, 16 spp, 4 bounces, 6 parameters, N = 16),
Eq. 9 against Eq. 10 on the toy scene, the batched form (64 uneven jobs in one
persistent graph launch against the plain per-request loop) and the served
form (Poisson arrivals from 256 jobs against a plain FIFO, with p50/p99
latency) run beside it under "extra_workloads".

Prints one JSON line.  `value` is gradient estimates per second over the timed
steps, `latency_ms` the per-step distribution (p10/p50/p90/p99); `roofline`
describes the fused render kernel: algorithmic node/triangle/reference bytes
per launch over its event-timed duration against 8 TB/s, with the measured
DRAM rate and the copy probe's achievable rate beside it (`cache_served` when
the algorithmic rate exceeds what DRAM can deliver); `roofline_alu` is the same
kernel's algorithmic binary32 arithmetic against the 157.3 TFLOP/s vector peak
and `valu` its measured VALU issue utilisation; `cpu_baseline` is the CPU
oracle timed on this host's cores on a bounded sample (antithetic pairs of the
first timed estimate), and `parity` compares those renders with the GPU's.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NODE_BYTES, TRI_BYTES, REF_BYTES_PER_PIXEL = 128, 48, 12
# algorithmic binary32 arithmetic per unit of work (fma = 2): a 4-wide node
# visit is four slab tests of 6 fma + 6 min/max; a Moeller-Trumbore test is two
# cross products, four dot products, one difference, one division, three
# products and one sum; shading per ray query is an estimate (100-200)
NODE_FLOPS, TRI_FLOPS, SHADE_FLOPS_PER_RAY = 4 * 18, 46, 150
FP32_PEAK_TFLOPS = 157.3
KERNEL_SRC = os.path.join(ROOT, "paper_2211_17263_amd", "csrc", "kernels.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2211_17263_amd import scenes as S
    if name == "cornell":
        pr = S.cornell_problem(seed=2)
        desc = "global illumination: Cornell box 12 quads + 2 x 5120-triangle jittered icospheres"
        return pr, desc, pr["sigma"], pr["sigma"]
    if name == "toy":
        pr = S.toy_problem(seed=1)
        return pr, "toy direct light: sphere over plane, point light", pr["sigma"], pr["sigma"]
    if name == "caustic":
        pr = S.caustic_problem(seed=3)
        desc = "caustic: glass sphere, area light, 50000-triangle occluder"
        return pr, desc, pr["sigma"], np.full_like(pr["sigma"], pr["sigma_end"])
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(workload):
    """Measured HBM bytes per launch of the render kernel on this workload, valid
    only for the kernel source the counters were taken on."""
    path = os.path.join(ROOT, "profiles", f"traffic_render_loss_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src_hash = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != src_hash:
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def alu_roofline(per, kernel_s):
    """The render kernel against the binary32 vector peak: algorithmic FP32
    operations of its node visits, triangle tests and shading per launch (from
    the counting copy's work on the same rays) over the event-timed duration."""
    flops = (per["nodes"] * NODE_FLOPS + per["tris"] * TRI_FLOPS +
             per["rays"] * SHADE_FLOPS_PER_RAY)
    achieved = flops / kernel_s / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "flops_per_launch": flops}


def valu_from_profile(workload, kernel_s):
    """VALU issue utilisation and FP32 rate of the render kernel from the
    committed issue counters (profiles/counters_render_loss_<workload>.txt),
    valid only for the kernel source they were taken on."""
    path = os.path.join(ROOT, "profiles", f"counters_render_loss_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src_hash = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != src_hash:
        return None
    try:
        return {"valu_issue_utilisation": float(kv["valu_issue_utilisation"]),
                "fp32_arith_share_of_valu": float(kv["fp32_arith_share_of_valu"]),
                "fp32_tflops_upper_bound": float(kv["fp32_flop_upper_bound_per_dispatch"]) / kernel_s / 1e12,
                "fp32_peak_tflops": FP32_PEAK_TFLOPS}
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="caustic",
                    choices=["cornell", "toy", "caustic", "batch", "serve", "inverse", "ablation",
                             "highd", "eq9"])
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="serve workload: length of each arrival phase")
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="serve workload: offered Poisson arrival rate (requests/s)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="caustic: skip the short global-illumination run beside the headline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU-oracle baseline: render antithetic pairs of the first timed "
                         "estimate until this much time passed")
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the streaming-copy probe (1 GiB, 20 copies) and print its rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the estimator "
              f"would shard by antithetic pairs across GPUs, which is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_17263_amd import native as NV

    if args.copy_probe:
        ctx = NV.Context(0)
        print(json.dumps({"copy_probe_GBps": copy_rate(ctx, NV, 1 << 30, 20), "bytes": 1 << 30}))
        ctx.close()
        return

    if args.workload == "batch":
        print(json.dumps(bench_batch(args, NV)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, NV)), flush=True)
        return
    if args.workload == "inverse":
        return bench_inverse(args, NV)
    if args.workload == "highd":
        return bench_highd(args, NV)
    if args.workload == "eq9":
        print(json.dumps(eq9_vs_eq10(args, NV, cpu=not args.no_cpu)), flush=True)
        return
    if args.workload == "ablation":
        return bench_ablation(args, NV)

    out = bench_estimator(args, NV, args.workload, cpu=not args.no_cpu)
    if args.workload == "caustic" and not args.no_extra:
        # the global-illumination workload beside the headline (short, no CPU leg)
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = 20, 5
        gi = bench_estimator(sub, NV, "cornell", cpu=False)
        out["extra_workloads"] = {"cornell": {k: gi[k] for k in (
            "value", "unit", "ms_per_step", "latency_ms", "config", "paths_per_s", "kernel",
            "roofline", "roofline_alu", "simd_efficiency")}}
        out["extra_workloads"]["toy_eq9_vs_eq10"] = eq9_vs_eq10(args, NV, cpu=not args.no_cpu)
        # the batched and served forms against the plain per-request estimator
        # (short runs: two timed batched and two plain passes over the 64 jobs;
        # four 5 s arrival phases of the server)
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup, sub.serve_seconds = 8, 1, 5.0
        for key, fn in (("batch", bench_batch), ("serve", bench_serve)):
            try:
                out["extra_workloads"][key] = fn(sub, NV)
            except Exception as e:  # noqa: BLE001 - the headline line must still print
                log(f"{key} workload failed: {e!r}")
                out["extra_workloads"][key] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


def eq9_vs_eq10(args, NV, cpu=True, steps=200, edge_samples=4096):
    """The toy workload (64x64, 1 spp, N = 4, sigma 0.5, direct light) with both
    estimators of Sec. 3.1: Eq. 10 (kernel derivative times the renderer,
    prdpt_grad_estimate, GAUSS) and Eq. 9 (the kernel-smoothed gradient of the
    differentiable renderer, prdpt_grad_estimate_dp): estimates per second over
    `steps` calls each, the per-estimate variance of the gradient at theta_0
    (same seeds), and, with cpu, one Eq. 9 estimate against the oracle's."""
    import torch
    from paper_2211_17263_amd import scenes as S
    pr = S.toy_problem(seed=1)
    sc_desc = S.dp_scene(width=64, height=64, spp=1)
    ctx = NV.Context(0)
    sc = NV.prdpt_scene_create(ctx, sc_desc)
    ref = NV.prdpt_render_reference(sc, pr["theta_ref"], args.seed + 7)
    th, sg, N = pr["theta0"], pr["sigma"], pr["N"]
    res = {"config": {"workload": "toy", "width": 64, "height": 64, "spp": 1, "N": N,
                      "sigma": float(sg[0]), "edge_samples_per_edge": edge_samples}}
    for name, fn in (("eq10", lambda seed: NV.prdpt_grad_estimate(sc, ref, th, sg, N, seed,
                                                                  NV.PRDPT_EST_GAUSS)),
                     ("eq9", lambda seed: NV.prdpt_grad_estimate_dp(sc, ref, th, sg, N, seed,
                                                                    edge_samples))):
        for t in range(5):
            fn(args.seed + t)
        torch.cuda.synchronize()
        grads = []
        t0 = time.perf_counter()
        for t in range(steps):
            grads.append(fn(args.seed + 100 + t)["grad"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g = np.asarray(grads)
        res[name] = {"estimates_per_s": steps / el, "ms_per_estimate": 1e3 * el / steps,
                     "grad_mean": g.mean(0).tolist(), "grad_var_sum": float(g.var(0, ddof=1).sum())}
    res["eq9_over_eq10_time"] = res["eq9"]["ms_per_estimate"] / res["eq10"]["ms_per_estimate"]
    res["eq9_over_eq10_variance"] = res["eq9"]["grad_var_sum"] / res["eq10"]["grad_var_sum"]
    if cpu:
        from oracle import oracle as O
        from tests import parity as PT
        osc = O.OracleScene(sc_desc)
        ref_h = ref.cpu().numpy()
        r = NV.prdpt_grad_estimate_dp(sc, ref, th, sg, N, args.seed, edge_samples)
        t0 = time.perf_counter()
        o = osc.dp_grad_estimate(ref_h, th, sg, N, args.seed, edge_samples=edge_samples)
        res["eq9_oracle_s_per_estimate"] = time.perf_counter() - t0
        rel = np.abs(r["losses"] - o["losses"]) / np.abs(o["losses"])
        grel = np.abs(r["grad"] - o["grad"]) / np.maximum(np.abs(o["grad"]), 1e-12)
        res["eq9_parity"] = {"max_rel_loss_err": float(rel.max()), "grad_gpu": r["grad"].tolist(),
                             "grad_oracle": o["grad"].tolist(), "max_rel_grad_err": float(grel.max()),
                             "pass_1e-4": bool(rel.max() <= PT.LOSS_REL and grel.max() <= 1e-4)}
    sc.destroy()
    ctx.close()
    return res


def bench_estimator(args, NV, name, cpu=True):
    """W warm-up and K timed steps of one estimator workload: per step the
    bandwidth of the annealing schedule, one prdpt_grad_estimate (perturbation
    draw, fused render + loss, losses, binary64 combine; inputs resident on the
    device, theta/sigma up and the gradient down through pinned memory) and
    the host Adam step.  Then the work of the timed launches (counting kernel),
    the roofline figures, and, with cpu, the oracle leg (timing + parity)."""
    import torch
    pr, desc, sigma0, sigma_end = workload(name)
    scene = pr["scene"]
    N, est, d = pr["N"], pr["est"], scene.d
    H, W, spp = scene.height, scene.width, scene.spp
    total_steps = args.warmup + args.steps

    ctx = NV.Context(0)
    t_build = time.perf_counter()
    sc = NV.prdpt_scene_create(ctx, scene)
    t_build = time.perf_counter() - t_build
    log(f"workload {name}: {W}x{H} spp={spp} N={N} d={d}, scene built in {t_build:.2f} s")
    ref = NV.prdpt_render_reference(sc, pr["theta_ref"], args.seed + 7)

    theta = pr["theta0"].astype(np.float64)
    m = np.zeros(d)
    v = np.zeros(d)
    lr = float(pr.get("lr", 0.01))
    trajectory = []
    lat = []

    def step(t):
        s = np.array([NV.prdpt_sigma_schedule(a, b, t, total_steps) for a, b in zip(sigma0, sigma_end)],
                     np.float32)
        th32 = theta.astype(np.float32)
        seed = args.seed + t
        t0 = time.perf_counter()
        r = NV.prdpt_grad_estimate(sc, ref, th32, s, N, seed, est)
        NV.prdpt_adam_step(theta, r["grad"], m, v, t + 1, lr)
        lat.append(time.perf_counter() - t0)
        trajectory.append((th32, s, seed, r))
        return r

    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} steps), timing {args.steps} steps")
    lat.clear()
    trajectory.clear()
    NV.prdpt_ctx_read_timing(ctx)
    NV.prdpt_ctx_set_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.warmup, total_steps):
        last = step(t)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, launches = NV.prdpt_ctx_read_timing(ctx)
    NV.prdpt_ctx_set_timing(ctx, False)
    log(f"timed {args.steps} steps in {elapsed:.3f} s; counting work of the timed launches")

    # algorithmic work of the timed launches, replayed with the counting kernel
    # (at most 8 evenly spaced timed steps; the per-estimate mean stands for all)
    keys = ("nodes", "tris", "rays", "paths", "wave_node_iters", "wave_tri_iters",
            "wave_ray_iters", "idle_lane_iters", "overflow_pushes")
    cnt = {k: 0 for k in keys}
    deepest = 0
    counted = sorted(set(np.linspace(0, len(trajectory) - 1, min(8, len(trajectory))).round().astype(int)))
    for i in counted:
        th32, s, seed, _ = trajectory[i]
        c = NV.prdpt_traversal_counts(sc, th32, s, N, seed, est)
        for k in keys:
            cnt[k] += c[k]
        deepest = max(deepest, c["deepest_stack"])
    K = args.steps
    per = {k: cnt[k] / len(counted) for k in keys}
    alg_bytes = per["nodes"] * NODE_BYTES + per["tris"] * TRI_BYTES + N * H * W * REF_BYTES_PER_PIXEL
    kernel_avg_s = (kernel_ms / launches) / 1e3 if launches else float("nan")
    achieved = alg_bytes / kernel_avg_s / 1e9
    paths_per_est = N * H * W * spp
    lat_ms = 1e3 * np.asarray(lat)

    out = {
        "metric": "gradient estimates/sec and paths/sec at 1e-4 rel. error; p50/p99 request latency",
        "value": K / elapsed,
        "unit": "gradient estimates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "scene": desc, "width": W, "height": H, "spp": spp,
                   "max_bounces": scene.max_bounces, "params": d, "N": N,
                   "estimator": ["gauss", "is", "is_perdim"][est], "triangles": scene.n_tris,
                   "sigma": f"{float(sigma0[0]):g} -> {float(sigma_end[0]):g} linearly over the "
                            f"{total_steps} steps" if float(sigma0[0]) != float(sigma_end[0])
                            else f"{float(sigma0[0]):g}"},
        "paths_per_s": paths_per_est * K / elapsed,
        "rays_per_s": per["rays"] * K / elapsed,
        "latency_ms": {"p10": float(np.percentile(lat_ms, 10)),
                       "p50": float(np.percentile(lat_ms, 50)),
                       "p90": float(np.percentile(lat_ms, 90)),
                       "p99": float(np.percentile(lat_ms, 99)),
                       "mean": float(lat_ms.mean())},
        "kernel": {"name": "render_loss_kernel", "avg_ms": 1e3 * kernel_avg_s, "launches": launches,
                   "share_of_step": (kernel_ms / 1e3) / elapsed},
        "work_per_estimate": {"nodes": per["nodes"], "triangles": per["tris"], "rays": per["rays"],
                              "paths": per["paths"], "counted_steps": len(counted),
                              "stack_pushes_beyond_lds": per["overflow_pushes"],
                              "deepest_stack": deepest},
        "step_ms_by_sigma": {f"{float(trajectory[i][1][0]):.4g}": float(lat_ms[i]) for i in
                             sorted({0, len(lat) // 2, len(lat) - 1})},
        "simd_efficiency": {
            "node_loop": per["nodes"] / max(64 * per["wave_node_iters"], 1),
            "triangle_loop": per["tris"] / max(64 * per["wave_tri_iters"], 1),
            "ray_loop": per["rays"] / max(64 * per["wave_ray_iters"], 1),
            "ray_loop_lanes_idle_done": per["idle_lane_iters"] / max(64 * per["wave_ray_iters"], 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(name),
                     "achieved_is": "algorithmic bytes (128 B per node visit, 48 B per triangle "
                                    "test, 12 B per reference pixel read) per launch over the "
                                    "event-timed launch"},
        "valu": valu_from_profile(name, kernel_avg_s),
        "roofline_alu": alu_roofline(per, kernel_avg_s),
        "scene_build_s": t_build,
        "final_loss": last["loss"],
    }
    rf = out["roofline"]
    achievable = copy_rate(ctx, NV, 256 << 20, 10)
    rf["achievable_copy_GBps"] = achievable
    rf["frac_of_achievable"] = achieved / achievable
    # above the copy probe's rate the gather is served from L2 / Infinity Cache
    rf["cache_served"] = bool(achieved > achievable)
    if rf["traffic"] is not None:
        rf["dram_GBps"] = rf["traffic"] / kernel_avg_s / 1e9
        rf["dram_frac"] = rf["dram_GBps"] / HBM_PEAK_GBS
    rf["fp32_frac"] = out["roofline_alu"]["frac"]
    if cpu:
        log("CPU oracle baseline leg")
        out["cpu_baseline"], out["parity"] = cpu_leg(sc, pr, ref, trajectory[0], args, NV)
    sc.destroy()
    ctx.close()
    return out


def bench_inverse(args, NV):
    """End-to-end inverse rendering with the driver (Adam + warm-started sigma
    schedule): the plateau demonstration (black sphere, no silhouette overlap at
    the start) for GAUSS, IS and sigma -> 0, sweeps of N and sigma_0 on it, and
    the global-illumination workload's 6 parameters."""
    import torch
    from paper_2211_17263_amd import optimize as OP
    from paper_2211_17263_amd import scenes as S
    ctx = NV.Context(0)
    out = {"metric": "inverse rendering: final parameter MSE (plateau and GI workloads)",
           "n_gpus": 1, "data": "synthetic", "dtype": "f32", "config": {"workload": "inverse"}}
    # plateau
    sc = NV.prdpt_scene_create(ctx, S.plateau_scene())
    tref = np.zeros(2, np.float32)
    th0 = np.array([0.9, 0.9], np.float32)
    ref = NV.prdpt_render_reference(sc, tref, 5)
    seeds = (100, 1100, 2100)

    def final(s0, N, est, sm=0.01):
        r = [OP.optimize(sc, ref, th0, s0, 300, 0.02, N, est=est, seed=sd, sigma_min=sm,
                         theta_ref=tref).param_mse[-1] for sd in seeds]
        return float(np.median(r))
    log("inverse: plateau demonstration")
    out["plateau"] = {"start_param_mse": float(np.mean(th0 ** 2)), "steps": 300, "lr": 0.02,
                      "N": 4, "sigma0": 0.5, "median_of_seeds": len(seeds),
                      "gauss": final(0.5, 4, NV.PRDPT_EST_GAUSS),
                      "is": final(0.5, 4, NV.PRDPT_EST_IS),
                      "sigma_to_zero_1e-6": final(1e-6, 4, NV.PRDPT_EST_IS, sm=1e-6)}
    log("inverse: N and sigma_0 sweeps")
    out["n_sweep_is_sigma0.5"] = {str(N): final(0.5, N, NV.PRDPT_EST_IS) for N in (2, 4, 8, 16)}
    out["sigma0_sweep_is_N4"] = {str(s0): final(s0, 4, NV.PRDPT_EST_IS)
                                 for s0 in (0.05, 0.1, 0.2, 0.35, 0.5, 0.75, 1.0)}
    sc.destroy()
    # global illumination
    log("inverse: global-illumination workload")
    pr = S.cornell_problem(seed=2)
    sc = NV.prdpt_scene_create(ctx, pr["scene"])
    ref = NV.prdpt_render_reference(sc, pr["theta_ref"], args.seed + 7)
    # the paper's GI bandwidth (sigma_0 = 0.125) with N = 16 renders and lr 0.01
    steps, lr, s0 = 400, 0.01, 0.125
    out["gi"] = {"steps": steps, "lr": lr, "N": pr["N"], "sigma0": s0, "sigma_min": 0.01,
                 "warm_start": 0.5, "runs": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for seed in (args.seed, args.seed + 4000):
        tr = OP.optimize(sc, ref, pr["theta0"], s0, steps, lr, pr["N"], est=pr["est"], seed=seed,
                         theta_ref=pr["theta_ref"], eval_every=100)
        out["gi"]["runs"].append({
            "seed": seed,
            "param_mse": {str(t): tr.param_mse[t] for t in range(0, steps + 1, 100)},
            "image_mse": {str(t): v for t, v in tr.image_mse},
            "ms_per_step": float(np.mean(tr.step_ms))})
    el = time.perf_counter() - t0
    noise = OP.image_mse(sc, ref, pr["theta_ref"], 12345)
    out["gi"]["image_mse_at_theta_ref"] = noise     # the Monte Carlo noise floor
    out["gi"]["wall_s"] = el
    out["value"] = 2 * steps / el
    out["unit"] = "GI optimisation steps/s (estimate + Adam + periodic image-MSE renders)"
    out["higher_is_better"] = True
    sc.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_ablation(args, NV):
    """Estimator ablation (Sec. 4.4, Tab. 4: noIS, noAP, noAT; stratified draws instead
    of antithetic pairs, Sec. 3.2) and variance study: per
    estimator arm, the per-render gradient variance and bias against a
    high-precision reference gradient on the global-illumination workload and
    on the plateau scene, the renders needed for 10 % relative RMS error, and
    the final parameter MSE of the optimisation with each component removed."""
    import torch
    from paper_2211_17263_amd import optimize as OP
    from paper_2211_17263_amd import scenes as S
    I = NV.PRDPT_EST_INDEPENDENT
    ST = NV.PRDPT_EST_INDEPENDENT | NV.PRDPT_EST_STRATIFIED
    arms = {"is (full)": NV.PRDPT_EST_IS, "gauss (noIS)": NV.PRDPT_EST_GAUSS,
            "is, independent (noAT)": NV.PRDPT_EST_IS | I,
            "is, stratified instead of antithetic": NV.PRDPT_EST_IS | ST,
            "gauss, independent (noIS+noAT)": NV.PRDPT_EST_GAUSS | I,
            "is per-dimension": NV.PRDPT_EST_IS_PERDIM}
    ctx = NV.Context(0)
    out = {"metric": "estimator variance per render and ablated optimisation", "n_gpus": 1,
           "data": "synthetic", "dtype": "f32", "config": {"workload": "ablation"}}

    def study(sc, ref, theta, sigma, N, K, K_ref):
        rg = np.array([NV.prdpt_grad_estimate(sc, ref, theta, sigma, N, 50000 + i,
                                              NV.PRDPT_EST_IS)["grad"] for i in range(K_ref)])
        refg, ref_var = rg.mean(0), rg.var(0, ddof=1) / K_ref
        res = {"reference_grad": refg.tolist(), "N": N, "estimates_per_arm": K,
               "reference_estimates": K_ref}
        norm2 = float(np.dot(refg, refg))
        for name, est in arms.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gs = np.array([NV.prdpt_grad_estimate(sc, ref, theta, sigma, N, 1000 + i, est)["grad"]
                           for i in range(K)])
            ms = 1e3 * (time.perf_counter() - t0) / K
            mean, var = gs.mean(0), gs.var(0, ddof=1)
            per_render = float(N * var.sum() / norm2)        # relative, summed over components
            se = np.sqrt(var / K + ref_var) + 1e-300     # arm mean minus reference mean
            res[name] = {"variance_per_render_rel": per_render,
                         "max_bias_in_se": float(np.max(np.abs(mean - refg) / se)),
                         "rel_bias": float(np.linalg.norm(mean - refg) / np.sqrt(norm2)),
                         "renders_for_10pct_rms": per_render / 0.01,
                         "ms_per_estimate": ms}
        return res
    log("ablation: variance on the global-illumination workload")
    pr = S.cornell_problem(seed=2)
    sc = NV.prdpt_scene_create(ctx, pr["scene"])
    ref = NV.prdpt_render_reference(sc, pr["theta_ref"], args.seed + 7)
    # at the workload's start the light is 0.06 below the ceiling and sigma =
    # 0.3, so many perturbations lift it through the ceiling and black out the
    # image: a heavy-tailed estimate; the second point keeps crossings rare
    out["variance_gi"] = study(sc, ref, pr["theta0"], pr["sigma"], 16, 96, 384)
    th_low = pr["theta0"].copy()
    th_low[1] = -0.3
    out["variance_gi_light_low"] = study(sc, ref, th_low, np.full(6, 0.1, np.float32), 16, 96, 384)
    out["variance_gi_light_low"]["theta"] = th_low.tolist()
    log("ablation: optimisation on the global-illumination workload")
    gi = {}
    for name, est, warm in (("full", NV.PRDPT_EST_IS, 0.5), ("noIS", NV.PRDPT_EST_GAUSS, 0.5),
                            ("noAP", NV.PRDPT_EST_IS, 1.0), ("noAT", NV.PRDPT_EST_IS | I, 0.5),
                            ("stratified", NV.PRDPT_EST_IS | ST, 0.5)):
        tr = OP.optimize(sc, ref, pr["theta0"], 0.125, 400, 0.01, 16, est=est, seed=args.seed,
                         warm_start=warm, theta_ref=pr["theta_ref"], eval_every=400)
        gi[name] = {"param_mse": tr.param_mse[-1], "image_mse": tr.image_mse[-1][1]}
    out["optimisation_gi"] = dict(gi, steps=400, N=16, sigma0=0.125, lr=0.01,
                                  start_param_mse=tr.param_mse[0])
    sc.destroy()
    log("ablation: plateau scene")
    sc = NV.prdpt_scene_create(ctx, S.plateau_scene())
    tref = np.zeros(2, np.float32)
    th0 = np.array([0.9, 0.9], np.float32)
    ref = NV.prdpt_render_reference(sc, tref, 5)
    out["variance_plateau"] = study(sc, ref, th0, np.full(2, 0.5, np.float32), 4, 400, 4000)
    pl = {}
    for name, est, warm in (("full", NV.PRDPT_EST_IS, 0.5), ("noIS", NV.PRDPT_EST_GAUSS, 0.5),
                            ("noAP", NV.PRDPT_EST_IS, 1.0), ("noAT", NV.PRDPT_EST_IS | I, 0.5),
                            ("stratified", NV.PRDPT_EST_IS | ST, 0.5)):
        r = [OP.optimize(sc, ref, th0, 0.5, 300, 0.02, 4, est=est, seed=sd, warm_start=warm,
                         theta_ref=tref).param_mse[-1] for sd in (100, 1100, 2100)]
        pl[name] = float(np.median(r))
    out["optimisation_plateau"] = dict(pl, steps=300, N=4, sigma0=0.5, lr=0.02,
                                       start_param_mse=float(np.mean(th0 ** 2)), median_of_seeds=3)
    sc.destroy()
    ctx.close()
    out["value"] = out["variance_gi"]["is (full)"]["variance_per_render_rel"]
    out["unit"] = "relative gradient variance per render (IS, GI workload)"
    out["higher_is_better"] = False
    print(json.dumps(out), flush=True)


def bench_highd(args, NV):
    """Many objects and high d (the Sort task's regime, Sec. 4.1): per-render
    gradient variance of the antithetic IS and GAUSS estimators as the number of
    bound objects grows (d = 2 ... 150 on one 75-sphere scene), and the
    optimisation of all 150 coordinates."""
    import copy
    import torch
    from paper_2211_17263_amd import optimize as OP
    from paper_2211_17263_amd import scenes as S
    ctx = NV.Context(0)
    pr = S.sort_problem(seed=5)
    full = pr["scene"]
    out = {"metric": "high-d estimator variance and 150-D optimisation", "n_gpus": 1,
           "data": "synthetic", "dtype": "f32",
           "config": {"workload": "highd", "objects": len(full.spheres), "d": full.d,
                      "width": full.width, "height": full.height, "spp": full.spp,
                      "max_bounces": full.max_bounces}}
    sc = NV.prdpt_scene_create(ctx, full)
    ref = NV.prdpt_render_reference(sc, pr["theta_ref"], args.seed + 7)
    N, K, K_ref, sig = 16, 64, 256, 0.05
    log("highd: variance against the number of bound coordinates")
    var = {}
    for d in (2, 10, 50, 150):
        sub = copy.deepcopy(full)
        # spheres beyond the first d / 2 are fixed where theta_0 puts them
        for j, (kind, idx, comp) in enumerate(full.bindings):
            if j >= d:
                sub.spheres[idx][comp] = float(np.float32(sub.spheres[idx][comp]) + pr["theta0"][j])
        sub.bindings = full.bindings[:d]
        ssc = sc if d == full.d else NV.prdpt_scene_create(ctx, sub)
        theta, sigma = pr["theta0"][:d], np.full(d, sig, np.float32)
        rg = np.array([NV.prdpt_grad_estimate(ssc, ref, theta, sigma, N, 70000 + i,
                                              NV.PRDPT_EST_IS)["grad"] for i in range(K_ref)])
        refg = rg.mean(0)
        norm2 = float(np.dot(refg, refg))
        row = {"reference_estimates": K_ref, "estimates_per_arm": K, "grad_norm": norm2 ** 0.5}
        for name, est in (("is", NV.PRDPT_EST_IS), ("gauss", NV.PRDPT_EST_GAUSS)):
            gs = np.array([NV.prdpt_grad_estimate(ssc, ref, theta, sigma, N, 3000 + i, est)["grad"]
                           for i in range(K)])
            row[name] = float(N * gs.var(0, ddof=1).sum() / norm2)
        var[str(d)] = row
        if ssc is not sc:
            ssc.destroy()
    out["variance_per_render_rel"] = var
    out["variance_note"] = ("N * sum_j Var(g_j) / |g_ref|^2 at theta_0, sigma 0.05, N 16; "
                            "a first-order model of either estimator predicts about d + 1")
    log("highd: optimisation of all 150 coordinates")
    opt = {}
    steps, lr, s0 = 1000, 0.002, 0.05
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for name, est in (("is", NV.PRDPT_EST_IS), ("gauss", NV.PRDPT_EST_GAUSS)):
        tr = OP.optimize(sc, ref, pr["theta0"], s0, steps, lr, N, est=est, seed=args.seed,
                         theta_ref=pr["theta_ref"], eval_every=250)
        opt[name] = {"param_mse": {str(t): tr.param_mse[t] for t in range(0, steps + 1, 250)},
                     "image_mse": {str(t): v for t, v in tr.image_mse},
                     "ms_per_step": float(np.mean(tr.step_ms))}
    el = time.perf_counter() - t0
    out["optimisation_150d"] = dict(opt, steps=steps, lr=lr, N=N, sigma0=s0, sigma_min=0.01,
                                    image_mse_at_theta_ref=OP.image_mse(sc, ref, pr["theta_ref"],
                                                                       12345))
    sc.destroy()
    ctx.close()
    out["value"] = 2 * steps / el
    out["unit"] = "150-D optimisation steps/s (estimate + Adam + periodic image-MSE renders)"
    out["higher_is_better"] = True
    print(json.dumps(out), flush=True)


def tune_cache_path():
    d = os.path.join(ROOT, "gpurun_out")
    return os.path.join(d if os.path.isdir(d) else "/tmp", "prdpt_autotune.jsonl")


def bench_batch(args, NV):
    """64 uneven jobs (sides 64..512, 1k..200k triangles, d 2..12, N 4..32): the
    batched persistent graph launch against the plain per-request loop."""
    import torch
    from paper_2211_17263_amd import scenes as S
    jobs = S.batch_jobs(seed=4)
    ctx = NV.Context(0)
    t0 = time.perf_counter()
    scs = [NV.prdpt_scene_create(ctx, j["scene"]) for j in jobs]
    t_build = time.perf_counter() - t0
    refs = [NV.prdpt_render_reference(sc, j["theta_ref"], args.seed + 3) for sc, j in zip(scs, jobs)]
    torch.cuda.synchronize()
    log(f"batch: {len(jobs)} scenes built in {t_build:.1f} s, "
        f"{sum(j['scene'].n_tris for j in jobs)} triangles")
    reqs = [NV.BatchRequest(sc, r, j["theta0"], j["sigma"], j["N"], j["seed"], j["est"])
            for sc, r, j in zip(scs, refs, jobs)]
    bpc, tpi, tune_ms = NV.prdpt_batch_autotune(ctx, reqs, tune_cache_path())
    log(f"autotuned: {bpc} work-groups per CU, {tpi} tiles per item ({tune_ms:.1f} ms)")
    K = max(1, args.steps // 4)
    for _ in range(args.warmup):
        NV.prdpt_batch_estimate(ctx, reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        NV.prdpt_batch_estimate(ctx, reqs)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / K
    assert all(r.status == 0 for r in reqs)
    for sc, r, j in zip(scs, refs, jobs):       # warm the plain path
        NV.prdpt_grad_estimate(sc, r, j["theta0"], j["sigma"], j["N"], j["seed"], j["est"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        for sc, r, j in zip(scs, refs, jobs):
            NV.prdpt_grad_estimate(sc, r, j["theta0"], j["sigma"], j["N"], j["seed"], j["est"])
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / K
    same = all(np.array_equal(q.grad[:sc.d], NV.prdpt_grad_estimate(
        sc, r, j["theta0"], j["sigma"], j["N"], j["seed"], j["est"])["grad"])
        for q, sc, r, j in zip(reqs, scs, refs, jobs))
    paths = sum(j["N"] * j["scene"].width * j["scene"].height * j["scene"].spp for j in jobs)
    out = {"metric": "gradient estimates/sec and paths/sec at 1e-4 rel. error; p50/p99 request latency",
           "value": len(jobs) / t_batch, "unit": "gradient estimates/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_batch, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch", "jobs": len(jobs), "paths_per_batch": paths,
                      "blocks_per_cu": bpc, "tiles_per_item": tpi, "graph": True},
           "paths_per_s": paths / t_batch,
           "plain_per_request": {"value": len(jobs) / t_plain, "ms_per_batch_of_requests": 1e3 * t_plain},
           "speedup_vs_plain": t_plain / t_batch, "bitwise_equal_to_plain": bool(same),
           "scene_build_s": t_build}
    # the roofline on the batch's largest scene (the least cacheable BVH)
    i = max(range(len(jobs)), key=lambda t: jobs[t]["scene"].n_tris)
    out["largest_scene_roofline"] = scene_roofline(NV, ctx, scs[i], refs[i], jobs[i], args.seed)
    for sc in scs:
        sc.destroy()
    ctx.close()
    return out


def scene_roofline(NV, ctx, sc, ref, job, seed, K=5):
    """Single-request render-kernel roofline of one scene: algorithmic bytes of
    an estimate (counting kernel) over the mean HIP-event render time of K
    estimates (events on the library's stream)."""
    import torch
    scene, N, est = job["scene"], job["N"], job["est"]
    for t in range(2):
        NV.prdpt_grad_estimate(sc, ref, job["theta0"], job["sigma"], N, seed + t, est)
    torch.cuda.synchronize()
    NV.prdpt_ctx_read_timing(ctx)
    NV.prdpt_ctx_set_timing(ctx, True)
    for t in range(K):
        NV.prdpt_grad_estimate(sc, ref, job["theta0"], job["sigma"], N, seed + t, est)
    torch.cuda.synchronize()
    kernel_ms, launches = NV.prdpt_ctx_read_timing(ctx)
    NV.prdpt_ctx_set_timing(ctx, False)
    c = NV.prdpt_traversal_counts(sc, job["theta0"], job["sigma"], N, seed, est)
    H, W = scene.height, scene.width
    alg = c["nodes"] * NODE_BYTES + c["tris"] * TRI_BYTES + N * H * W * REF_BYTES_PER_PIXEL
    avg_s = kernel_ms / launches / 1e3
    achieved = alg / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel_avg_ms": 1e3 * avg_s,
            "algorithmic_bytes_per_launch": alg,
            "scene": {"width": W, "height": H, "spp": scene.spp, "max_bounces": scene.max_bounces,
                      "triangles": scene.n_tris, "N": N, "d": scene.d}}


def serve_phase(NV, ctx, jobs, refs, rate, seconds, max_batch, max_inflight, budget, seed):
    """Open-loop Poisson arrivals at `rate` for `seconds`; returns completion stats.
    Requests still queued at the end are cancelled and reported as not completed."""
    rng = np.random.default_rng(seed)
    sv = NV.Server(ctx, hbm_budget=budget, max_batch=max_batch, max_inflight=max_inflight)
    t_add = time.perf_counter()
    ids = [sv.add_job(j["scene"], r) for j, r in zip(jobs, refs)]
    log(f"serve phase rate={rate:.1f}: {len(ids)} jobs registered in {time.perf_counter() - t_add:.1f} s")
    # warm: every job once (admission, graph capture)
    warm = [sv.submit(ids[i], jobs[i]["theta0"], jobs[i]["sigma"], jobs[i]["N"], 1, jobs[i]["est"])
            for i in range(0, len(jobs), max(1, len(jobs) // 16))]
    got = 0
    while got < len(warm):
        got += len(sv.poll(timeout_ms=200))
    done, submitted = [], {}
    t0 = time.perf_counter()
    t_next = t0
    while True:
        now = time.perf_counter()
        if now - t0 >= seconds:
            break
        while t_next <= now:
            k = int(rng.integers(len(jobs)))
            j = jobs[k]
            th = (j["theta0"] + rng.normal(0, 0.02, j["scene"].d)).astype(np.float32)
            tk = sv.submit(ids[k], th, j["sigma"], j["N"], int(rng.integers(1, 2**62)), j["est"])
            submitted[tk] = now
            t_next += rng.exponential(1.0 / rate)
        done += sv.poll(timeout_ms=1)
    left = set(submitted) - {c["ticket"] for c in done}
    for tk in left:
        sv.cancel(tk)
    drain_t = time.perf_counter()
    while len(done) < len(submitted) and time.perf_counter() - drain_t < 60:
        done += sv.poll(timeout_ms=100)
    st = sv.stats()
    sv.stop()
    ok = [c for c in done if c["status"] == 0 and c["ticket"] in submitted]
    lat = np.array([c["t_done"] - c["t_submit"] for c in ok])
    # the arrival window on the server's clock: first to last submission
    w0 = min(c["t_submit"] for c in done if c["ticket"] in submitted) if done else 0.0
    w1 = max(c["t_submit"] for c in done if c["ticket"] in submitted) if done else 0.0
    span = max(w1 - w0, 1e-9)
    window_done = [c for c in ok if w0 <= c["t_done"] <= w1]
    paths = sum(jobs[c["job"]]["N"] * jobs[c["job"]]["scene"].width * jobs[c["job"]]["scene"].height
                * jobs[c["job"]]["scene"].spp for c in window_done)
    return {"offered_rate": rate, "seconds": span, "submitted": len(submitted),
            "completed_in_window": len(window_done), "completed_total": len(ok),
            "cancelled_at_end": len(left), "throughput_req_s": len(window_done) / span,
            "paths_per_s": paths / span,
            "latency_p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "latency_p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "epochs": st["epochs"], "admissions": st["admissions"], "evictions": st["evictions"]}


def bench_serve(args, NV):
    """256 jobs drawn like the batched workload; Poisson arrivals; the continuous-
    batching server against the plain per-request estimator (FIFO, one request at
    a time), at the offered rate and at a sustainable rate."""
    import torch
    from paper_2211_17263_amd import scenes as S
    jobs = S.batch_jobs(seed=5, n_jobs=256)
    ctx = NV.Context(0)
    refs = []
    t0 = time.perf_counter()
    for i, j in enumerate(jobs):
        sc = NV.prdpt_scene_create(ctx, j["scene"])
        refs.append(NV.prdpt_render_reference(sc, j["theta_ref"], args.seed + 3).cpu().numpy())
        sc.destroy()
        if i % 32 == 31:
            log(f"serve: {i + 1} references rendered")
    log(f"serve: {len(jobs)} references rendered in {time.perf_counter() - t0:.1f} s")
    budget = 512 << 20          # below the 256 jobs' total footprint: admission binds
    res = {}
    res["served"] = serve_phase(NV, ctx, jobs, refs, args.serve_rate, args.serve_seconds, 64, 2,
                                budget, 11)
    log("served at offered rate:", res["served"])
    res["plain"] = serve_phase(NV, ctx, jobs, refs, args.serve_rate, args.serve_seconds, 1, 1,
                               budget, 11)
    log("plain at offered rate:", res["plain"])
    sustain = 0.7 * res["served"]["throughput_req_s"]
    res["served_sustainable"] = serve_phase(NV, ctx, jobs, refs, sustain, args.serve_seconds, 64, 2,
                                            budget, 12)
    log("served at 70% of its throughput:", res["served_sustainable"])
    sustain_plain = 0.7 * res["plain"]["throughput_req_s"]
    res["plain_sustainable"] = serve_phase(NV, ctx, jobs, refs, sustain_plain, args.serve_seconds, 1,
                                           1, budget, 12)
    log("plain at 70% of its throughput:", res["plain_sustainable"])
    ctx.close()
    s = res["served"]
    out = {"metric": "gradient estimates/sec and paths/sec at 1e-4 rel. error; p50/p99 request latency",
           "value": s["throughput_req_s"], "unit": "gradient estimates/s", "n_gpus": 1,
           "steps": s["completed_in_window"], "warmup": 0, "ms_per_step": 1e3 / max(s["throughput_req_s"], 1e-9),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "serve", "jobs": len(jobs), "offered_rate": args.serve_rate,
                      "hbm_budget": budget, "max_batch": 64, "epochs_in_flight": 2},
           "latency_s": {"p50": s["latency_p50_s"], "p99": s["latency_p99_s"]},
           "plain_per_request": {"value": res["plain"]["throughput_req_s"],
                                 "latency_s": {"p50": res["plain"]["latency_p50_s"],
                                               "p99": res["plain"]["latency_p99_s"]}},
           "speedup_vs_plain": s["throughput_req_s"] / max(res["plain"]["throughput_req_s"], 1e-9),
           "phases": res}
    return out


def copy_rate(ctx, NV, nbytes, iters):
    """Achievable HBM bandwidth (GB/s, read + write) of the library's streaming copy."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = NV.prdpt_copy_probe(ctx, src, dst, iters)
    del src, dst
    return 2 * nbytes / (ms / 1e3) / 1e9


def cpu_leg(sc, pr, ref, first, args, NV):
    """The CPU oracle on the host's cores, on a bounded sample of the same
    workload: the antithetic pairs of the first timed estimate (same
    parameters, bandwidth, seed and reference), rendered pair by pair until
    about --cpu-seconds have passed (the whole estimate when it fits).  The
    oracle is built for this host (-O3 -march=native; bit-identical to the
    tests' build).  Parity on the same sample: every rendered oracle image
    against the GPU's image of the same perturbation, pixel by pixel, its loss
    against the GPU's per-image loss, and, when all pairs were rendered, the
    gradient."""
    import torch

    from oracle import build as OB
    from oracle import oracle as O
    from tests import parity as PT
    try:
        O.use_library(OB.build(native=True))
        build = "gcc -O3 -march=native (host-tuned)"
    except Exception as e:  # noqa: BLE001 - the portable build gives the same results
        log(f"host-tuned oracle build failed ({e}); timing the portable build")
        build = "gcc -O3 (portable)"
    scene = pr["scene"]
    N, est = pr["N"], pr["est"]
    P = N // 2
    th32, sigma, seed, r = first
    cores = len(os.sched_getaffinity(0))
    osc = O.OracleScene(scene)
    ref_h = ref.cpu().numpy()
    imgs = NV.prdpt_render_perturbed(sc, th32, sigma, N, seed, est)[0].cpu().numpy()
    tau, c = O.draw_tau(est, sigma, P, seed)
    L = np.zeros(N)
    worst_img = {"flips": 0, "rel_rmse": 0.0}
    t_cpu = 0.0
    done = 0
    while done < P:
        p = done
        for mm in range(2):
            X = (th32 + tau[p]) if mm == 0 else (th32 - tau[p])
            t1 = time.perf_counter()
            img = osc.render(X.astype(np.float32), tag=O.TAG_PATH, pair=p, seed=seed, nthreads=cores)
            t_cpu += time.perf_counter() - t1
            L[2 * p + mm] = O.mse(img, ref_h)
            st = PT.image_stats(imgs[2 * p + mm], img)
            worst_img["flips"] = max(worst_img["flips"], st["flips"])
            worst_img["rel_rmse"] = max(worst_img["rel_rmse"], st["rel_rmse"])
        done += 1
        if t_cpu >= args.cpu_seconds:
            break
    renders = 2 * done
    paths = renders * scene.width * scene.height * scene.spp
    # one thread: about 4096 evenly spread pixels of the first render
    npix = scene.width * scene.height
    pix = np.arange(0, npix, max(1, npix // 4096), dtype=np.int32)
    t1 = time.perf_counter()
    osc.render_pixels((th32 + tau[0]).astype(np.float32), pix, seed=seed, pair=0, nthreads=1)
    single = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    base = {"value": (renders / N) / t_cpu, "unit": "gradient estimates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{renders} of the {N} renders of the first timed estimate "
                      f"({done} antithetic pair(s), {paths} paths) in {t_cpu:.1f} s on {cores} "
                      f"threads; estimates/s = renders per second / N",
            "paths_per_s": paths / t_cpu, "cpu_model": model, "build": build,
            "single_thread_paths_per_s": pix.size * scene.spp / single}
    rel = np.abs(r["losses"][:renders] - L[:renders]) / np.abs(L[:renders])
    parity = {"checked_renders": renders, "of_renders": N, "pixels_per_render": npix,
              "max_flip_pixels": int(worst_img["flips"]), "max_image_rel_rmse": worst_img["rel_rmse"],
              "max_rel_loss_err": float(rel.max()),
              "pass_1e-4": bool(worst_img["flips"] == 0 and worst_img["rel_rmse"] <= PT.REL_RMSE
                                and rel.max() <= PT.LOSS_REL)}
    if done == P:
        g_orc, q_orc = O.combine(c, L)
        S = PT.grad_scale(c, L)
        gerr = np.abs(r["grad"] - g_orc) / S
        parity.update({"max_grad_err_over_scale": float(gerr.max()),
                       "q_hat_gpu": float(r["loss"]), "q_hat_oracle": float(q_orc)})
        parity["pass_1e-4"] = bool(parity["pass_1e-4"] and gerr.max() <= PT.GRAD_REL)
    return base, parity


if __name__ == "__main__":
    main()

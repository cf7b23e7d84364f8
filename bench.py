#!/usr/bin/env python3
"""Benchmark of one training step of differentiable tile splatting on one GPU.

Workload (default): the main scene -- 1,000,000 Gaussians drawn from 64
isotropic clusters whose weights span 100x, SH degree 3 (48 FP32 coefficients
per Gaussian), rendered at 1600x1064 with 16x16 tiles from a 32-camera orbit of
radius 4.  One step = project, bin/sort, forward compositing (through the
torch.autograd.Function), L1 loss against a seeded target image, backward
compositing and projection backward -- every stage a HIP kernel behind the C
ABI.  Inputs (parameters, cameras, targets) are resident in HBM before timing.

Prints ONE JSON line.  The step time comes from HIP events around each timed
step; per-kernel durations from the library's kernel timer (HIP events
recorded around every launch on the stream the kernel runs on) in a second
pass over the same steps.  Extra keys time one training iteration with the
fused Adam step, the heavy and the learned-colour workloads, and report the
decoder's image quality.
"""
from __future__ import annotations

import argparse
import contextlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# MI355X published dense FP32 vector peak (it counts packed dual-FP32 issue);
# the library is built without packed FP32 (-packed-fp32-ops), whose ceiling
# is half of it: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 157.3
ALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic work per unit.  FLOPs count an FMA as 2 and every other FP32
# operation (including exp and reciprocal) as 1.
#   projection: read 44 + 12 (D+1)^2 B of parameters, write the 36 B record +
#               depth + radius + tile count and the 40 B colour gradient (d
#               colour / d direction and the clamp mask) per Gaussian
#   bin/sort:   read u, v, radius, depth (16 B) per Gaussian, write the 4 B
#               list entry per (tile, Gaussian) pair and 8 B of range per tile
#   forward compositing: 14 flop per examined pair (offset, quadratic form,
#               exp, opacity, clamp, two skip tests) + 10 per blended pair
#               (1 - alpha, T update, stop test, weight, three colour FMAs);
#               HBM: the list, each record once, 20 B per pixel written
#   backward compositing: 14 flop per walked pair (alpha re-evaluation) + 52
#               per blended pair (T recovery, dL/dalpha, light behind, nine
#               gradient terms and their nine sums over pixels); HBM: the
#               list, each record once, 32 B per pixel read, 36 B per
#               Gaussian of record gradients written
#   projection backward: read the 44 B of geometry parameters, the 40 B
#               colour gradient and 36 B of record gradients, write parameter
#               gradients (44 + 12 (D+1)^2 B)
#   L1 loss: read image and target, write the gradient (36 B per pixel)
#   Adam: read parameter, gradient and both moments, write parameter and
#               moments: 28 B per value, 11 + 3 (D+1)^2 values per Gaussian
PROJECT_BYTES_PER_G = {d: 44 + 12 * (d + 1) ** 2 + 48 + 40 for d in range(4)}
PROJECT_BWD_BYTES_PER_G = {d: 44 + 40 + 36 + 44 + 12 * (d + 1) ** 2 for d in range(4)}
ADAM_BYTES_PER_G = {d: 28 * (11 + 3 * (d + 1) ** 2) for d in range(4)}
BIN_BYTES_PER_G, BIN_BYTES_PER_DUP, BIN_BYTES_PER_TILE = 16, 4, 8
FWD_BYTES_PER_DUP, FWD_BYTES_PER_G, FWD_BYTES_PER_PX = 4, 48, 20
BWD_BYTES_PER_DUP, BWD_BYTES_PER_G, BWD_BYTES_PER_PX = 4, 48 + 36, 32
L1_BYTES_PER_PX = 36
FWD_FLOP_EXAMINED, FWD_FLOP_BLENDED = 14, 10
BWD_FLOP_WALKED, BWD_FLOP_BLENDED = 14, 52


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# kernels of each stage (the names the kernel timer and rocprofv3 report)
STAGE_KERNELS = {
    "project": ("k_project<", "k_mlp_fwd<1>"),
    "bin_sort": ("k_depth_keys", "k_os_", "k_rs_hist", "k_rs_scatter", "k_scan_", "k_chunk_",
                 "k_tile_starts", "k_emit", "k_ranges", "k_put_zero_k"),
    "render_fwd": ("k_render_fwd_light", "k_render_fwd<false", "k_tile_plan"),
    "l1_loss": ("k_l1_",),
    "render_bwd": ("k_render_bwd", "k_acc_to_g2d", "k_det_", "k_zero4", "k_batch_plan"),
    "colour_hash_table": ("k_chs_table",),
    "density_control": ("k_dc_",),
    "project_bwd": ("k_project_bwd", "k_mlp_bwd<1>", "k_mlp_reduce"),
    "adam": ("k_adam_gaussians",),
}

# sources whose kernels run in each stage
STAGE_SOURCES = {
    "project": ("gs_project.hip", "gs_sh.h", "gs_mlp.hip", "gs_internal.h"),
    "bin_sort": ("gs_binsort.hip", "gs_internal.h"),
    "render_fwd": ("gs_render.hip", "gs_plan.hip", "gs_internal.h"),
    "l1_loss": ("gs_loss.hip", "gs_internal.h"),
    "render_bwd": ("gs_render.hip", "gs_plan.hip", "gs_internal.h"),
    "colour_hash_table": ("gs_render.hip", "gs_internal.h"),
    "density_control": ("gs_density.hip", "gs_binsort.hip", "gs_internal.h"),
    "project_bwd": ("gs_project.hip", "gs_sh.h", "gs_mlp.hip", "gs_internal.h"),
    "adam": ("gs_optim.hip", "gs_internal.h"),
}


def stage_of(kernel):
    for st, prefixes in STAGE_KERNELS.items():
        if kernel.startswith(prefixes):
            return st
    return None


def counter_traffic_bytes(kernel):
    """Calibrated HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    factors) per launch of one kernel, from the committed counter summary;
    None if it is missing, lacks the kernel, or a source of the kernel's stage
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_main_workload.txt")
    if not os.path.exists(path):
        return None
    csrc = os.path.join(ROOT, "paper_2510_14564_amd", "csrc")
    stage = stage_of(kernel)
    for line in open(path):
        m = re.match(r"# source-sha256 (\S+) (\w+)", line)
        if m:
            f = os.path.join(csrc, m.group(1))
            changed = not os.path.exists(f) or hashlib.sha256(open(f, "rb").read()).hexdigest()[:16] != m.group(2)
            if changed and stage is not None and m.group(1) in STAGE_SOURCES[stage]:
                return None
            continue
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        if parts[0] == kernel.replace(" ", ""):
            try:
                return float(parts[-1]) * 1e6
            except ValueError:
                return None
    return None


def cpu_baseline(scene, cam, target, tile_stride=8):
    """The FP64 oracle, as it stands, on a bounded sample of one step:
    projection, binning and projection backward over every Gaussian; forward and
    backward compositing over every `tile_stride`-th tile, scaled by the stride."""
    import oracle
    t = {}
    t0 = time.perf_counter()
    pr = oracle.project(scene, cam)
    t["project"] = time.perf_counter() - t0
    rec = pr["rec"]
    t0 = time.perf_counter()
    pl, ranges, _, _ = oracle.bin_sort(rec[:, 0], rec[:, 1], pr["radius"], pr["depth"].astype(np.float32),
                                       cam.width, cam.height)
    t["bin_sort"] = time.perf_counter() - t0
    ntiles = ranges.shape[0]
    mask = np.zeros(ntiles, np.uint8)
    mask[::tile_stride] = 1
    t0 = time.perf_counter()
    img, _, _, _ = oracle.render_fwd(rec, pl, ranges, cam, tile_mask=mask)
    t["render_fwd"] = (time.perf_counter() - t0) * tile_stride
    G = np.sign(img - target.astype(np.float64)) / img.size
    t0 = time.perf_counter()
    g2d = oracle.render_bwd(rec, pl, ranges, cam, G, tile_mask=mask)
    t["render_bwd"] = (time.perf_counter() - t0) * tile_stride
    t0 = time.perf_counter()
    oracle.project_bwd(scene, cam, g2d)
    t["project_bwd"] = time.perf_counter() - t0
    total_ms = 1e3 * sum(t.values())
    return {"value": round(total_ms, 1), "unit": "ms/iter", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"camera 0, N={scene.n}: projection, binning and projection backward on all Gaussians; "
                       f"compositing fwd+bwd on every {tile_stride}th tile ({int(mask.sum())} of {ntiles}), "
                       f"scaled x{tile_stride}"),
            "stages_s": {k: round(v, 3) for k, v in t.items()}}


ADAM_LRS = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "logits": 5e-2, "sh_dc": 2.5e-3,
            "sh_rest": 1.25e-4}


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


class Harness:
    """One workload's scene, cameras, targets and rasterizer on the device."""

    def __init__(self, torch, gs, scenes, cfg, dev, wait_k=False, ncam=None):
        from paper_2510_14564_amd.raster import Rasterizer
        self.torch, self.gs, self.cfg, self.dev = torch, gs, cfg, dev
        log(f"[bench] generating workload {cfg} ...")
        self.scene = scenes.config_scene(cfg)
        ncam = ncam or (32 if cfg == 3 else 1)
        self.cams = [scenes.config_camera(cfg, k) for k in range(ncam)]
        self.params = {k: torch.from_numpy(v).to(dev).requires_grad_(True)
                       for k, v in self.scene.arrays().items() if k != "latents"}
        self.targets = [torch.from_numpy(scenes.target_image(c, 3000 + k)).to(dev) for k, c in enumerate(self.cams)]
        self.partials = torch.empty(gs.L1_PARTIALS, dtype=torch.float32, device=dev)
        self.rast = Rasterizer(self.cams[0], self.scene.sh_degree, device=dev)
        # list capacity for every camera (one waiting bin/sort each), so that
        # the timed steps bin without the host wait: each frame's K is then
        # checked at the next frame and at the end, and an overflow raises
        if not wait_k:
            p = self.params
            with torch.no_grad():
                kmax = 0
                for cam in self.cams:
                    self.rast.set_camera(cam)
                    st = self.rast.forward(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"])
                    kmax = max(kmax, st.k)
            self.rast._alloc_lists(int(kmax * 1.1) + 1024)
            self.rast.async_k = True

    def step(self, i, colour=None, learned=None):
        """One training step without the optimiser: project, bin/sort, forward
        compositing, L1, backward.  learned: a decoder.Decoder for the learned
        colour."""
        from paper_2510_14564_amd.raster import l1_loss, rasterize, rasterize_learned
        p = self.params
        k = i % len(self.cams)
        self.rast.set_camera(self.cams[k])
        for t in p.values():
            t.grad = None
        if learned is None:
            img = rasterize(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], self.rast)
        else:
            learned.latents.grad = None
            learned.params.grad = None
            img = rasterize_learned(p["means"], p["log_scales"], p["quats"], p["logits"], learned, self.rast)
        loss, dimg = l1_loss(img, self.targets[k], self.partials)
        img.backward(dimg)
        return loss

    def run(self, step_fn, label, steps, warmup):
        """Time `steps` steps after `warmup`: per-step HIP events for the mean
        and the p10/p50/p90, then the same steps again under the library's
        kernel timer (HIP events around every launch on its stream) for the
        per-kernel durations."""
        torch = self.torch
        log(f"[bench] {label}: warmup {warmup} steps")
        for i in range(warmup):
            step_fn(i)
        torch.cuda.synchronize()
        log(f"[bench] {label}: timing {steps} steps")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for i in range(steps):
            step_fn(warmup + i)
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        ms = ev[0].elapsed_time(ev[-1]) / steps
        self.gs.kernel_timer_start()
        try:
            for i in range(steps):
                step_fn(warmup + i)
            torch.cuda.synchronize()
        finally:
            kt = self.gs.kernel_timer_stop()
        kernels = {name: {"launches_per_step": c / steps, "avg_us": 1e3 * t / c, "us_per_step": 1e3 * t / steps}
                   for name, (c, t) in kt.items()}
        stages = {}
        for name, kv in kernels.items():
            st = stage_of(name)
            if st is not None:
                stages[st] = stages.get(st, 0.0) + kv["us_per_step"] / 1e3
        log(f"[bench] {label}: {ms:.3f} ms/step (p10 {_pct(per, 10):.3f}, p90 {_pct(per, 90):.3f}); kernels " +
            ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))
        return {"ms": ms, "p10": _pct(per, 10), "p50": _pct(per, 50), "p90": _pct(per, 90), "kernels": kernels,
                "stages_ms": stages}

    def pair_counts(self, first, steps):
        """Algorithmic work of the timed frames, recounted untimed: pairs
        examined and blended by the forward, walked by the backward, and K."""
        torch, gs, p = self.torch, self.gs, self.params
        self.rast.check_async()
        self.rast.async_k = False
        walked, examined, blended, ks = [], [], [], []
        counts = torch.zeros(2, dtype=torch.int64, device=self.dev)
        for i in range(steps):
            self.rast.set_camera(self.cams[(first + i) % len(self.cams)])
            with torch.no_grad():
                st = self.rast.forward(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"])
                gs.render_count(st.n, st.proj, st.point_list, st.ranges, st.k, st.cs, counts)
            walked.append(float(st.n_contrib.to(torch.int64).sum().item()))
            c = counts.cpu().numpy()
            examined.append(float(c[0]))
            blended.append(float(c[1]))
            ks.append(st.k)
        return tuple(float(np.mean(x)) for x in (examined, walked, blended, ks))


def rooflines_of(run, n, deg, npx, ntiles, p_exam, p_walk, p_blend, K, ms_step, cfg):
    """Per-stage algorithmic work over the stages' summed kernel time, the
    dominant kernel's roofline, and the whole step's binding-roofline
    fraction: sum over stages of max(t_HBM, t_ALU) at the published peaks,
    over the measured step time."""
    fwd_flop = FWD_FLOP_EXAMINED * p_exam + FWD_FLOP_BLENDED * p_blend
    bwd_flop = BWD_FLOP_WALKED * p_walk + BWD_FLOP_BLENDED * p_blend
    work = {   # stage -> (algorithmic HBM bytes, algorithmic FP32 flop) per step
        "project": (PROJECT_BYTES_PER_G[deg] * n, 0.0),
        "bin_sort": (BIN_BYTES_PER_G * n + BIN_BYTES_PER_DUP * K + BIN_BYTES_PER_TILE * ntiles, 0.0),
        "render_fwd": (FWD_BYTES_PER_DUP * K + FWD_BYTES_PER_G * n + FWD_BYTES_PER_PX * npx, fwd_flop),
        "l1_loss": (L1_BYTES_PER_PX * npx, 0.0),
        "render_bwd": (BWD_BYTES_PER_DUP * K + BWD_BYTES_PER_G * n + BWD_BYTES_PER_PX * npx, bwd_flop),
        "project_bwd": (PROJECT_BWD_BYTES_PER_G[deg] * n, 0.0),
    }
    stages = {}
    bind_s = hbm_s = 0.0
    for st, (b, f) in work.items():
        t_h = b / (HBM_PEAK_GBS * 1e9)
        t_a = f / (ALU_PEAK_TFLOPS * 1e12)
        bind_s += max(t_h, t_a)
        hbm_s += t_h
        t = run["stages_ms"].get(st)
        if t is None:
            continue
        bound = "alu" if t_a > t_h else "hbm"
        ach = (f / 1e12 if bound == "alu" else b / 1e9) / (t * 1e-3)
        peak = ALU_PEAK_TFLOPS if bound == "alu" else HBM_PEAK_GBS
        stages[st] = {"bound": bound, "achieved": round(ach, 2), "peak": peak,
                      "unit": "TFLOP/s" if bound == "alu" else "GB/s", "frac": round(ach / peak, 4),
                      "kernel_ms": round(t, 4), "hbm_bytes_alg": round(b), "flop_alg": round(f)}
    binding = {"frac": round(bind_s / (ms_step * 1e-3), 4), "hbm_only_frac": round(hbm_s / (ms_step * 1e-3), 4),
               "roofline_ms": round(1e3 * bind_s, 4),
               "definition": "sum over stages of max(algorithmic bytes / 8 TB/s, algorithmic flop / 157.3 TFLOP/s), "
                             "over the measured step time"}
    # dominant kernel: the one with the most time per step
    kern = max(run["kernels"].items(), key=lambda kv: kv[1]["us_per_step"])
    name, kv = kern
    avg_s = kv["avg_us"] * 1e-6
    st = stage_of(name)
    per_launch = 1.0 / max(kv["launches_per_step"], 1e-9)
    if st in ("render_bwd", "render_fwd"):
        flop = (bwd_flop if st == "render_bwd" else fwd_flop) * per_launch
        ach = flop / avg_s / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / ALU_PEAK_TFLOPS, 4), "frac_nonpacked": round(ach / ALU_NONPACKED_TFLOPS, 4),
                "flop_per_launch": round(flop)}
    else:
        b = work.get(st, (0.0, 0.0))[0] * per_launch
        ach = b / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": round(b)}
    tb = counter_traffic_bytes(name) if cfg == 3 else None
    roof.update({"kernel": name, "avg_launch_us": round(kv["avg_us"], 2), "traffic": None if tb is None else round(tb),
                 "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)"})
    return roof, stages, binding


def learned_quality(torch, gs, scenes, dev, epochs=400):
    """Distil the decoder on the learned-colour scene (200k Gaussians, 64
    directions each) and compare its renders over the 32-view orbit at
    800x800 with the SH renders: PSNR against the SH render and the delta
    against a noisy target at the paper's 3DGS PSNR level."""
    from paper_2510_14564_amd.decoder import Decoder, Distiller
    from paper_2510_14564_amd.raster import Rasterizer
    scene = scenes.config_scene(5)
    cams = [scenes.orbit_camera(k, 32, 800, 800) for k in range(32)]
    p = {k: torch.from_numpy(v).to(dev) for k, v in scene.arrays().items() if k != "latents"}
    dec = Decoder(scene.n, device=dev, seed=5, latents_bits=scene.latents)
    t0 = time.perf_counter()
    Distiller(dec, p["sh"], 3, per=64, seed=5001).train(epochs)
    torch.cuda.synchronize()
    t_dist = time.perf_counter() - t0
    rast = Rasterizer(cams[0], 3, device=dev)
    se_mlp = se_noisy_sh = se_noisy_mlp = 0.0
    gen = torch.Generator(device=dev).manual_seed(5002)
    sigma = 0.03569
    for cam in cams:
        rast.set_camera(cam)
        with torch.no_grad():
            ref = rast.forward(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"]).image
            mlp = rast.forward(p["means"], p["log_scales"], p["quats"], p["logits"], dec.colour()).image
            noisy = ref + sigma * torch.randn(ref.shape, generator=gen, device=dev)
            se_mlp += torch.mean((mlp - ref) ** 2).item()
            se_noisy_sh += torch.mean((ref - noisy) ** 2).item()
            se_noisy_mlp += torch.mean((mlp - noisy) ** 2).item()
    psnr = lambda se: 10 * math.log10(len(cams) / se)  # noqa: E731
    return {"psnr_vs_sh_db": round(psnr(se_mlp), 3), "noisy_target_delta_db": round(psnr(se_noisy_sh) -
                                                                                   psnr(se_noisy_mlp), 4),
            "distill_epochs": epochs, "distill_s": round(t_dist, 3)}


def sampling_quality(torch, gs, scenes, dev, cfg, coherent=False):
    """The colour-hash sampling mode against the exact method on camera 0 of
    a workload: PSNR of the sampled render against the exact render, and the
    fraction of list entries merged into a group representative."""
    from paper_2510_14564_amd.raster import Rasterizer
    scene = scenes.config_scene(cfg)
    if coherent:
        scene = scenes.coherent_colour(scene, 1000 * cfg + 77)
    cam = scenes.config_camera(cfg, 0)
    p = {k: torch.from_numpy(v).to(dev) for k, v in scene.arrays().items() if k != "latents"}
    imgs = []
    for sched in (gs.SCHEDULE_BALANCED, gs.SCHEDULE_BALANCED | gs.RENDER_COLOUR_HASH):
        rast = Rasterizer(cam, scene.sh_degree, device=dev, schedule=sched)
        with torch.no_grad():
            st = rast.forward(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"])
        imgs.append(st.image.clamp(0.0, 1.0))
    rep = torch.empty(max(st.k, 1), dtype=torch.int32, device=dev)
    gs.colour_hash_table(st.n, st.proj, st.point_list, st.ranges, st.k, st.cs, None, None, None, rep)
    merged = (rep[:st.k].to(torch.int64) != torch.arange(st.k, device=dev)).double().mean().item()
    mse = torch.mean((imgs[0] - imgs[1]) ** 2).item()
    return {"scene": f"{scenes.CONFIG_NAMES[cfg]}{', coherent colour' if coherent else ''}", "k": st.k,
            "merged_fraction": round(merged, 4), "psnr_vs_exact_db": round(10 * math.log10(1.0 / max(mse, 1e-30)), 3)}


def density_timing(torch, gs, scenes, dev, cfg, rounds=3):
    """One round of density control (Sec. III-C) on a workload's Gaussians:
    ms per round (the call waits once for the output size) and its kernels."""
    scene = scenes.config_scene(cfg)
    n, deg = scene.n, scene.sh_degree
    r = scenes.DENSITY_RADIUS[cfg]
    p = {k: torch.from_numpy(v).to(dev) for k, v in scene.arrays().items() if k != "latents"}
    g = gs.gaussians_struct(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], deg)
    cap = 2 * n
    nc = (deg + 1) ** 2
    out = {"means": torch.empty((3, cap), device=dev), "log_scales": torch.empty((3, cap), device=dev),
           "quats": torch.empty((4, cap), device=dev), "logits": torch.empty(cap, device=dev),
           "sh": torch.empty((nc, 3, cap), device=dev)}
    noise = torch.from_numpy(scenes.density_noise(n, 1000 * cfg + 78)).to(dev)
    ws = torch.empty(gs.density_control_workspace(n), dtype=torch.uint8, device=dev)
    prm = {"radius": r}
    rep = gs.density_control(g, prm, noise, out, cap, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        gs.density_control(g, prm, noise, out, cap, ws)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / rounds
    gs.kernel_timer_start()
    try:
        gs.density_control(g, prm, noise, out, cap, ws)
        torch.cuda.synchronize()
    finally:
        kt = gs.kernel_timer_stop()
    return {"workload": f"{scenes.CONFIG_NAMES[cfg]}: {n} Gaussians, r = {r}, k = 3, alpha = beta = gamma = 1",
            "ms_per_round": round(ms, 4), "kernels_us": {k: round(1e3 * t / c, 2) for k, (c, t) in kt.items()},
            "rho_mean": round(rep["rho_mean"], 3), "rho_std": round(rep["rho_std"], 3), "n_new": rep["n_new"],
            "n_merged": rep["n_merged"], "n_out": rep["n_out"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-colour timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the heavy-workload and learned-colour-workload timings and the decoder quality")
    ap.add_argument("--extras", default="",
                    help="comma-separated subset of the extra timings to run: heavy, learned, density, decoder "
                         "(default: all)")
    ap.add_argument("--compare-plain", action="store_true",
                    help="also time the SH step with the plain and the merged work splits, and with the "
                         "deterministic reduction")
    ap.add_argument("--wait-k", action="store_true",
                    help="bin/sort waits for the entry count every frame (no gs_bin_sort_async)")
    ap.add_argument("--no-sampling", action="store_true", help="skip the colour-hash sampling timing and quality")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="also time a 2 GiB device-to-device copy (achievable HBM bandwidth, counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: only one GPU is supported in this build (got --gpus {args.gpus}); "
              "the multi-GPU camera data-parallel design is documented but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_14564_amd import gs, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = args.config
    hw = Harness(torch, gs, scenes, cfg, dev, wait_k=args.wait_k)
    scene, cams = hw.scene, hw.cams
    n, deg = scene.n, scene.sh_degree
    H, W = cams[0].height, cams[0].width
    npx, ntiles = H * W, cams[0].tiles_x * cams[0].tiles_y

    sh = hw.run(hw.step, "SH colour", args.steps, args.warmup)
    other_splits = None
    if args.compare_plain:
        other_splits = {}
        for name, sched in (("plain", gs.SCHEDULE_PLAIN), ("merged", gs.SCHEDULE_MERGED)):
            hw.rast.schedule = sched
            r = hw.run(hw.step, f"SH colour, {name} work split", args.steps, args.warmup)
            other_splits[name] = {"ms_per_step": round(r["ms"], 4),
                                  "stages_ms": {k: round(v, 4) for k, v in r["stages_ms"].items()}}
        hw.rast.schedule = gs.SCHEDULE_BALANCED
        hw.rast.deterministic = True
        r = hw.run(hw.step, "SH colour, deterministic reduction", args.steps, args.warmup)
        other_splits["balanced, deterministic"] = {"ms_per_step": round(r["ms"], 4),
                                                   "stages_ms": {k: round(v, 4) for k, v in r["stages_ms"].items()}}
        hw.rast.deterministic = False

    # the approximate colour-hash sampling mode (Sec. IV-C.1) on the same steps
    sampled = None
    if not args.no_sampling:
        hw.rast.schedule = gs.SCHEDULE_BALANCED | gs.RENDER_COLOUR_HASH
        sampled = hw.run(hw.step, "SH colour, colour-hash sampling", args.steps, args.warmup)
        hw.rast.schedule = gs.SCHEDULE_BALANCED

    # learned colour on the same scene, cameras and targets: random-init
    # decoder (the step's cost does not depend on the weight values)
    mlp = None
    if not args.no_mlp:
        from paper_2510_14564_amd.decoder import Decoder
        dec = Decoder(n, device=dev, seed=cfg, latents_bits=scene.latents)
        dec.latents.requires_grad_(True)
        dec.params.requires_grad_(True)
        mlp = hw.run(lambda i: hw.step(i, learned=dec), "learned colour", args.steps, args.warmup)

    p_exam, p_walk, p_blend, K = hw.pair_counts(args.warmup, args.steps)
    roof, stage_roofs, binding = rooflines_of(sh, n, deg, npx, ntiles, p_exam, p_walk, p_blend, K, sh["ms"], cfg)

    # one training iteration: the step above plus the fused Adam over every
    # parameter array (run last: it moves the parameters)
    m = {k: torch.zeros_like(v) for k, v in hw.params.items()}
    v = {k: torch.zeros_like(t) for k, t in hw.params.items()}
    it = [0]

    def train_step(i):
        loss = hw.step(i)
        it[0] += 1
        gs.adam_gaussians(n, deg, {k: t.detach() for k, t in hw.params.items()},
                          {k: t.grad for k, t in hw.params.items()}, m, v, ADAM_LRS, it[0])
        return loss

    hw.rast.async_k = not args.wait_k
    train = hw.run(train_step, "training iteration (with Adam)", args.steps, args.warmup)
    hw.rast.check_async()
    adam_ms = train["stages_ms"].get("adam", 0.0)

    def summary(r):
        return {"ms_per_step": round(r["ms"], 4), "p10_ms": round(r["p10"], 4), "p50_ms": round(r["p50"], 4),
                "p90_ms": round(r["p90"], 4), "stages_ms": {k: round(x, 4) for k, x in r["stages_ms"].items()}}

    result = {
        "metric": "fwd+bwd raster ms/iter (SH vs MLP colour), 1M Gaussians @1600x1064",
        "value": round(sh["ms"], 4),
        "unit": "ms/iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sh["ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": {1: "tiny", 2: "skewed", 3: "main", 4: "heavy", 5: "learned colour"}[cfg] +
                   f": {n} Gaussians, SH degree {deg}, {W}x{H}, 16x16 tiles, "
                   f"{len(cams)} camera(s), colour SH, L1 loss",
                   "gaussians": n, "width": W, "height": H, "sh_degree": deg, "colour": "sh",
                   "bin_sort": "waits for K" if args.wait_k else "no host wait (K checked a frame later)",
                   "parallelism": "single GPU"},
        "p10_ms": round(sh["p10"], 4), "p50_ms": round(sh["p50"], 4), "p90_ms": round(sh["p90"], 4),
        "stages_ms": {k: round(x, 4) for k, x in sh["stages_ms"].items()},
        "kernels_avg_us": {k: round(kv["avg_us"], 2) for k, kv in sh["kernels"].items()},
        "pairs_per_step": {"examined_fwd": round(p_exam), "walked_bwd": round(p_walk), "blended": round(p_blend)},
        "k_per_step": round(K),
        "roofline": roof,
        "stage_rooflines": stage_roofs,
        "binding_roofline": binding,
        "training_iteration": dict(summary(train), adam_ms=round(adam_ms, 4),
                                   adam_frac_hbm=round(ADAM_BYTES_PER_G[deg] * n / (adam_ms * 1e-3) / 1e9 /
                                                       HBM_PEAK_GBS, 4) if adam_ms else None),
    }
    if other_splits is not None:
        result["other_work_splits"] = other_splits
    if mlp is not None:
        result["learned_colour"] = dict(summary(mlp), speedup_vs_sh=round(sh["ms"] / mlp["ms"], 4),
                                        speedup_vs_sh_p50=round(sh["p50"] / mlp["p50"], 4))
    if sampled is not None:
        log("[bench] colour-hash sampling quality ...")
        result["colour_hash_sampling"] = dict(
            summary(sampled), speedup_vs_exact=round(sh["ms"] / sampled["ms"], 4),
            speedup_vs_exact_p50=round(sh["p50"] / sampled["p50"], 4),
            approximate=True,
            quality=[sampling_quality(torch, gs, scenes, dev, c, coh) for c in (2, 3) for coh in (False, True)])
    want = set(args.extras.split(",")) if args.extras else {"heavy", "learned", "density", "decoder"}
    if not args.no_extras and cfg == 3:
        extras = {}
        del hw
        torch.cuda.empty_cache()
    if not args.no_extras and cfg == 3 and "heavy" in want:
        h4 = Harness(torch, gs, scenes, 4, dev, wait_k=args.wait_k)
        r4 = h4.run(h4.step, "heavy workload", 5, 2)
        extras["heavy"] = dict(summary(r4), workload=f"heavy: {h4.scene.n} Gaussians, anisotropic, SH degree 3, "
                                                    "1920x1080, orbit camera 0, L1 loss")
        del h4
        torch.cuda.empty_cache()
    if not args.no_extras and cfg == 3 and "learned" in want:
        h5 = Harness(torch, gs, scenes, 5, dev, wait_k=args.wait_k)
        r5 = h5.run(h5.step, "learned-colour workload, SH", args.steps, args.warmup)
        from paper_2510_14564_amd.decoder import Decoder
        dec5 = Decoder(h5.scene.n, device=dev, seed=5, latents_bits=h5.scene.latents)
        dec5.latents.requires_grad_(True)
        dec5.params.requires_grad_(True)
        r5m = h5.run(lambda i: h5.step(i, learned=dec5), "learned-colour workload, decoder", args.steps,
                     args.warmup)
        extras["learned_colour_workload"] = {
            "workload": f"learned colour: {h5.scene.n} Gaussians, 800x800, SH degree 3 vs 16-value BF16 latent + "
                        "32-64-64-3 decoder",
            "sh": summary(r5), "decoder": summary(r5m), "speedup_vs_sh": round(r5["ms"] / r5m["ms"], 4),
            "speedup_vs_sh_p50": round(r5["p50"] / r5m["p50"], 4)}
        del h5
        torch.cuda.empty_cache()
    if not args.no_extras and cfg == 3 and "density" in want:
        log("[bench] density control ...")
        extras["density_control"] = [density_timing(torch, gs, scenes, dev, c) for c in (2, 3)]
    if not args.no_extras and cfg == 3 and "decoder" in want:
        log("[bench] decoder quality (400 distillation epochs, 32 views) ...")
        extras["decoder_quality"] = learned_quality(torch, gs, scenes, dev)
    if not args.no_extras and cfg == 3:
        result["extra_workloads"] = extras
    if args.hbm_probe:
        nbytes = 2 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        result["hbm_probe"] = {"bytes_per_copy": 2 * nbytes, "GB/s": round(2 * nbytes / sec / 1e9, 1)}
        del a, b
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a bounded sample) ...")
        cam0 = cams[0]
        result["cpu_baseline"] = cpu_baseline(scene, cam0, scenes.target_image(cam0, 3000))
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

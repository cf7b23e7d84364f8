#!/usr/bin/env python3
"""Benchmark of one training step of differentiable tile splatting on one GPU.

Workload (default): the main scene -- 1,000,000 Gaussians drawn from 64
isotropic clusters whose weights span 100x, SH degree 3 (48 FP32 coefficients
per Gaussian), rendered at 1600x1064 with 16x16 tiles from a 32-camera orbit of
radius 4.  One step = project, bin/sort, forward compositing (through the
torch.autograd.Function), L1 loss against a seeded target image, backward
compositing and projection backward -- every stage a HIP kernel behind the C
ABI.  Inputs (parameters, cameras, targets) are resident in HBM before timing.

Prints ONE JSON line.  Per-kernel durations come from HIP events recorded on
the stream the kernels run on.
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
# FP32 VALU without packed math: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic work per unit ("Measurement").  FLOPs count an FMA as
# 2 and every other FP32 operation (including exp and reciprocal) as 1.
#   projection: read 44 + 12 (D+1)^2 B of parameters, write the 36 B record +
#               depth + radius + tile count per Gaussian
#   projection backward: read parameters + 36 B of 2D gradients, write
#               parameter gradients (44 + 12 (D+1)^2 B)
#   forward compositing: 14 flop per examined pair (offset, quadratic form,
#               exp, opacity, clamp, two skip tests) + 10 per blended pair
#               (1 - alpha, T update, stop test, weight, three colour FMAs)
#   backward compositing: 14 flop per walked pair (alpha re-evaluation) + 52
#               per blended pair (T recovery, dL/dalpha, light behind, nine
#               gradient terms and their nine sums over pixels)
PROJECT_BYTES_PER_G = {d: 44 + 12 * (d + 1) ** 2 + 48 for d in range(4)}
PROJECT_BWD_BYTES_PER_G = {d: 2 * (44 + 12 * (d + 1) ** 2) + 36 for d in range(4)}
FWD_FLOP_EXAMINED, FWD_FLOP_BLENDED = 14, 10
BWD_FLOP_WALKED, BWD_FLOP_BLENDED = 14, 52


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# kernels of each stage (as named in the rocprofv3 summaries under profiles/)
STAGE_KERNELS = {
    "project": ("k_project<", "k_mlp_fwd<1>"),
    "bin_sort": ("k_depth_keys", "k_os_", "k_rs_hist", "k_rs_scatter", "k_scan_", "k_gather_counts", "k_chunk_",
                 "k_tile_starts", "k_emit", "k_ranges"),
    "render_fwd": ("k_render_fwd_light", "k_render_fwd<false>"),
    "render_bwd": ("k_render_bwd", "k_acc_to_g2d", "k_det_", "k_zero4"),
    "project_bwd": ("k_project_bwd<", "k_mlp_bwd<1>", "k_mlp_reduce"),
}


# sources whose kernels run in each stage
STAGE_SOURCES = {
    "project": ("gs_project.hip", "gs_sh.h", "gs_mlp.hip", "gs_internal.h"),
    "bin_sort": ("gs_binsort.hip", "gs_internal.h"),
    "render_fwd": ("gs_render.hip", "gs_plan.hip", "gs_internal.h"),
    "render_bwd": ("gs_render.hip", "gs_plan.hip", "gs_internal.h"),
    "project_bwd": ("gs_project.hip", "gs_sh.h", "gs_mlp.hip", "gs_internal.h"),
}


def counter_traffic_bytes(stage):
    """Calibrated HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    factors) per call of a stage, from the committed counter summary; None if
    it is missing or any kernel source changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_main_workload.txt")
    if not os.path.exists(path):
        return None
    csrc = os.path.join(ROOT, "paper_2510_14564_amd", "csrc")
    total, seen = 0.0, False
    for line in open(path):
        m = re.match(r"# source-sha256 (\S+) (\w+)", line)
        if m:
            f = os.path.join(csrc, m.group(1))
            changed = not os.path.exists(f) or hashlib.sha256(open(f, "rb").read()).hexdigest()[:16] != m.group(2)
            if changed and m.group(1) in STAGE_SOURCES[stage]:
                return None
            continue
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        name = parts[0]
        if name.startswith(STAGE_KERNELS[stage]) or (name == "k_tile_plan" and stage in ("render_fwd", "render_bwd")):
            try:
                mb = float(parts[-1])
            except ValueError:
                continue
            total += mb * 1e6 * (0.5 if name == "k_tile_plan" else 1.0)
            seen = True
    return total if seen else None


class StageTimer:
    """Records a pair of events on the current stream around each stage."""

    def __init__(self, torch):
        self.torch = torch
        self.events = {}
        self.enabled = False

    def __call__(self, name):
        if not self.enabled:
            return contextlib.nullcontext()
        return self._ctx(name)

    @contextlib.contextmanager
    def _ctx(self, name):
        t = self.torch
        a = t.cuda.Event(enable_timing=True)
        b = t.cuda.Event(enable_timing=True)
        a.record(t.cuda.current_stream())
        yield
        b.record(t.cuda.current_stream())
        self.events.setdefault(name, []).append((a, b))

    def ms(self):
        return {k: [a.elapsed_time(b) for a, b in v] for k, v in self.events.items()}

    def reset(self):
        self.events = {}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-colour timing")
    ap.add_argument("--compare-plain", action="store_true",
                    help="also time the SH step with the plain and the merged work splits, and with the "
                         "deterministic reduction")
    ap.add_argument("--wait-k", action="store_true",
                    help="bin/sort waits for the entry count every frame (no gs_bin_sort_async)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="also time a 2 GiB device-to-device copy (achievable HBM bandwidth, counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: only one GPU is supported in this build (got --gpus {args.gpus}); "
              "the multi-GPU camera data-parallel design is documented but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_14564_amd import gs, scenes
    from paper_2510_14564_amd.raster import Rasterizer, l1_loss, rasterize

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = args.config
    log(f"[bench] generating workload {cfg} ...")
    scene = scenes.config_scene(cfg)
    ncam = 32 if cfg == 3 else 1
    cams = [scenes.config_camera(cfg, k) for k in range(ncam)]
    H, W = cams[0].height, cams[0].width
    params = {k: torch.from_numpy(v).to(dev).requires_grad_(True) for k, v in scene.arrays().items()}
    targets = [torch.from_numpy(scenes.target_image(cams[k], 3000 + k)).to(dev) for k in range(ncam)]
    partials = torch.empty(gs.L1_PARTIALS, dtype=torch.float32, device=dev)
    rast = Rasterizer(cams[0], scene.sh_degree, device=dev)
    # list capacity for the whole orbit (one waiting bin/sort per camera), so
    # that the timed steps can bin without the host wait: each frame's K is
    # then checked at the next frame and at the end, and an overflow would
    # raise instead of passing unnoticed
    if not args.wait_k:
        with torch.no_grad():
            kmax = 0
            for cam in cams:
                rast.set_camera(cam)
                st = rast.forward(params["means"], params["log_scales"], params["quats"], params["logits"],
                                  params["sh"])
                kmax = max(kmax, st.k)
        rast._alloc_lists(int(kmax * 1.1) + 1024)
        rast.async_k = True
    timer = StageTimer(torch)
    rast.timer = timer

    def step(i):
        cam = cams[i % ncam]
        rast.set_camera(cam)
        for p in params.values():
            p.grad = None
        img = rasterize(params["means"], params["log_scales"], params["quats"], params["logits"], params["sh"],
                        rast)
        with timer("l1_loss"):
            loss, dimg = l1_loss(img, targets[i % ncam], partials)
        img.backward(dimg)
        return loss

    def run_timed(step_fn, label):
        log(f"[bench] {label}: warmup {args.warmup} steps")
        for i in range(args.warmup):
            step_fn(i)
        torch.cuda.synchronize()
        # the step time is taken without the per-stage events (their host calls
        # fall where the GPU waits for the host after the bin/sort readback);
        # the same steps then run again with them for the stage breakdown
        log(f"[bench] {label}: timing {args.steps} steps")
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        wall0 = time.perf_counter()
        for i in range(args.steps):
            step_fn(args.warmup + i)
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        timer.reset()
        timer.enabled = True
        for i in range(args.steps):
            step_fn(args.warmup + i)
        torch.cuda.synchronize()
        timer.enabled = False
        ms = t0.elapsed_time(t1) / args.steps
        st_ms = {k: float(np.mean(v)) for k, v in timer.ms().items()}
        log(f"[bench] {label}: {ms:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}); stages " +
            ", ".join(f"{k} {v:.3f}" for k, v in st_ms.items()))
        return ms, st_ms

    ms_step, stage_ms = run_timed(step, "SH colour")
    other_splits = None
    if args.compare_plain:
        other_splits = {}
        for name, sched in (("plain", gs.SCHEDULE_PLAIN), ("merged", gs.SCHEDULE_MERGED)):
            rast.schedule = sched
            p_ms, p_stage = run_timed(step, f"SH colour, {name} work split")
            other_splits[name] = {"ms_per_step": round(p_ms, 4),
                                  "stages_ms": {k: round(v, 4) for k, v in p_stage.items()}}
        rast.schedule = gs.SCHEDULE_BALANCED
        rast.deterministic = True
        p_ms, p_stage = run_timed(step, "SH colour, deterministic reduction")
        other_splits["balanced, deterministic"] = {"ms_per_step": round(p_ms, 4),
                                                   "stages_ms": {k: round(v, 4) for k, v in p_stage.items()}}
        rast.deterministic = False

    # learned colour on the same scene, cameras and targets: random-init
    # decoder (the step's cost does not depend on the weight values)
    mlp_ms, mlp_stage_ms = None, None
    if not args.no_mlp:
        from paper_2510_14564_amd.decoder import Decoder
        from paper_2510_14564_amd.raster import rasterize_learned
        dec = Decoder(scene.n, device=dev, seed=cfg, latents_bits=scene.latents)
        dec.latents.requires_grad_(True)
        dec.params.requires_grad_(True)

        def step_mlp(i):
            cam = cams[i % ncam]
            rast.set_camera(cam)
            for p in list(params.values()) + [dec.latents, dec.params]:
                p.grad = None
            img = rasterize_learned(params["means"], params["log_scales"], params["quats"], params["logits"], dec,
                                    rast)
            with timer("l1_loss"):
                loss, dimg = l1_loss(img, targets[i % ncam], partials)
            img.backward(dimg)
            return loss

        mlp_ms, mlp_stage_ms = run_timed(step_mlp, "learned colour")

    # every frame binned without the wait fitted its lists (else this raises)
    rast.check_async()
    rast.async_k = False
    # algorithmic work of the timed steps (recounted untimed, same cameras)
    walked, examined, blended, ks = [], [], [], []
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    for i in range(args.steps):
        cam = cams[(args.warmup + i) % ncam]
        rast.set_camera(cam)
        with torch.no_grad():
            st = rast.forward(params["means"], params["log_scales"], params["quats"], params["logits"],
                              params["sh"])
            gs.render_count(st.n, st.proj, st.point_list, st.ranges, st.k, rast.cs, counts)
        walked.append(float(st.n_contrib.to(torch.int64).sum().item()))
        c = counts.cpu().numpy()
        examined.append(float(c[0]))
        blended.append(float(c[1]))
        ks.append(st.k)
    torch.cuda.synchronize()
    p_walk, p_exam, p_blend = (float(np.mean(x)) for x in (walked, examined, blended))
    fwd_flop = FWD_FLOP_EXAMINED * p_exam + FWD_FLOP_BLENDED * p_blend
    bwd_flop = BWD_FLOP_WALKED * p_walk + BWD_FLOP_BLENDED * p_blend
    n = scene.n
    deg = scene.sh_degree
    rooflines = {
        "render_bwd": {"bound": "alu", "achieved": bwd_flop / (stage_ms["render_bwd"] * 1e-3) / 1e12,
                       "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s"},
        "render_fwd": {"bound": "alu", "achieved": fwd_flop / (stage_ms["render_fwd"] * 1e-3) / 1e12,
                       "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s"},
        "project": {"bound": "hbm", "achieved": PROJECT_BYTES_PER_G[deg] * n / (stage_ms["project"] * 1e-3) / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"},
        "project_bwd": {"bound": "hbm",
                        "achieved": PROJECT_BWD_BYTES_PER_G[deg] * n / (stage_ms["project_bwd"] * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s"},
    }
    for name, r in rooflines.items():
        r["achieved"] = round(r["achieved"], 2)
        r["frac"] = round(r["achieved"] / r["peak"], 4)
        # the committed counters were taken on the main workload only
        tb = counter_traffic_bytes(name) if cfg == 3 else None
        # measured HBM traffic of the stage per call, as a rate over its time
        r["traffic"] = None if tb is None else round(tb / (stage_ms[name] * 1e-3) / 1e9, 1)
        r["traffic_unit"] = "GB/s"
        r["traffic_bytes_per_call"] = None if tb is None else round(tb)
    dominant = max(("render_bwd", "render_fwd", "project", "project_bwd"), key=lambda s: stage_ms.get(s, 0))
    roof = dict(rooflines[dominant])
    roof["kernel"] = dominant

    result = {
        "metric": "fwd+bwd raster ms/iter (SH vs MLP colour), 1M Gaussians @1600x1064",
        "value": round(ms_step, 4),
        "unit": "ms/iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": {1: "tiny", 2: "skewed", 3: "main", 4: "heavy", 5: "learned colour"}[cfg] +
                   f": {n} Gaussians, SH degree {deg}, {W}x{H}, 16x16 tiles, "
                   f"{ncam} camera(s), colour SH, L1 loss",
                   "gaussians": n, "width": W, "height": H, "sh_degree": deg, "colour": "sh",
                   "bin_sort": "waits for K" if args.wait_k else "no host wait (K checked a frame later)",
                   "parallelism": "single GPU"},
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "pairs_per_step": {"examined_fwd": round(p_exam), "walked_bwd": round(p_walk), "blended": round(p_blend)},
        "k_per_step": round(float(np.mean(ks))),
        "roofline": roof,
        "rooflines": rooflines,
    }
    if other_splits is not None:
        result["other_work_splits"] = other_splits
    if mlp_ms is not None:
        result["learned_colour"] = {"ms_per_step": round(mlp_ms, 4),
                                    "stages_ms": {k: round(v, 4) for k, v in mlp_stage_ms.items()},
                                    "speedup_vs_sh": round(ms_step / mlp_ms, 4)}
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

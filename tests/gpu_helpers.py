"""Shared helpers for the GPU parity tests: upload seeded inputs, run the HIP
stages through the C ABI, and compare against the FP64 oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

DEV = "cuda"

# tolerances (parity section)
PIX_ATOL = 1e-4          # pixels and final_T, absolute
GRAD_RTOL = 1e-3         # gradients: |g - g*| <= 1e-3 max(|g*|, 1e-3 max|g*|, 3e-2 mass)
# mass = sum of |per-pair terms| of g*: an FP32 sum of n terms carries a
# rounding error up to n * 2^-24 of its mass (about sqrt(n) * 2^-24 in
# practice); a Gaussian covering 10^4-10^5 pixels reaches a few 1e-5 of it
MASS_FLOOR = 3e-2
PROJ_RTOL = 2e-5         # projected quantities, relative to the field's scale


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def upload(scene):
    return {k: to_dev(v) for k, v in scene.arrays().items()}


def gpu_project(gs, scene, cam):
    p = upload(scene)
    g = gs.gaussians_struct(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], scene.sh_degree)
    out = gs.ProjectedBuffers(scene.n, DEV)
    gs.project(g, gs.camera_struct(cam), out)
    torch.cuda.synchronize()
    return p, g, out


def proj_host(out):
    rec = out.records.cpu().numpy()
    return dict(rec=rec, u=rec[:, 0], v=rec[:, 1], depth=out.depth.cpu().numpy(),
                radius=out.radius.cpu().numpy(), tiles_touched=out.tiles_touched.cpu().numpy())


def grad_close(got, want, rtol=GRAD_RTOL, name="", mass=None, stats=None):
    """Relative error 1e-3 against max(|g*|, 1e-3 max|g*|) and, when the oracle's
    term mass is given, 1e-2 of it: a sum that cancels by more than 100x is
    judged against its terms, which is what its rounding error scales with.
    Returns the worst ratio to the plain (mass-free) relative bound."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = np.abs(want).max() if want.size else 0.0
    ref = np.maximum(np.abs(want), 1e-3 * scale)
    plain = rtol * ref
    bound = plain if mass is None else rtol * np.maximum(ref, MASS_FLOOR * np.asarray(mass, np.float64))
    err = np.abs(got - want)
    bad = err > bound + 1e-30
    if bad.any():
        i = np.argmax(err - bound)
        raise AssertionError(f"{name}: {bad.sum()}/{bad.size} outside tolerance; worst idx {np.unravel_index(i, want.shape)} "
                             f"got {got.flat[i]!r} want {want.flat[i]!r} (scale {scale:.3e})")
    if stats is not None:
        stats[name] = int((err > plain + 1e-30).sum())
    return float((err / (ref + 1e-30)).max()) if want.size else 0.0


def chain_mass(scene, cam, *weights):
    """Term mass of the projection backward: for each weights[n][9] >= 0, per
    parameter sum_j |d param / d record_j| weights[:, j], from one oracle pass
    per record channel j (a Gaussian's parameter gradient depends on its own
    record gradient only).  With weights = |g2d| this is the sum of the chain
    rule's per-channel terms, which the FP32 rounding of a cancelling
    parameter gradient scales with."""
    n = scene.n
    out = [None] * len(weights)
    for j in range(9):
        e = np.zeros((n, 9))
        e[:, j] = 1.0
        col = oracle.project_bwd(scene, cam, e)
        for w_i, w in enumerate(weights):
            acc = {k: np.abs(v) * w[:, j] for k, v in col.items()}
            out[w_i] = acc if out[w_i] is None else {k: out[w_i][k] + acc[k] for k in acc}
    return out


def gpu_bin_sort(gs, n, out, cam, capacity=None):
    cs = gs.camera_struct(cam)
    cap = capacity if capacity is not None else max(1024, int(out.tiles_touched.sum().item()))
    ws = torch.empty(gs.bin_sort_workspace(n, cap, cs), dtype=torch.uint8, device=DEV)
    pl = torch.empty(max(cap, 1), dtype=torch.int32, device=DEV)
    ranges = torch.empty((gs.n_tiles(cam), 2), dtype=torch.int32, device=DEV)
    k = gs.bin_sort(n, out, cs, ws, pl, ranges)
    torch.cuda.synchronize()
    return k, pl, ranges


def gpu_render(gs, n, out, pl, ranges, k, cam, schedule=1):
    cs = gs.camera_struct(cam)
    H, W = cam.height, cam.width
    image = torch.empty((3, H, W), dtype=torch.float32, device=DEV)
    fT = torch.empty((H, W), dtype=torch.float32, device=DEV)
    nc = torch.empty((H, W), dtype=torch.int32, device=DEV)
    ck = torch.empty(gs.render_ckpt_floats(k, cs), dtype=torch.float32, device=DEV)
    gs.render_fwd(n, out, pl, ranges, k, cs, image, fT, nc, ck, schedule=schedule)
    torch.cuda.synchronize()
    return image, fT, nc, ck


def gpu_render_bwd(gs, n, out, pl, ranges, k, cam, fT, nc, ck, G, deterministic=False, schedule=1):
    cs = gs.camera_struct(cam)
    g2d = torch.empty((gs.G2D, n), dtype=torch.float32, device=DEV)
    ws = torch.empty(max(gs.render_bwd_workspace(n, k, cs, deterministic), 1), dtype=torch.uint8, device=DEV)
    gs.render_bwd(n, out, pl, ranges, k, cs, fT, nc, ck, G, g2d, ws, deterministic, schedule=schedule)
    torch.cuda.synchronize()
    return g2d


def compare_render(image, fT, nc, o_img, o_T, o_nc, o_flags, mask=None):
    """Pixels within PIX_ATOL except pixels the oracle flags as near a threshold;
    n_contrib exact except flagged pixels.  Returns (max err, #flagged)."""
    img = image.cpu().numpy().astype(np.float64)
    T = fT.cpu().numpy().astype(np.float64)
    n = nc.cpu().numpy()
    ok = (o_flags == 0) if mask is None else ((o_flags == 0) & mask)
    err_img = np.abs(img - o_img).max(axis=0)
    assert (err_img[ok] <= PIX_ATOL).all(), f"max pixel err {err_img[ok].max()}"
    assert (np.abs(T - o_T)[ok] <= PIX_ATOL).all(), f"max final_T err {np.abs(T - o_T)[ok].max()}"
    mism = (n != o_nc) & ok
    assert not mism.any(), f"{mism.sum()} unflagged n_contrib mismatches"
    return float(err_img[ok].max()) if ok.any() else 0.0, int((o_flags != 0).sum())

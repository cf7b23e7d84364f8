"""Staged parity of the HIP path against the FP64 oracle (needs the GPU).

Each stage feeds the oracle the HIP path's own FP32 outputs of the previous
stage (widened exactly), so threshold decisions that FP32 and FP64 may take
differently are located, flagged and counted rather than hidden:
  1 project     : u, v and depth within 4x their FP32 rounding bound; opacity
                  and colour within 1e-6 / 2e-5; conic within 2e-5 + 4e-7 cond(Sigma') of its
                  largest entry; radius exact unless 3 sqrt(lambda) is within
                  2e-5 of an integer (flagged)
  2 bin/sort    : tiles_touched, K, point_list and ranges bit-exact
  3 render fwd  : pixels and final_T within 1e-4; n_contrib exact, except at
                  pixels the oracle flags as within 1e-4 (relative) of the
                  1/255, 1e-4 or 0.99 thresholds
  4 render bwd  : per-Gaussian record gradients within 1e-3 relative, against
                  max(|g*|, 1e-3 max|g*|, 1e-2 sum|terms|) -- a sum that cancels
                  by over 100x is judged against its terms, which its rounding
                  error scales with; flagged pixels get dL = 0
  5 project bwd : parameter gradients, same tolerance
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import (DEV, PROJ_RTOL, compare_render, gpu_bin_sort, gpu_project, gpu_render, gpu_render_bwd,
                         grad_close, proj_host, say, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_14564_amd import gs as mod
    return mod


def _case(name):
    if name == "tiny":
        return scenes.config_scene(1), scenes.config_camera(1)
    if name == "tiny_bg":
        return scenes.config_scene(1), scenes.config_camera(1, bg=(0.2, 0.5, 0.8))
    if name == "ragged":
        s = scenes.skewed_scene(20000, 77, n_clusters=16, log_scale_mean=-3.6, sh_degree=3)
        return s, scenes.pinhole(100, 70, 60.0, np.eye(3), (0.05, -0.02, 3.0), bg=(0.1, 0.0, 0.3))
    if name == "sh1_sh2":
        s = scenes.uniform_scene(6000, 12, log_scale_mean=-3.2, sh_degree=2)
        return s, scenes.orbit_camera(5, 32, 200, 136, 3.5, 60.0)
    if name == "skewed":
        return scenes.config_scene(2), scenes.config_camera(2)
    raise KeyError(name)


CASES = ["tiny", "tiny_bg", "ragged", "sh1_sh2", "skewed"]


def _project_stage(gs, scene, cam):
    p, g, out = gpu_project(gs, scene, cam)
    h = proj_host(out)
    o = oracle.project(scene, cam)
    flag_r = (o["flags"] & 1) != 0
    flag_cull = (o["flags"] & 2) != 0
    live_g = h["radius"] > 0
    live_o = o["radius"] > 0
    assert np.array_equal(live_g[~flag_cull], live_o[~flag_cull]), "cull decisions differ"
    both = live_g & live_o
    ok_r = both & ~flag_r
    assert np.array_equal(h["radius"][ok_r], o["radius"][ok_r]), "radius mismatch"
    rg, ro = h["rec"][both], o["rec"][both]
    # FP32 rounding bounds for t = W mu + t_cw and u = fx tx / tz + cx (4x safety):
    #   |dt_i| <= 3 eps (sum_j |W_ij mu_j| + |t_i|),
    #   |du| <= fx/tz |dtx| + |u - cx| (4 eps + |dtz|/tz) + eps (|u| + |cx|)
    eps = 2.0 ** -24
    W = np.asarray(cam.R_cw, np.float64)
    mu = scene.means.astype(np.float64)[:, both]
    tc = np.asarray(cam.t_cw, np.float64)
    mag = np.abs(W) @ np.abs(mu) + np.abs(tc)[:, None]
    dt = 3 * eps * mag
    tz = o["depth"][both]
    for j, name, f, c in ((0, "u", cam.fx, cam.cx), (1, "v", cam.fy, cam.cy)):
        bound = f / tz * dt[j] + np.abs(ro[:, j] - c) * (4 * eps + dt[2] / tz) + eps * (np.abs(ro[:, j]) + c)
        err = np.abs(rg[:, j] - ro[:, j])
        assert (err <= 4 * bound).all(), (name, err.max(), (err / bound).max())
    # the FP32 error of a 2x2 inverse grows with the condition number of Sigma'
    A, B, C = ro[:, 2], ro[:, 3], ro[:, 4]
    disc = np.sqrt(((A - C) / 2) ** 2 + B ** 2)
    cond = ((A + C) / 2 + disc) / ((A + C) / 2 - disc)
    cs = np.abs(ro[:, 2:5]).max(axis=1)
    err = (np.abs(rg[:, 2:5] - ro[:, 2:5]).max(axis=1)) / cs
    tol = PROJ_RTOL + 4e-7 * cond
    assert (err <= tol).all(), ("conic", err.max(), (err / tol).max())
    assert np.abs(rg[:, 5] - ro[:, 5]).max() <= 1e-6, "opacity"
    assert np.abs(rg[:, 6:9] - ro[:, 6:9]).max() <= PROJ_RTOL, ("colour", np.abs(rg[:, 6:9] - ro[:, 6:9]).max())
    dz = np.abs(h["depth"][both] - o["depth"][both])
    assert (dz <= 4 * dt[2]).all(), ("depth", (dz / dt[2]).max())
    # culled records are zero and have no tiles
    assert (h["tiles_touched"][~live_g] == 0).all() and (h["rec"][~live_g] == 0).all()
    say(f"  project: {both.sum()} live, {flag_r.sum()} radius-flagged")
    return p, g, out, h, o


@pytest.mark.parametrize("name", CASES)
def test_staged_parity(gs, name):
    scene, cam = _case(name)
    say(f"[parity {name}] n={scene.n} {cam.width}x{cam.height} deg={scene.sh_degree}")
    p, g, out, h, o = _project_stage(gs, scene, cam)

    # ---- 2: bin/sort bit-exact on the HIP path's FP32 projection
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    o_pl, o_ranges, o_tt, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], cam.width, cam.height)
    assert np.array_equal(h["tiles_touched"].astype(np.int64), o_tt), "tiles_touched"
    assert k == len(o_pl), (k, len(o_pl))
    assert np.array_equal(pl[:k].cpu().numpy().view(np.uint32), o_pl), "point_list"
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), o_ranges), "ranges"
    nt = (o_ranges[:, 1] - o_ranges[:, 0]).astype(np.int64)
    say(f"  bin/sort: K={k}, max list {nt.max()}, empty tiles {(nt == 0).sum()}")

    # ---- 3: render forward
    image, fT, nc, ck = gpu_render(gs, scene.n, out, pl, ranges, k, cam)
    o_img, o_T, o_nc, o_fl = oracle.render_fwd(h["rec"][:, :9], o_pl, o_ranges, cam, margin=1e-4)
    err, nflag = compare_render(image, fT, nc, o_img, o_T, o_nc, o_fl)
    say(f"  render fwd: max err {err:.2e}, flagged pixels {nflag}")
    # the other work splits give the same image bit for bit
    for sched in (gs.SCHEDULE_PLAIN, gs.SCHEDULE_MERGED):
        image_p, fT_p, nc_p, _ = gpu_render(gs, scene.n, out, pl, ranges, k, cam, schedule=sched)
        assert torch.equal(image, image_p) and torch.equal(fT, fT_p) and torch.equal(nc, nc_p), sched

    # ---- 4: render backward (flagged pixels carry no upstream gradient)
    G = scenes.upstream_grad(cam, 1001)
    G[:, o_fl != 0] = 0.0
    g2d = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, to_dev(G))
    o_g2d, o_mass = oracle.render_bwd(h["rec"][:, :9], o_pl, o_ranges, cam, G, with_mass=True)
    g2d_h = g2d.cpu().numpy().T
    worst = 0.0
    mass_used = {}
    for j, nm in enumerate("u v Sxx Sxy Syy o r g b".split()):
        worst = max(worst, grad_close(g2d_h[:, j], o_g2d[:, j], name=f"g2d.{nm}", mass=o_mass[:, j],
                                      stats=mass_used))
    say(f"  render bwd: worst rel err {worst:.2e}; entries judged against term mass: "
        f"{sum(mass_used.values())} of {g2d_h.size}")
    # the other work splits: same gradients up to the order of the atomic sums
    for sched in (gs.SCHEDULE_PLAIN, gs.SCHEDULE_MERGED):
        g2d_p = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, to_dev(G),
                               schedule=sched).cpu().numpy().T
        for j, nm in enumerate("u v Sxx Sxy Syy o r g b".split()):
            grad_close(g2d_p[:, j], o_g2d[:, j], name=f"schedule {sched} g2d.{nm}", mass=o_mass[:, j])

    # ---- 5: projection backward from the HIP path's g2d
    grads = {kk: torch.empty_like(v) for kk, v in p.items()}
    gs.project_bwd(g, gs.camera_struct(cam), g2d, grads)
    torch.cuda.synchronize()
    o_gr = oracle.project_bwd(scene, cam, g2d_h.astype(np.float64))
    skip = (o["flags"] & 0b1110) != 0
    worst = 0.0
    for kk in ("means", "log_scales", "quats", "logits", "sh"):
        got = grads[kk].cpu().numpy()
        want = o_gr[kk]
        sel = ~skip
        worst = max(worst, grad_close(got[..., sel], want[..., sel], name=kk))
    say(f"  project bwd: worst rel err {worst:.2e}")


def test_empty_and_fully_culled_scenes(gs):
    cam = scenes.config_camera(1, bg=(0.3, 0.2, 0.1))
    for label, scene in (("empty", scenes.uniform_scene(0, 1)), ("behind", scenes.uniform_scene(300, 2))):
        say(f"[edge {label}]")
        if label == "behind":
            scene.means[2] = -5.0
        n = scene.n
        out = gs.ProjectedBuffers(n, DEV)
        if n:
            p, g, out = gpu_project(gs, scene, cam)
        k, pl, ranges = gpu_bin_sort(gs, n, out, cam, capacity=1024)
        assert k == 0 and (ranges.cpu().numpy() == 0).all()
        image, fT, nc, _ = gpu_render(gs, n, out, pl, ranges, k, cam)
        bg = np.asarray(cam.bg, np.float32)
        assert np.array_equal(image.cpu().numpy(), np.broadcast_to(bg[:, None, None], (3, 128, 128)))
        assert (fT.cpu().numpy() == 1).all() and (nc.cpu().numpy() == 0).all()


def test_capacity_overflow_reports_required_size(gs):
    scene, cam = _case("tiny")
    p, g, out = gpu_project(gs, scene, cam)
    with pytest.raises(gs.GsError) as ei:
        gpu_bin_sort(gs, scene.n, out, cam, capacity=100)
    assert ei.value.status == gs.GS_ERR_CAPACITY
    want = int(out.tiles_touched.sum().item())
    assert ei.value.required == want
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam, capacity=want)
    assert k == want


def test_l1_loss(gs):
    rng = np.random.default_rng(3)
    a = rng.random((3, 37, 53), dtype=np.float32)
    b = rng.random((3, 37, 53), dtype=np.float32)
    from paper_2510_14564_amd.raster import l1_loss
    loss, grad = l1_loss(to_dev(a), to_dev(b))
    torch.cuda.synchronize()
    want = np.abs(a.astype(np.float64) - b).mean()
    assert abs(loss.item() - want) < 1e-6
    assert np.array_equal(np.sign(grad.cpu().numpy()), np.sign(a - b))
    assert np.allclose(np.abs(grad.cpu().numpy()), 1.0 / a.size)


def test_main_workload_sampled_parity(gs):
    """The bench's workload and launch configuration (1M Gaussians, SH degree 3,
    1600x1064, orbit camera 0, balanced work split): projection and the whole
    bin/sort checked in full; compositing forward and backward on every 16th
    tile, which the oracle computes tile by tile (the upstream gradient is zero
    elsewhere, so the HIP backward's sums hold exactly those tiles' terms)."""
    scene, cam = scenes.config_scene(3), scenes.config_camera(3, 0)
    say(f"[parity main] n={scene.n} {cam.width}x{cam.height}")
    p, g, out, h, o = _project_stage(gs, scene, cam)
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    o_pl, o_ranges, o_tt, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], cam.width, cam.height)
    assert k == len(o_pl), (k, len(o_pl))
    assert np.array_equal(pl[:k].cpu().numpy().view(np.uint32), o_pl), "point_list"
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), o_ranges), "ranges"
    say(f"  bin/sort: K={k} bit-exact")
    ntiles = o_ranges.shape[0]
    tmask = np.zeros(ntiles, np.uint8)
    tmask[::16] = 1
    tx = (cam.width + 15) // 16
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    pix_mask = tmask[(ys // 16) * tx + (xs // 16)].astype(bool)
    image, fT, nc, ck = gpu_render(gs, scene.n, out, pl, ranges, k, cam)
    o_img, o_T, o_nc, o_fl = oracle.render_fwd(h["rec"][:, :9], o_pl, o_ranges, cam, margin=1e-4, tile_mask=tmask)
    err, nflag = compare_render(image, fT, nc, o_img, o_T, o_nc, o_fl, mask=pix_mask)
    say(f"  render fwd on {int(tmask.sum())} tiles: max err {err:.2e}, flagged pixels {nflag}")
    G = scenes.upstream_grad(cam, 3001)
    G[:, ~pix_mask] = 0.0
    G[:, o_fl != 0] = 0.0
    o_g2d, o_mass = oracle.render_bwd(h["rec"][:, :9], o_pl, o_ranges, cam, G, tile_mask=tmask, with_mass=True)
    g2d = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, to_dev(G))
    g2d_h = g2d.cpu().numpy().T
    worst = 0.0
    used = {}
    for j, nm in enumerate("u v Sxx Sxy Syy o r g b".split()):
        worst = max(worst, grad_close(g2d_h[:, j], o_g2d[:, j], name=f"g2d.{nm}", mass=o_mass[:, j], stats=used))
    say(f"  entries judged against term mass: {sum(used.values())} of {g2d_h.size}")
    grads = {kk: torch.empty_like(v) for kk, v in p.items()}
    gs.project_bwd(g, gs.camera_struct(cam), g2d, grads)
    torch.cuda.synchronize()
    o_gr = oracle.project_bwd(scene, cam, g2d_h.astype(np.float64))
    sel = (o["flags"] & 0b1110) == 0
    for kk in ("means", "log_scales", "quats", "logits", "sh"):
        grad_close(grads[kk].cpu().numpy()[..., sel], o_gr[kk][..., sel], name=kk)
    say(f"  render bwd + project bwd: worst rel err {worst:.2e}")

"""Staged parity of the HIP path against the FP64 oracle (needs the GPU).

Each stage feeds the oracle the HIP path's own FP32 outputs of the previous
stage (widened exactly), so threshold decisions that FP32 and FP64 may take
differently are located, flagged and counted rather than hidden:
  1 project     : u, v and depth within 4x their FP32 rounding bound; opacity
                  and colour within 1e-6 / 2e-5; conic within 2e-5 + 4e-7 cond(Sigma') of its
                  largest entry; radius exact unless 3 sqrt(lambda) is within
                  2e-5 of an integer (flagged)
  2 bin/sort    : tiles_touched, K, point_list and ranges bit-exact
  3 render fwd  : every pixel: colour and final_T within 1e-4, n_contrib
                  exact.  A pixel with a decision near its threshold (alpha
                  within 1e-5 of 1/255, o e^power within 1e-5 of 0.99, T'
                  within 1e-4 plus its accumulated FP32 bound of 1e-4) must be
                  one of the oracle's outcomes over both branches of those
                  decisions; the oracle then follows the branch the HIP path
                  took there (counts per decision type are reported)
  4 render bwd  : per-Gaussian record gradients within 1e-3 relative, against
                  max(|g*|, 1e-3 max|g*|, 1e-2 sum|terms|) -- a sum that cancels
                  by over 100x is judged against its terms, which its rounding
                  error scales with; the oracle's conic gradients are carried to
                  the covariance Sigma' (the HIP path's form) in FP64; only
                  pixels whose branch cannot be identified get dL = 0
  5 project bwd : parameter gradients, same tolerance, with the chain rule's
                  term mass sum_j |d param / d record_j g2d_j| in place of the
                  render's (a quaternion gradient can cancel by 1000x)
  6 end to end  : raw parameters on both sides (no HIP intermediate reaches
                  the oracle); tiles whose lists differ are validated and left
                  out, the rest meet the tolerances above
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import (DEV, E2E_MARGINS, GRAD_RTOL, MASS_FLOOR, PROJ_RTOL, chain_mass, check_render, fmt_flags,
                         gpu_bin_sort, gpu_project, gpu_render, gpu_render_bwd, grad_close, oracle_render_bwd_sigma,
                         proj_host, record_sensitivity, say, sigma_to_conic_grad, to_dev, upload)

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


def _record_bounds(scene, cam, o):
    """Per-Gaussian FP32 error bounds of the projection's record fields
    (u, v, A, B, C, opacity, r, g, b) around the oracle's FP64 values, as the
    projection stage checks them: u, v from the rounding of t = W mu + t_cw
    and of the perspective division; the conic 2e-5 + 4e-7 cond(Sigma') of its
    largest entry; opacity 1e-6; colour 2e-5."""
    eps = 2.0 ** -24
    rec = o["rec"]
    W = np.asarray(cam.R_cw, np.float64)
    mu = scene.means.astype(np.float64)
    tc = np.asarray(cam.t_cw, np.float64)
    dt = 3 * eps * (np.abs(W) @ np.abs(mu) + np.abs(tc)[:, None])
    tz = np.where(o["depth"] > 0, o["depth"], 1.0)
    out = np.zeros((scene.n, 9))
    for j, f, c in ((0, cam.fx, cam.cx), (1, cam.fy, cam.cy)):
        out[:, j] = 4 * (f / tz * dt[j] + np.abs(rec[:, j] - c) * (4 * eps + dt[2] / tz) + eps * (np.abs(rec[:, j]) + c))
    A, B, C = rec[:, 2], rec[:, 3], rec[:, 4]
    disc = np.sqrt(((A - C) / 2) ** 2 + B ** 2)
    den = (A + C) / 2 - disc
    cond = np.where(den > 0, ((A + C) / 2 + disc) / np.where(den > 0, den, 1.0), 0.0)
    out[:, 2:5] = ((PROJ_RTOL + 4e-7 * cond) * np.abs(rec[:, 2:5]).max(axis=1))[:, None]
    out[:, 5] = 1e-6
    out[:, 6:9] = PROJ_RTOL
    out[o["radius"] <= 0] = 0.0
    return out


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
    _, _, _, flips, amb, st = check_render(image, fT, nc, h["rec"][:, :9], o_pl, o_ranges, cam)
    say(f"  render fwd: max err {st['max_err']:.2e}; " + fmt_flags(st))
    # the other work splits give the same image bit for bit
    for sched in (gs.SCHEDULE_PLAIN, gs.SCHEDULE_MERGED):
        image_p, fT_p, nc_p, _ = gpu_render(gs, scene.n, out, pl, ranges, k, cam, schedule=sched)
        assert torch.equal(image, image_p) and torch.equal(fT, fT_p) and torch.equal(nc, nc_p), sched

    # ---- 4: render backward (the oracle on the HIP path's branches)
    G = scenes.upstream_grad(cam, 1001)
    G[:, amb] = 0.0
    g2d = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, to_dev(G))
    _, o_g2d, o_mass = oracle_render_bwd_sigma(h["rec"][:, :9], o_pl, o_ranges, cam, G, flips=flips)
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
    o_gr = oracle.project_bwd(scene, cam, sigma_to_conic_grad(o["rec"], g2d_h))
    (cm,) = chain_mass(scene, cam, np.abs(g2d_h.astype(np.float64)))
    sel = (o["flags"] & 0b1110) == 0
    worst = 0.0
    for kk in ("means", "log_scales", "quats", "logits", "sh"):
        got = grads[kk].cpu().numpy()
        want = o_gr[kk]
        worst = max(worst, grad_close(got[..., sel], want[..., sel], name=kk, mass=cm[kk][..., sel]))
    say(f"  project bwd: worst rel err {worst:.2e}")
    # the same from the projection's colour gradient (d colour / d direction
    # and the clamp mask, written by gs_project) instead of the SH coefficients
    assert out.colour_grad is not None
    grads_j = {kk: torch.empty_like(v) for kk, v in p.items()}
    gs.project_bwd(g, gs.camera_struct(cam), g2d, grads_j, proj=out)
    torch.cuda.synchronize()
    worst = 0.0
    for kk in ("means", "log_scales", "quats", "logits", "sh"):
        got = grads_j[kk].cpu().numpy()
        worst = max(worst, grad_close(got[..., sel], o_gr[kk][..., sel], name=f"{kk} (colour_grad)",
                                      mass=cm[kk][..., sel]))
    say(f"  project bwd from colour_grad: worst rel err {worst:.2e}")


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
    tmask = np.zeros(o_ranges.shape[0], np.uint8)
    tmask[::16] = 1
    _sampled_compositing(gs, scene, cam, p, g, out, h, o, pl, ranges, k, o_pl, o_ranges, tmask, 3001)


def _sampled_compositing(gs, scene, cam, p, g, out, h, o, pl, ranges, k, o_pl, o_ranges, tmask, seed):
    """Forward and backward compositing, then projection backward, checked on
    the tiles of `tmask` (the upstream gradient is zero elsewhere, so the HIP
    backward's sums hold exactly those tiles' terms)."""
    tx = (cam.width + 15) // 16
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    pix_mask = tmask[(ys // 16) * tx + (xs // 16)].astype(bool)
    image, fT, nc, ck = gpu_render(gs, scene.n, out, pl, ranges, k, cam)
    _, _, _, flips, amb, st = check_render(image, fT, nc, h["rec"][:, :9], o_pl, o_ranges, cam, tile_mask=tmask,
                                           pix_mask=pix_mask)
    say(f"  render fwd on {int(tmask.sum())} tiles: max err {st['max_err']:.2e}; " + fmt_flags(st))
    G = scenes.upstream_grad(cam, seed)
    G[:, ~pix_mask] = 0.0
    G[:, amb] = 0.0
    _, o_g2d, o_mass = oracle_render_bwd_sigma(h["rec"][:, :9], o_pl, o_ranges, cam, G, tile_mask=tmask,
                                               flips=flips)
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
    o_gr = oracle.project_bwd(scene, cam, sigma_to_conic_grad(o["rec"], g2d_h))
    (cm,) = chain_mass(scene, cam, np.abs(g2d_h.astype(np.float64)))
    sel = (o["flags"] & 0b1110) == 0
    for kk in ("means", "log_scales", "quats", "logits", "sh"):
        grad_close(grads[kk].cpu().numpy()[..., sel], o_gr[kk][..., sel], name=kk, mass=cm[kk][..., sel])
    say(f"  render bwd + project bwd: worst rel err {worst:.2e}")


def test_projection_row_offsets_beyond_int32(gs):
    """Projection and its backward (both colour paths) at n = 48M, SH degree
    3: the last SH rows start beyond 2^31 elements (47 n > 2^31), so row
    offsets must be formed in 64 bits.  The scene is a 20k-Gaussian scene
    repeated 2,400 times, and every Gaussian's work depends only on its own
    parameters, so each output must equal bit for bit that of its copy in a
    run on the small scene, whose projection is checked against the oracle
    here and whose backward the staged test checks."""
    small, cam = _case("ragged")
    n0, reps = small.n, 2400
    n = n0 * reps
    assert small.sh_degree == 3 and 47 * n > 2 ** 31
    say(f"[large n] n={n}")
    p0, g0, out0, _, _ = _project_stage(gs, small, cam)
    cs = gs.camera_struct(cam)
    rng = torch.Generator(device=DEV).manual_seed(4242)
    g2d0 = torch.randn((9, n0), generator=rng, device=DEV, dtype=torch.float32)
    want = {}
    for path, proj in (("sh", None), ("jacobian", out0)):
        gr = {k: torch.empty_like(v) for k, v in p0.items()}
        gs.project_bwd(g0, cs, g2d0, gr, proj=proj)
        want[path] = gr
    torch.cuda.synchronize()

    def tile(v):
        return v.repeat(*([1] * (v.dim() - 1)), reps)

    p = {k: tile(v) for k, v in p0.items()}
    g = gs.gaussians_struct(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], 3)
    out = gs.ProjectedBuffers(n, DEV)
    gs.project(g, cs, out)
    torch.cuda.synchronize()
    # the last two copies in full and 100k Gaussians drawn over the whole range
    idx = torch.cat([torch.arange(n - 2 * n0, n, device=DEV),
                     torch.randint(0, n, (100000,), generator=rng, device=DEV)])
    src = idx % n0
    assert torch.equal(out.records[idx], out0.records[src]), "records"
    for name in ("depth", "radius", "tiles_touched"):
        assert torch.equal(getattr(out, name)[idx], getattr(out0, name)[src]), name
    assert torch.equal(out.colour_grad[:, idx], out0.colour_grad[:, src]), "colour_grad"
    g2d = tile(g2d0)
    for path, proj in (("sh", None), ("jacobian", out)):
        gr = {k: torch.empty_like(v) for k, v in p.items()}
        gs.project_bwd(g, cs, g2d, gr, proj=proj)
        torch.cuda.synchronize()
        for k in gr:
            assert torch.equal(gr[k][..., idx], want[path][k][..., src]), (path, k)
        del gr
    say(f"  projection and backward at n={n}: bit-equal to the small scene's run")


def test_heavy_workload_parity(gs):
    """Heavy workload (3M anisotropic Gaussians, 1920x1080, about 2.7e8
    entries) in the bench's launch configuration.  The whole bin/sort is
    checked without the oracle's full sort: per-tile counts and ranges
    against the oracle's rectangles, every entry's Gaussian covering its tile,
    and every tile's list strictly increasing in (depth bits, index) -- equal
    counts, membership and strict order make each list the oracle's list.
    Compositing forward and backward on every 16th tile, with the oracle's
    own lists for those tiles (sorted by the oracle under a tile mask)."""
    scene, cam = scenes.config_scene(4), scenes.config_camera(4, 0)
    say(f"[parity heavy] n={scene.n} {cam.width}x{cam.height}")
    p, g, out, h, o = _project_stage(gs, scene, cam)
    W, H = cam.width, cam.height
    rect, counts, K = oracle.bin_rects(h["u"], h["v"], h["radius"], W, H)
    area = np.where(rect[:, 1] >= rect[:, 0], (rect[:, 1] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 2] + 1), 0)
    assert np.array_equal(h["tiles_touched"].astype(np.int64), area.astype(np.int64)), "tiles_touched"
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    assert k == K, (k, K)
    want_ranges = np.stack([np.cumsum(counts) - counts, np.cumsum(counts)], 1).astype(np.uint32)
    g_ranges = ranges.cpu().numpy().view(np.uint32)
    assert np.array_equal(g_ranges, want_ranges), "ranges"
    say(f"  bin/sort: K={k}, ranges exact; per tile min {counts.min()}, max {counts.max()}")
    g_pl = pl[:k].cpu().numpy().view(np.uint32)
    dbits = h["depth"].view(np.uint32).astype(np.uint64)
    tiles_x = (W + 15) // 16
    ntiles = len(counts)
    for t0 in range(0, ntiles, 256):
        t1 = min(ntiles, t0 + 256)
        idx = g_pl[int(want_ranges[t0, 0]):int(want_ranges[t1 - 1, 1])]
        assert (idx < scene.n).all(), ("index", t0)
        tid = np.repeat(np.arange(t0, t1, dtype=np.int64), counts[t0:t1])
        r = rect[idx]
        tx, ty = tid % tiles_x, tid // tiles_x
        inside = (r[:, 0] <= tx) & (tx <= r[:, 1]) & (r[:, 2] <= ty) & (ty <= r[:, 3])
        assert inside.all(), ("membership", t0, int((~inside).sum()))
        key = (dbits[idx] << np.uint64(32)) | idx.astype(np.uint64)
        up = (key[1:] > key[:-1]) | (tid[1:] != tid[:-1])
        assert up.all(), ("order", t0, int((~up).sum()))
    say("  bin/sort: every entry inside its Gaussian's rectangle, every list strictly ordered")
    tmask = np.zeros(ntiles, np.uint8)
    tmask[::16] = 1
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], W, H, tile_mask=tmask)
    for t in np.nonzero(tmask)[0]:
        a, b = g_ranges[t], o_ranges[t]
        assert np.array_equal(g_pl[a[0]:a[1]], o_pl[b[0]:b[1]]), ("sampled tile", t)
    del g_pl, rect
    _sampled_compositing(gs, scene, cam, p, g, out, h, o, pl, ranges, k, o_pl, o_ranges, tmask, 4001)


def _marginal(o, delta=2e-3):
    """Gaussians whose tile set may differ between FP64 and FP32 projection:
    radius or cull decision near its threshold (the oracle's flags), or a
    rectangle edge u -+ r, v -+ r within delta + 2e-6 |edge| px of a tile
    boundary (several times the FP32 error bound of u and v)."""
    u, v, r = o["rec"][:, 0], o["rec"][:, 1], o["radius"].astype(np.float64)
    near = np.zeros(len(u), bool)
    for x in (u - r, u + r, v - r, v + r):
        d = np.abs(x - 16.0 * np.round(x / 16.0))
        near |= d <= delta + 2e-6 * np.abs(x)
    return near | ((o["flags"] & 3) != 0)


def _list_flips(g_pl, g_ranges, o_pl, o_ranges, marginal, depth, tiles):
    """Tiles (of `tiles`) whose HIP list differs from the oracle's.  Every such
    difference must be one that the FP32/FP64 split allows: members that only
    one side holds are marginal Gaussians, and the HIP order of the common
    members follows the oracle's FP64 depth up to 1e-5 relative (two FP32
    depths within a few units of the last place may sort either way)."""
    diff = np.zeros(len(o_ranges), bool)
    for t in tiles:
        a = g_pl[g_ranges[t, 0]:g_ranges[t, 1]]
        b = o_pl[o_ranges[t, 0]:o_ranges[t, 1]]
        if a.shape == b.shape and np.array_equal(a, b):
            continue
        diff[t] = True
        x = np.setxor1d(a, b)
        assert marginal[x].all(), ("tile membership", t, x[~marginal[x]][:8])
        d = depth[a[np.isin(a, b)]]
        assert (d[1:] >= d[:-1] * (1 - 1e-5)).all(), ("tile order", t)
    return diff


E2E_CASES = CASES + ["main"]


@pytest.mark.parametrize("name", E2E_CASES)
def test_end_to_end_parity(gs, name):
    """Raw FP32 parameters in, on both sides: the oracle projects, bins, sorts
    and composites from the parameters alone (sort keys: its FP64 depth rounded
    to FP32), the HIP path runs its whole chain.  Tiles whose lists differ are
    validated (membership and order differences only where the two precisions
    may decide differently), then left out of the comparison; every other
    tile's pixels and the gradients meet the staged tolerances.  The main
    workload is checked on every 16th tile."""
    if name == "main":
        scene, cam = scenes.config_scene(3), scenes.config_camera(3, 0)
    else:
        scene, cam = _case(name)
    say(f"[end to end {name}] n={scene.n} {cam.width}x{cam.height}")
    W, H = cam.width, cam.height
    ntiles = ((W + 15) // 16) * ((H + 15) // 16)
    tmask = np.ones(ntiles, np.uint8)
    if name == "main":
        tmask[:] = 0
        tmask[::16] = 1
    # HIP path
    p, g, out = gpu_project(gs, scene, cam)
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    image, fT, nc, ck = gpu_render(gs, scene.n, out, pl, ranges, k, cam)
    # oracle, from the parameters only
    o = oracle.project(scene, cam)
    u, v = o["rec"][:, 0], o["rec"][:, 1]
    o_pl, o_ranges, _, _ = oracle.bin_sort(u, v, o["radius"], o["depth"].astype(np.float32), W, H,
                                           tile_mask=None if name != "main" else tmask)
    diff = _list_flips(pl[:k].cpu().numpy().view(np.uint32), ranges.cpu().numpy().view(np.uint32), o_pl, o_ranges,
                       _marginal(o), o["depth"], np.nonzero(tmask)[0])
    cmp_tiles = (tmask != 0) & ~diff
    say(f"  lists: {int(diff.sum())} of {int(tmask.sum())} tiles differ (validated, left out)")
    assert cmp_tiles.sum() >= 0.9 * tmask.sum(), "too many tiles differ"
    tx = (W + 15) // 16
    ys, xs = np.mgrid[0:H, 0:W]
    pix = cmp_tiles[(ys // 16) * tx + (xs // 16)]
    _, _, _, flips, amb, st = check_render(image, fT, nc, o["rec"][:, :9], o_pl, o_ranges, cam, margins=E2E_MARGINS,
                                           tile_mask=cmp_tiles.astype(np.uint8), pix_mask=pix, t_rtol=2e-3)
    say(f"  render fwd: max err {st['max_err']:.2e}; " + fmt_flags(st))
    G = scenes.upstream_grad(cam, 1001)
    G[:, ~pix] = 0.0
    G[:, amb] = 0.0
    o_g2c, o_g2d, o_mass = oracle_render_bwd_sigma(o["rec"][:, :9], o_pl, o_ranges, cam, G,
                                                   tile_mask=cmp_tiles.astype(np.uint8), flips=flips,
                                                   margins=E2E_MARGINS)
    # the two sides' records differ by the projection's FP32 error: on top of
    # the staged tolerance, the gradients may differ by the oracle's own
    # response to that much -- its first-order response to each record field
    # moved by its error bound, plus twice what it changes by when its own
    # records are merely rounded to FP32 (which also catches what the
    # first-order passes miss: a few sums that cancel)
    sens = record_sensitivity(o["rec"][:, :9], o_pl, o_ranges, cam, G, _record_bounds(scene, cam, o),
                              tile_mask=cmp_tiles.astype(np.uint8), flips=flips, margins=E2E_MARGINS)
    rec32 = o["rec"][:, :9].astype(np.float32).astype(np.float64)
    _, o_g2d_32, _ = oracle_render_bwd_sigma(rec32, o_pl, o_ranges, cam, G, tile_mask=cmp_tiles.astype(np.uint8),
                                             flips=flips, margins=E2E_MARGINS)
    sens = sens + 2.0 * np.abs(o_g2d_32 - o_g2d)
    g2d = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, to_dev(G))
    g2d_h = g2d.cpu().numpy().T
    worst = 0.0
    n_sens = 0
    for j, nm in enumerate("u v Sxx Sxy Syy o r g b".split()):
        ref = np.maximum(np.abs(o_g2d[:, j]), 1e-3 * np.abs(o_g2d[:, j]).max())
        staged = GRAD_RTOL * np.maximum(ref, MASS_FLOOR * o_mass[:, j])
        n_sens += int((np.abs(g2d_h[:, j] - o_g2d[:, j]) > staged).sum())
        worst = max(worst, grad_close(g2d_h[:, j], o_g2d[:, j], name=f"g2d.{nm}", mass=o_mass[:, j],
                                      extra=sens[:, j]))
    say(f"  record gradients: {n_sens} entries needed the record-error allowance")
    o_g2d_tol = np.abs(o_g2d) + sens / GRAD_RTOL
    grads = {kk: torch.empty_like(vv) for kk, vv in p.items()}
    gs.project_bwd(g, gs.camera_struct(cam), g2d, grads)
    torch.cuda.synchronize()
    o_gr = oracle.project_bwd(scene, cam, o_g2c)
    # the parameter gradients carry the record gradients' tolerance through the
    # projection's Jacobian J: bound sum_j |J e_j| tol_j, from one oracle pass
    # per record channel j (each Gaussian's gradient depends on its own row only)
    # (the projection's own rounding is judged against the chain's term mass)
    tol = np.maximum(np.maximum(o_g2d_tol, 1e-3 * np.abs(o_g2d).max(axis=0)), MASS_FLOOR * o_mass)
    carried, cm = chain_mass(scene, cam, tol, np.abs(o_g2d))
    sel = (o["flags"] & 0b1110) == 0
    for kk in ("means", "log_scales", "quats", "logits", "sh"):
        mass = np.maximum(carried[kk] / MASS_FLOOR, cm[kk])[..., sel]
        worst = max(worst, grad_close(grads[kk].cpu().numpy()[..., sel], o_gr[kk][..., sel], name=kk, mass=mass))
    say(f"  render bwd + project bwd: worst rel err {worst:.2e}")


@pytest.mark.parametrize("name", ["ragged", "skewed", "main"])
def test_deterministic_backward(gs, name):
    """deterministic = 1: every (tile, Gaussian) entry's partial is written once
    and each Gaussian's partials are added in a fixed order (no atomics).  Two
    runs give the same bits under every work split, and the gradients meet the
    staged tolerance (the main workload on every 16th tile)."""
    if name == "main":
        scene, cam = scenes.config_scene(3), scenes.config_camera(3, 0)
    else:
        scene, cam = _case(name)
    say(f"[deterministic {name}] n={scene.n} {cam.width}x{cam.height}")
    p, g, out = gpu_project(gs, scene, cam)
    h = proj_host(out)
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    W, H = cam.width, cam.height
    tiles_x = (W + 15) // 16
    tmask = np.ones(tiles_x * ((H + 15) // 16), np.uint8)
    if name == "main":
        tmask[:] = 0
        tmask[::16] = 1
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], W, H, tile_mask=tmask)
    image, fT, nc, ck = gpu_render(gs, scene.n, out, pl, ranges, k, cam)
    ys, xs = np.mgrid[0:H, 0:W]
    pix = tmask[(ys // 16) * tiles_x + (xs // 16)].astype(bool)
    _, _, _, flips, amb, _ = check_render(image, fT, nc, h["rec"][:, :9], o_pl, o_ranges, cam, tile_mask=tmask,
                                          pix_mask=pix)
    G = scenes.upstream_grad(cam, 1001)
    G[:, ~pix] = 0.0
    G[:, amb] = 0.0
    _, o_g2d, o_mass = oracle_render_bwd_sigma(h["rec"][:, :9], o_pl, o_ranges, cam, G, tile_mask=tmask, flips=flips)
    Gd = to_dev(G)
    for sched in (gs.SCHEDULE_PLAIN, gs.SCHEDULE_BALANCED, gs.SCHEDULE_MERGED):
        a = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, Gd, deterministic=True, schedule=sched)
        b = gpu_render_bwd(gs, scene.n, out, pl, ranges, k, cam, fT, nc, ck, Gd, deterministic=True, schedule=sched)
        assert torch.equal(a, b), f"schedule {sched}: two deterministic runs differ"
        ah = a.cpu().numpy().T
        worst = 0.0
        for j, nm in enumerate("u v Sxx Sxy Syy o r g b".split()):
            worst = max(worst, grad_close(ah[:, j], o_g2d[:, j], name=f"schedule {sched} g2d.{nm}",
                                          mass=o_mass[:, j]))
        say(f"  schedule {sched}: bit-identical reruns, worst rel err {worst:.2e}")


@pytest.mark.parametrize("width", [2400, 4800])
def test_bin_sort_wide_frame_fallback(gs, width):
    """Wide frames: 150 x 63 tiles (9,450: the direct emission, 19 x 8 super
    tiles with ragged edges) and 300 x 63 (18,900 tiles, more than the direct
    emission's 16,384: the two-pass radix tile sort, which the no-wait call
    refuses).  Both must give the oracle's lists bit for bit."""
    scene = scenes.skewed_scene(30000, 91, n_clusters=16, log_scale_mean=-3.6, sh_degree=1)
    cam = scenes.pinhole(width, 1000, 70.0, np.eye(3), (0.0, 0.0, 3.0))
    say(f"[bin/sort wide] n={scene.n} {cam.width}x{cam.height}")
    direct = gs.n_tiles(gs.camera_struct(cam)) <= 16384
    assert direct == (width == 2400)
    p, g, out = gpu_project(gs, scene, cam)
    h = proj_host(out)
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], cam.width, cam.height)
    assert k == len(o_pl) and k > 0
    assert np.array_equal(pl[:k].cpu().numpy().view(np.uint32), o_pl), "point_list"
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), o_ranges), "ranges"
    say(f"  K={k} bit-exact")


def _slab_scene(n_small=20000, n_big=700, seed=93):
    """Small Gaussians everywhere plus large ones in a thin depth slab: rank
    groups inside the slab touch thousands of tiles, the others a few hundred."""
    a = scenes.uniform_scene(n_small, seed, log_scale_mean=-4.5, log_scale_std=0.3, sh_degree=1)
    b = scenes.uniform_scene(n_big, seed + 1, log_scale_mean=-1.8, log_scale_std=0.2, sh_degree=1)
    means = b.means.copy()
    means[2] = np.float32(0.5) + np.float32(0.05) * (means[2] + 1) / 2
    cat = lambda x, y: np.concatenate([x, y], axis=-1)
    return scenes.Scene(n_small + n_big, 1, cat(a.means, means), cat(a.log_scales, b.log_scales),
                        cat(a.quats, b.quats), cat(a.logits, b.logits), cat(a.sh, b.sh))


def test_bin_sort_many_tiles_per_group(gs):
    """Direct emission where some groups of 256 consecutive depth ranks cover
    thousands of tiles (their rank-waves hold very different entry counts) and
    the others a few hundred: the lists must still be the oracle's bit for bit."""
    scene = _slab_scene()
    cam = scenes.front_camera(1600, 1064, 3.0, 60.0)
    say(f"[bin/sort many tiles] n={scene.n} {cam.width}x{cam.height}")
    p, g, out = gpu_project(gs, scene, cam)
    h = proj_host(out)
    rect, _, _ = oracle.bin_rects(h["u"], h["v"], h["radius"], cam.width, cam.height)
    order = np.lexsort((np.arange(scene.n), h["depth"].astype(np.float32).view(np.uint32)))
    tx = cam.tiles_x
    wide = []
    for g0 in range(0, scene.n, 256):
        tiles = set()
        for k in order[g0:g0 + 256]:
            x0, x1, y0, y1 = rect[k]
            for y in range(y0, y1 + 1):
                tiles.update(range(y * tx + x0, y * tx + x1 + 1))
        wide.append(len(tiles) > 2048)
    assert any(wide) and not all(wide), "the scene must mix wide and narrow rank groups"
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], cam.width, cam.height)
    assert k == len(o_pl) and k > 0
    assert np.array_equal(pl[:k].cpu().numpy().view(np.uint32), o_pl), "point_list"
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), o_ranges), "ranges"
    say(f"  K={k}, {sum(wide)} of {len(wide)} aligned rank groups wide, bit-exact")


def _depth_case_scene(kind, n=20000, seed=95):
    """Scenes whose depth keys exercise the depth sort's digit structure
    (camera at distance 3 on the z axis: depth = z + 3)."""
    sc = scenes.uniform_scene(n, seed, log_scale_mean=-4.0, log_scale_std=0.3, sh_degree=1)
    means = sc.means.copy()
    if kind == "quantised":    # depths 2, 2.5, 3, 3.5: bytes 0-1 and 3 shared
        means[2] = np.float32(-1.0) + np.float32(0.5) * (np.arange(n) % 4).astype(np.float32)
    elif kind == "equal":      # one depth: every digit shared
        means[2] = np.float32(0.0)
    return dataclasses.replace(sc, means=means)


@pytest.mark.parametrize("kind", ["straddle", "quantised", "equal"])
def test_bin_sort_depth_digit_cases(gs, kind):
    """The depth sort skips passes whose digit every key shares and finishes
    in the last pass that reorders: top byte varying (straddle: depths across
    2.0, all four passes), only byte 2 varying (quantised: two copies, then the
    last reordering pass), no byte varying (equal: one copy).  The lists must
    be the oracle's bit for bit."""
    scene = _depth_case_scene(kind)
    cam = scenes.front_camera(800, 800, 2.5 if kind == "straddle" else 3.0, 60.0)
    say(f"[bin/sort depth digits] {kind} n={scene.n}")
    p, g, out = gpu_project(gs, scene, cam)
    h = proj_host(out)
    live = h["radius"] > 0
    bits = h["depth"].astype(np.float32).view(np.uint32)[live]
    varying = [len(np.unique((bits >> (8 * q)) & 255)) > 1 for q in range(4)]
    expect = {"straddle": varying[3], "quantised": varying == [False, False, True, False],
              "equal": not any(varying)}[kind]
    assert expect, (kind, varying)
    k, pl, ranges = gpu_bin_sort(gs, scene.n, out, cam)
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], cam.width, cam.height)
    assert k == len(o_pl) and k > 0
    assert np.array_equal(pl[:k].cpu().numpy().view(np.uint32), o_pl), "point_list"
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), o_ranges), "ranges"
    say(f"  K={k}, varying digits {varying}, bit-exact")


def test_bin_sort_async_matches_sync(gs):
    """Frames binned without the host wait (gs_bin_sort_async, K checked one
    frame later) give the same images and, with the deterministic reduction,
    the same gradients bit for bit as the waiting call; a frame whose lists do
    not fit is reported at the check with the size it needed."""
    from paper_2510_14564_amd.raster import Rasterizer
    scene = scenes.config_scene(2)
    cams = [scenes.orbit_camera(k, 32, 800, 800) for k in (0, 3, 9, 17)]
    p = upload(scene)
    G = to_dev(scenes.upstream_grad(cams[0], 2001))
    args = (p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"])
    outs = {}
    for mode in (False, True):
        rast = Rasterizer(cams[0], 3, device=DEV, deterministic=True, async_k=mode, capacity=8_000_000)
        frames = []
        for cam in cams:
            rast.set_camera(cam)
            st = rast.forward(*args)
            g = rast.backward(st, *args, G)
            frames.append((st.image.clone(), st.n_contrib.clone(), {kk: v.clone() for kk, v in g.items()}))
        assert rast.check_async() is not None
        outs[mode] = frames
    for (i0, n0, g0), (i1, n1, g1) in zip(outs[False], outs[True]):
        assert torch.equal(i0, i1) and torch.equal(n0, n1)
        for kk in g0:
            assert torch.equal(g0[kk], g1[kk]), kk
    say("  async bin/sort: 4 frames bit-identical to the waiting call")
    rast = Rasterizer(cams[0], 3, device=DEV, async_k=True)
    rast.forward(*args)                    # first frame waits and learns K
    k0 = rast.last_k
    rast._alloc_lists(k0 // 2)             # the next frame's lists cannot fit
    rast.forward(*args)
    with pytest.raises(gs.GsError) as ei:
        rast.check_async()
    assert ei.value.status == gs.GS_ERR_CAPACITY and ei.value.required == k0
    rast.forward(*args)                    # capacity grown by the check
    assert rast.check_async() == k0

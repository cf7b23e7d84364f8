"""The training step through the autograd Function (needs the GPU).

raster.rasterize / rasterize_learned -> the library's L1 loss -> .backward():
every parameter's .grad is compared with the FP64 oracle, and at the tiny
workload with central finite differences of the GPU step itself.

Oracle side (staged, as the parity tests): the oracle bins and composites the
HIP path's own FP32 records (a second gs_project of the same parameters gives
the same bits), resolves every near-threshold decision to the branch the HIP
image took, back-propagates the same upstream gradient and applies the
projection's chain rule to the record gradients.  Parameter gradients are
judged with the record gradients' tolerance carried through the projection's
Jacobian (plus the chain rule's own term mass); the entries that need more
than the plain 1e-3 relative bound are counted and printed.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import brute
from paper_2510_14564_amd import scenes
from gpu_helpers import (DEV, MASS_FLOOR, chain_mass, check_render, fmt_flags, grad_close, oracle_render_bwd_sigma,
                         proj_host, say, sigma_to_conic_grad, to_dev)
from mlp_bounds import U, bwd_bounds, kaiming_params

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "quats", "logits", "sh")


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_14564_amd import gs as mod
    return mod


def _leaf(scene):
    return {k: to_dev(v).requires_grad_(True) for k, v in scene.arrays().items() if k in PARAMS}


def _gpu_records(gs, g, n, cam):
    """The HIP projection of the same parameters (deterministic: the same bits
    the rasterizer's forward used)."""
    out = gs.ProjectedBuffers(n, DEV)
    gs.project(g, gs.camera_struct(cam), out)
    torch.cuda.synchronize()
    return proj_host(out)


def _lists(st):
    """A frame's sorted lists and ranges (host copies) from a waiting bin/sort."""
    return st.point_list[:st.k].cpu().numpy().tobytes() + st.ranges.cpu().numpy().tobytes()


def _carried_check(scene, cam, grads, o_g2s, o_mass, names, label):
    """Parameter gradients against the oracle's chain rule applied to its own
    record gradients, with the record tolerance carried through the
    projection's Jacobian.  Returns the count of entries beyond the plain
    1e-3 relative bound."""
    o = oracle.project(scene, cam)
    o_gr = oracle.project_bwd(scene, cam, sigma_to_conic_grad(o["rec"], o_g2s))
    tol = np.maximum(np.maximum(np.abs(o_g2s), 1e-3 * np.abs(o_g2s).max(axis=0)), MASS_FLOOR * o_mass)
    carried, cm = chain_mass(scene, cam, tol, np.abs(o_g2s))
    sel = (o["flags"] & 0b1110) == 0
    beyond = {}
    worst = 0.0
    for kk in names:
        mass = np.maximum(carried[kk] / MASS_FLOOR, cm[kk])[..., sel]
        worst = max(worst, grad_close(grads[kk][..., sel], o_gr[kk][..., sel], name=f"{label} {kk}", mass=mass,
                                      stats=beyond))
    total = sum(int(np.prod(grads[kk][..., sel].shape)) for kk in names)
    say(f"  {label}: worst plain rel err {worst:.2e}; beyond plain 1e-3: {sum(beyond.values())} of {total} "
        f"({', '.join(f'{k} {v}' for k, v in beyond.items())})")
    return o_gr, sel


@pytest.mark.parametrize("name", ["skewed", "main"])
def test_autograd_sh_step_matches_oracle(gs, name):
    """rasterize() + L1 + backward at the skewed workload (200k Gaussians,
    800x800) in full and at the main workload (1M, 1600x1064, orbit camera 0)
    with the upstream gradient kept on every 16th tile."""
    from paper_2510_14564_amd.raster import Rasterizer, l1_loss, rasterize
    cfg = 2 if name == "skewed" else 3
    scene, cam = scenes.config_scene(cfg), scenes.config_camera(cfg, 0)
    say(f"[autograd SH {name}] n={scene.n} {cam.width}x{cam.height}")
    p = _leaf(scene)
    rast = Rasterizer(cam, scene.sh_degree, device=DEV)
    img = rasterize(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], rast)
    _, dimg = l1_loss(img.detach(), to_dev(scenes.target_image(cam, 3000 + cfg)))
    torch.cuda.synchronize()
    g = gs.gaussians_struct(p["means"].detach(), p["log_scales"].detach(), p["quats"].detach(),
                            p["logits"].detach(), p["sh"].detach(), scene.sh_degree)
    h = _gpu_records(gs, g, scene.n, cam)
    W, H = cam.width, cam.height
    ntiles = cam.tiles_x * cam.tiles_y
    tmask = None
    pix = np.ones((H, W), bool)
    if name == "main":
        tmask = np.zeros(ntiles, np.uint8)
        tmask[::16] = 1
        ys, xs = np.mgrid[0:H, 0:W]
        pix = tmask[(ys // 16) * cam.tiles_x + (xs // 16)].astype(bool)
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], W, H, tile_mask=tmask)
    _, _, _, flips, amb, st = check_render(img.detach(), rast.last_frame.final_T, rast.last_frame.n_contrib,
                                           h["rec"][:, :9], o_pl, o_ranges, cam, tile_mask=tmask, pix_mask=pix)
    say(f"  image: max err {st['max_err']:.2e}; " + fmt_flags(st))
    G = dimg.cpu().numpy().astype(np.float32)
    G[:, ~pix] = 0.0
    G[:, amb] = 0.0
    img.backward(to_dev(G))
    torch.cuda.synchronize()
    grads = {k: p[k].grad.cpu().numpy().astype(np.float64) for k in PARAMS}
    _, o_g2s, o_mass = oracle_render_bwd_sigma(h["rec"][:, :9], o_pl, o_ranges, cam, G.astype(np.float64),
                                               tile_mask=tmask, flips=flips)
    _carried_check(scene, cam, grads, o_g2s, o_mass, PARAMS, "autograd SH")


def test_autograd_learned_step_matches_oracle(gs):
    """rasterize_learned() + L1 + backward on the learned-colour scene (200k
    Gaussians, 800x800, random BF16 decoder): geometry gradients against the
    oracle's chain rule, decoder weight and latent gradients against torch
    autograd in FP64 of the decoder within the BF16 rounding bounds, and the
    means with the view direction's share added."""
    from paper_2510_14564_amd.decoder import Decoder
    from paper_2510_14564_amd.raster import Rasterizer, l1_loss, rasterize_learned
    scene, cam = scenes.config_scene(5), scenes.config_camera(5)
    n = scene.n
    say(f"[autograd learned] n={n} {cam.width}x{cam.height}")
    Pbits = kaiming_params(12)
    dec = Decoder(n, device=DEV, latents_bits=scene.latents, params_bits=Pbits)
    dec.latents.requires_grad_(True)
    dec.params.requires_grad_(True)
    p = {k: to_dev(v).requires_grad_(True) for k, v in scene.arrays().items() if k in PARAMS[:4]}
    rast = Rasterizer(cam, 0, device=DEV)
    img = rasterize_learned(p["means"], p["log_scales"], p["quats"], p["logits"], dec, rast)
    _, dimg = l1_loss(img.detach(), to_dev(scenes.target_image(cam, 3005)))
    g = gs.gaussians_struct_mlp(p["means"].detach(), p["log_scales"].detach(), p["quats"].detach(),
                                p["logits"].detach(), dec.latents_bf16, dec.packed)
    h = _gpu_records(gs, g, n, cam)
    o_pl, o_ranges, _, _ = oracle.bin_sort(h["u"], h["v"], h["radius"], h["depth"], cam.width, cam.height)
    _, _, _, flips, amb, st = check_render(img.detach(), rast.last_frame.final_T, rast.last_frame.n_contrib,
                                           h["rec"][:, :9], o_pl, o_ranges, cam)
    say(f"  image: max err {st['max_err']:.2e}; " + fmt_flags(st))
    G = dimg.cpu().numpy().astype(np.float32)
    G[:, amb] = 0.0
    img.backward(to_dev(G))
    torch.cuda.synchronize()
    _, o_g2s, o_mass = oracle_render_bwd_sigma(h["rec"][:, :9], o_pl, o_ranges, cam, G.astype(np.float64),
                                               flips=flips)
    # geometry: the oracle's chain rule on a degree-0 copy with zero SH (no
    # direction term), judged like the SH step
    s0 = scenes.Scene(n, 0, scene.means, scene.log_scales, scene.quats, scene.logits,
                      np.zeros((1, 3, n), np.float32))
    grads = {k: p[k].grad.cpu().numpy().astype(np.float64) for k in PARAMS[:4]}
    geo_names = ("log_scales", "quats", "logits")
    o_geo, sel = _carried_check(s0, cam, grads, o_g2s, o_mass, geo_names, "autograd learned geometry")
    # decoder: torch autograd in FP64 of the decoder at the live Gaussians, with
    # the oracle's colour gradients (record channels 6..8) as the upstream
    live = h["radius"] > 0
    idx = np.nonzero(live)[0]
    ca = oracle.cam_array(cam)
    centre = -(ca[7:16].reshape(3, 3).T @ ca[16:19])
    mt = torch.tensor(scene.means[:, idx].astype(np.float64), requires_grad=True)
    zt = torch.tensor(scenes.bf16_to_f32(scene.latents[idx]).astype(np.float64), requires_grad=True)
    P = scenes.bf16_to_f32(Pbits).astype(np.float64)
    Pt = torch.tensor(P, requires_grad=True)
    Gc = o_g2s[idx, 6:9]
    (brute.learned_colour(mt, centre, zt, Pt) * torch.tensor(Gc)).sum().backward()
    dirs = scene.means[:, idx].astype(np.float64).T - centre
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x = oracle.mlp_inputs(zt.detach().numpy(), dirs[:, None, :])
    ex = np.concatenate([np.zeros((len(idx), 16)), (U + 1e-5) * np.abs(x[:, 16:]) + 1e-6], axis=1)
    # the HIP colour gradients differ from the oracle's within the record tolerance
    eG = 1e-3 * np.maximum(np.maximum(np.abs(Gc), 1e-3 * np.abs(o_g2s[:, 6:9]).max(axis=0)),
                           MASS_FLOOR * o_mass[idx, 6:9])
    bP, bdx, _ = bwd_bounds(x, P, Gc, eG=eG, ex=ex)
    got_P = dec.params.grad.cpu().numpy().astype(np.float64)
    got_z = dec.latents.grad.cpu().numpy().astype(np.float64)
    errP = np.abs(got_P - Pt.grad.numpy())
    errz = np.abs(got_z[idx] - zt.grad.numpy())
    assert (errP <= bP).all(), f"decoder weights: worst err/bound {(errP / bP).max():.2f}"
    assert (errz <= bdx[:, :16]).all(), f"latents: worst err/bound {(errz / bdx[:, :16]).max():.2f}"
    assert (got_z[~live] == 0).all()
    say(f"  decoder: max err/bound weights {(errP / bP).max():.3f}, latents {(errz / bdx[:, :16]).max():.3f}")
    # means: geometry (carried tolerance of the SH step, 1e-3 relative) plus the
    # direction's share, whose error is at most |grad Y_j| <= 10 on the unit
    # sphere times the dL/dY bound, over |v|
    share = mt.grad.numpy()
    want_m = o_geo["means"].copy()
    want_m[:, idx] += share
    ref = np.maximum(np.abs(o_geo["means"]), 1e-3 * np.abs(o_geo["means"]).max())
    tol = np.maximum(np.abs(o_g2s), 1e-3 * np.abs(o_g2s).max(axis=0))
    tol = np.maximum(tol, MASS_FLOOR * o_mass)
    carried, cm = chain_mass(s0, cam, tol, np.abs(o_g2s))
    bound = 1e-3 * np.maximum(ref, np.maximum(carried["means"], MASS_FLOOR * cm["means"]))
    vlen = np.linalg.norm(scene.means[:, idx].astype(np.float64).T - centre, axis=1)
    bound[:, idx] += 1e-5 * np.abs(share) + (10 * bdx[:, 16:].sum(1) / vlen)[None, :]
    err = np.abs(grads["means"] - want_m)
    assert (err[:, sel] <= bound[:, sel]).all(), (err[:, sel] / bound[:, sel]).max()
    say(f"  means: max err/bound {(err[:, sel] / bound[:, sel]).max():.3f}")


def test_autograd_matches_finite_differences(gs):
    """Central differences of the GPU step itself at the tiny workload (4,096
    Gaussians, 128x128): L = sum(G * image) with G the L1 gradient at the
    start point, for the Gaussians with the largest gradients.  A point is
    used only if no decision moves within the step: the perturbed renders keep
    every list, every pixel's n_contrib (the stop) and the number of blended
    pairs (a skip flip at alpha = 1/255 changes it by one; it moves one
    pixel by about c/255, which is a sizeable part of L's change over a step
    of 2e-4 in a mean), and the two one-sided differences agree within 5 %.
    The FP32 difference quotient is then accurate to about 1e-4 and must
    agree with the autograd gradient to 1e-2."""
    from paper_2510_14564_amd.raster import Rasterizer, l1_loss, rasterize
    scene, cam = scenes.config_scene(1), scenes.config_camera(1, bg=(0.2, 0.5, 0.8))
    say(f"[autograd FD] n={scene.n}")
    p = _leaf(scene)
    rast = Rasterizer(cam, scene.sh_degree, device=DEV, deterministic=True)
    img = rasterize(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], rast)
    _, dimg = l1_loss(img.detach(), to_dev(scenes.target_image(cam, 3001)))
    G = dimg.clone()
    img.backward(G)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy().astype(np.float64)
    base = img.detach().cpu().numpy().astype(np.float64)
    L0 = float((Gh * base).sum())
    nc0 = rast.last_frame.n_contrib.cpu().numpy()
    pl0 = _lists(rast.last_frame)
    counts = torch.zeros(2, dtype=torch.int64, device=DEV)

    def blended(st):
        gs.render_count(st.n, st.proj, st.point_list, st.ranges, st.k, st.cs, counts)
        return int(counts[1].item())

    bl0 = blended(rast.last_frame)

    def loss_at(key, idx, value):
        q = {k: v.detach().clone() for k, v in p.items()}
        q[key][idx] = value
        with torch.no_grad():
            st = rast.forward(q["means"], q["log_scales"], q["quats"], q["logits"], q["sh"])
            torch.cuda.synchronize()
            im = st.image.cpu().numpy().astype(np.float64)
            same = (np.array_equal(st.n_contrib.cpu().numpy(), nc0) and _lists(st) == pl0 and
                    blended(st) == bl0)
        return float((Gh * im).sum()), same

    steps = {"means": 2e-4, "log_scales": 2e-3, "quats": 2e-3, "logits": 2e-3, "sh": 2e-3}
    checked = 0
    for key in PARAMS:
        grad = p[key].grad.cpu().numpy()
        flat = np.argsort(-np.abs(grad).reshape(-1))[:12]
        for fi in flat:
            idx = np.unravel_index(fi, grad.shape)
            x0 = float(p[key].detach()[idx].item())
            h = steps[key] * max(1.0, abs(x0))
            xp, xm = np.float32(x0 + h), np.float32(x0 - h)
            Lp, okp = loss_at(key, idx, float(xp))
            Lm, okm = loss_at(key, idx, float(xm))
            if not (okp and okm):
                continue
            dp, dm = (Lp - L0) / (float(xp) - x0), (L0 - Lm) / (x0 - float(xm))
            if abs(dp - dm) > 5e-2 * max(abs(dp), abs(dm)):
                continue
            fd = (Lp - Lm) / (float(xp) - float(xm))
            an = float(grad[idx])
            assert abs(fd - an) <= 1e-2 * abs(an) + 1e-9, (key, idx, fd, an)
            checked += 1
    say(f"  {checked} finite-difference points agree within 1e-2")
    assert checked >= 25


def test_two_views_one_backward(gs):
    """Two views rendered before one backward of the summed loss give the sum
    of the views' gradients (each frame keeps its own buffers and camera); the
    deterministic reduction makes the comparison exact."""
    from paper_2510_14564_amd.raster import Rasterizer, l1_loss, rasterize
    scene = scenes.config_scene(2, n=50000)
    cams = [scenes.orbit_camera(k, 32, 400, 300) for k in (0, 5)]
    say("[autograd two views]")
    p = _leaf(scene)
    rast = Rasterizer(cams[0], scene.sh_degree, device=DEV, deterministic=True)
    targets = [to_dev(scenes.target_image(c, 77 + i)) for i, c in enumerate(cams)]
    single = []
    for cam, tgt in zip(cams, targets):
        rast.set_camera(cam)
        img = rasterize(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], rast)
        _, dimg = l1_loss(img.detach(), tgt)
        img.backward(dimg)
        single.append({k: p[k].grad.clone() for k in PARAMS})
        for k in PARAMS:
            p[k].grad = None
    imgs, grads_in = [], []
    for cam, tgt in zip(cams, targets):
        rast.set_camera(cam)
        img = rasterize(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], rast)
        _, dimg = l1_loss(img.detach(), tgt)
        imgs.append(img)
        grads_in.append(dimg)
    torch.autograd.backward(imgs, grads_in)
    torch.cuda.synchronize()
    for k in PARAMS:
        want = single[0][k] + single[1][k]
        assert torch.equal(p[k].grad, want), k
    assert any(single[1][k].abs().sum() > 0 for k in PARAMS)
    say("  summed two-view gradients equal the per-view sums bit for bit")

"""Parity of the learned colour decoder's matrix-core kernels with the FP64 oracle.

Both sides use the same BF16 latents and weights (widened exactly to FP64 in
the oracle).  In the forward the HIP path carries the SH encoding of the
direction and both hidden activations as hi + lo BF16 pairs (relative error
at most 2^-17, bounded here by UA = 2^-16) and accumulates in FP32; the
backward does the same for the gradients entering each product and for both
operands of the weight-gradient products (whose dropped lo x lo term is
below 2^-17 relative).  The tolerance
is the running error bound of exactly those roundings, propagated through |W|
in FP64 (ReLU is 1-Lipschitz, the sigmoid 1/4).  The observed maximum error
is printed.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import DEV, say, sigma_to_conic_grad, to_dev
from mlp_bounds import F32, U, UA, _check_grads, bwd_bounds, error_bound, fwd_bounds, kaiming_params, reading18  # noqa: F401

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_14564_amd import gs as mod
    return mod


def _dirs(n, per, seed):
    d = np.random.default_rng(seed).normal(size=(n, per, 3))
    return (d / np.linalg.norm(d, axis=2, keepdims=True)).astype(np.float32)


def _packed(gs, Pbits):
    packed = torch.empty(gs.MLP_PACKED_BYTES // 4 + 4, dtype=torch.float32, device=DEV)
    gs.mlp_pack(to_dev(Pbits.view(np.int16)), packed)
    return packed


# (16384, 64): a distillation minibatch, 1,048,576 samples, as the distiller runs it
@pytest.mark.parametrize("n,per", [(1, 1), (37, 3), (4096, 4), (20000, 1), (16384, 64)])
def test_mlp_forward_matches_oracle_within_bf16_bound(gs, n, per):
    say(f"[mlp fwd] n={n} per={per}")
    Pbits = kaiming_params(10 + n)
    z = scenes.bf16_bits(np.random.default_rng(n).normal(0, 0.5, (n, 16)).astype(np.float32))
    d = _dirs(n, per, 20 + n)
    packed = _packed(gs, Pbits)
    S = n * per
    rgb = torch.empty((S, 3), dtype=torch.float32, device=DEV)
    gs.mlp_fwd(S, per, to_dev(z.view(np.int16)), to_dev(d.reshape(S, 3)), packed, rgb)
    torch.cuda.synchronize()
    P = scenes.bf16_to_f32(Pbits).astype(np.float64)
    x = oracle.mlp_inputs(scenes.bf16_to_f32(z).astype(np.float64), d.astype(np.float64))
    want = oracle.mlp_fwd(x, P)
    got = rgb.cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    bound = error_bound(x, P)
    assert (err <= bound).all(), f"max err {err.max():.3e}, worst ratio {(err / bound).max():.2f}"
    assert err.max() <= 1e-3
    say(f"  max |err| {err.max():.2e}, max err/bound {(err / bound).max():.3f}")


def test_mlp_zero_weights_give_sigmoid_bias(gs):
    P = np.zeros(oracle.MLP_PARAMS, np.float32)
    P[oracle.MLP_SLICES["b3"][0]:] = [-1.0, 0.25, 2.0]
    Pbits = scenes.bf16_bits(P)
    n = 100
    z = scenes.bf16_bits(np.random.default_rng(1).normal(size=(n, 16)).astype(np.float32))
    d = _dirs(n, 1, 2)
    rgb = torch.empty((n, 3), dtype=torch.float32, device=DEV)
    gs.mlp_fwd(n, 1, to_dev(z.view(np.int16)), to_dev(d.reshape(n, 3)), _packed(gs, Pbits), rgb)
    want = 1.0 / (1.0 + np.exp(-scenes.bf16_to_f32(Pbits)[-3:].astype(np.float64)))
    assert np.abs(rgb.cpu().numpy() - want).max() < 1e-6


@pytest.mark.parametrize("n", [20000, 200000])
def test_project_with_learned_colour(gs, n):
    """colour_mode 1: geometry identical to the SH projection, colour = decoder of
    (latent, SH encoding of the camera-to-Gaussian direction) for live Gaussians;
    200,000 is the learned-colour workload in full."""
    scene = scenes.config_scene(5, n=n)
    cam = scenes.config_camera(5)
    say(f"[project learned colour] n={scene.n}")
    Pbits = kaiming_params(5)
    packed = _packed(gs, Pbits)
    p = {k: to_dev(v) for k, v in scene.arrays().items()}
    lat = to_dev(scene.latents.view(np.int16))
    g = gs.gaussians_struct_mlp(p["means"], p["log_scales"], p["quats"], p["logits"], lat, packed)
    out = gs.ProjectedBuffers(scene.n, DEV)
    gs.project(g, gs.camera_struct(cam), out)
    g_sh = gs.gaussians_struct(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], scene.sh_degree)
    out_sh = gs.ProjectedBuffers(scene.n, DEV)
    gs.project(g_sh, gs.camera_struct(cam), out_sh)
    torch.cuda.synchronize()
    rec, rec_sh = out.records.cpu().numpy(), out_sh.records.cpu().numpy()
    live = out.radius.cpu().numpy() > 0
    assert np.array_equal(live, out_sh.radius.cpu().numpy() > 0)
    geo = [0, 1, 2, 3, 4, 5, 9]
    assert np.array_equal(rec[:, geo], rec_sh[:, geo])
    assert (rec[~live] == 0).all()
    # oracle colour at the FP64 view direction of each live Gaussian
    ca = oracle.cam_array(cam)
    centre = -(ca[7:16].reshape(3, 3).T @ ca[16:19])
    dirs = scene.means.astype(np.float64).T - centre
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x = oracle.mlp_inputs(scenes.bf16_to_f32(scene.latents).astype(np.float64), dirs[:, None, :])
    P = scenes.bf16_to_f32(Pbits).astype(np.float64)
    want = oracle.mlp_fwd(x, P)
    err = np.abs(rec[live, 6:9] - want[live])
    bound = error_bound(x, P)[live] + 1e-5     # + the FP32 view direction
    assert (err <= bound).all(), (err.max(), (err / bound).max())
    say(f"  live {live.sum()}, max colour err {err.max():.2e}")


def _bwd_workspace(gs, S, per):
    return torch.empty(gs.mlp_bwd_workspace(S, per), dtype=torch.uint8, device=DEV)


@pytest.mark.parametrize("n,per", [(1, 1), (37, 4), (300, 64), (5000, 1), (2000, 16), (16384, 64)])
def test_mlp_backward_matches_oracle_within_bound(gs, n, per):
    say(f"[mlp bwd] n={n} per={per}")
    Pbits = kaiming_params(30 + n)
    z = scenes.bf16_bits(np.random.default_rng(n + 1).normal(0, 0.5, (n, 16)).astype(np.float32))
    d = _dirs(n, per, 40 + n)
    S = n * per
    G = np.random.default_rng(n + 2).normal(size=(S, 3)).astype(np.float32)
    packed = _packed(gs, Pbits)
    dlat = torch.empty((n, 16), dtype=torch.float32, device=DEV)
    dP = torch.empty(oracle.MLP_PARAMS, dtype=torch.float32, device=DEV)
    ws = _bwd_workspace(gs, S, per)
    zd, dd, Gd = to_dev(z.view(np.int16)), to_dev(d.reshape(S, 3)), to_dev(G)
    gs.mlp_bwd(S, per, zd, dd, packed, dlat, dP, ws, dL_drgb=Gd)
    torch.cuda.synchronize()
    got_P, got_z = dP.cpu().numpy().astype(np.float64), dlat.cpu().numpy().astype(np.float64)
    # bit-reproducible: a second call gives the same bits
    gs.mlp_bwd(S, per, zd, dd, packed, dlat, dP, ws, dL_drgb=Gd)
    torch.cuda.synchronize()
    assert np.array_equal(dP.cpu().numpy(), got_P.astype(np.float32))
    assert np.array_equal(dlat.cpu().numpy(), got_z.astype(np.float32))
    P = scenes.bf16_to_f32(Pbits).astype(np.float64)
    x = oracle.mlp_inputs(scenes.bf16_to_f32(z).astype(np.float64), d.astype(np.float64))
    want_P, dx = oracle.mlp_bwd(x, P, G.astype(np.float64))
    bP, bdx, massP = bwd_bounds(x, P, G.astype(np.float64))
    want_z = dx[:, :16].reshape(n, per, 16).sum(1)
    bz = bdx[:, :16].reshape(n, per, 16).sum(1) + per * F32 * np.abs(dx[:, :16]).reshape(n, per, 16).sum(1)
    _check_grads(f"n={n} per={per}", got_P, want_P, bP, got_z, want_z, bz, massP)


def test_mlp_distillation_loss_and_gradient(gs):
    """Loss mode: L = scale * sum |c - target|^2 with the gradient taken from
    the kernel's own colours."""
    n, per = 256, 64
    S = n * per
    say(f"[mlp distill loss] S={S}")
    Pbits = kaiming_params(77)
    z = scenes.bf16_bits(np.random.default_rng(78).normal(0, 0.5, (n, 16)).astype(np.float32))
    d = _dirs(n, per, 79)
    tgt = np.random.default_rng(80).uniform(0, 1, (S, 3)).astype(np.float32)
    scale = 1.0 / S
    packed = _packed(gs, Pbits)
    dlat = torch.empty((n, 16), dtype=torch.float32, device=DEV)
    dP = torch.empty(oracle.MLP_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    gs.mlp_bwd(S, per, to_dev(z.view(np.int16)), to_dev(d.reshape(S, 3)), packed, dlat, dP,
               _bwd_workspace(gs, S, per), target=to_dev(tgt), scale=scale, loss=loss)
    torch.cuda.synchronize()
    P = scenes.bf16_to_f32(Pbits).astype(np.float64)
    x = oracle.mlp_inputs(scenes.bf16_to_f32(z).astype(np.float64), d.astype(np.float64))
    c = oracle.mlp_fwd(x, P)
    t = tgt.astype(np.float64)
    dc = error_bound(x, P)
    want_loss = scale * np.sum((c - t) ** 2)
    bl = scale * np.sum(2 * np.abs(c - t) * dc + dc * dc) + S * 3 * F32 * want_loss
    assert abs(loss.item() - want_loss) <= bl, (loss.item(), want_loss, bl)
    G = 2 * scale * (c - t)
    want_P, dx = oracle.mlp_bwd(x, P, G)
    bP, bdx, massP = bwd_bounds(x, P, G, eG=2 * scale * dc)
    want_z = dx[:, :16].reshape(n, per, 16).sum(1)
    bz = bdx[:, :16].reshape(n, per, 16).sum(1) + per * F32 * np.abs(dx[:, :16]).reshape(n, per, 16).sum(1)
    _check_grads("distill", dP.cpu().numpy().astype(np.float64), want_P, bP,
                 dlat.cpu().numpy().astype(np.float64), want_z, bz, massP)


@pytest.mark.parametrize("n", [6000, 200000])
def test_project_bwd_learned_colour(gs, n):
    """colour_mode 1 backward: geometry gradients as the SH path's (degree 0
    carries no direction term), plus the decoder's latent, weight and
    view-direction gradients, against the FP64 oracle / torch autograd;
    200,000 is the learned-colour workload in full (its weight gradient sums
    over all of them)."""
    from oracle import brute
    from gpu_helpers import grad_close
    scene = scenes.config_scene(5, n=n)
    cam = scenes.config_camera(5)
    n = scene.n
    say(f"[project bwd learned colour] n={n}")
    Pbits = kaiming_params(6)
    packed = _packed(gs, Pbits)
    p = {k: to_dev(v) for k, v in scene.arrays().items()}
    lat = to_dev(scene.latents.view(np.int16))
    g = gs.gaussians_struct_mlp(p["means"], p["log_scales"], p["quats"], p["logits"], lat, packed)
    out = gs.ProjectedBuffers(n, DEV)
    cs = gs.camera_struct(cam)
    gs.project(g, cs, out)
    g2d_h = np.random.default_rng(7).normal(size=(gs.G2D, n)).astype(np.float32)
    grads = {kk: torch.empty_like(p[kk]) for kk in ("means", "log_scales", "quats", "logits")}
    grads["latents"] = torch.empty((n, 16), dtype=torch.float32, device=DEV)
    grads["mlp"] = torch.empty(oracle.MLP_PARAMS, dtype=torch.float32, device=DEV)
    ws = torch.empty(gs.project_bwd_workspace(g), dtype=torch.uint8, device=DEV)
    gs.project_bwd(g, cs, to_dev(g2d_h), grads, proj=out, ws=ws)
    torch.cuda.synchronize()
    live = out.radius.cpu().numpy() > 0
    # geometry: the oracle's SH backward on a degree-0 copy (no direction term)
    s0 = scenes.Scene(n, 0, scene.means, scene.log_scales, scene.quats, scene.logits,
                      np.zeros((1, 3, n), np.float32))
    # g2d carries dL/dSigma' (the library's record-gradient form); the oracle's
    # projection backward takes the conic form: converted on the oracle's records
    o = oracle.project(s0, cam)
    geo = oracle.project_bwd(s0, cam, sigma_to_conic_grad(o["rec"], g2d_h.T))
    ok = (o["flags"] & 0b1110) == 0
    for kk in ("log_scales", "quats", "logits"):
        grad_close(grads[kk].cpu().numpy()[..., ok], geo[kk][..., ok], name=kk)
    # decoder part through torch autograd in FP64 (live Gaussians only)
    ca = oracle.cam_array(cam)
    centre = -(ca[7:16].reshape(3, 3).T @ ca[16:19])
    idx = np.nonzero(live)[0]
    mt = torch.tensor(scene.means[:, idx].astype(np.float64), requires_grad=True)
    zt = torch.tensor(scenes.bf16_to_f32(scene.latents[idx]).astype(np.float64), requires_grad=True)
    P = scenes.bf16_to_f32(Pbits).astype(np.float64)
    Pt = torch.tensor(P, requires_grad=True)
    Gc = g2d_h[6:9, idx].T.astype(np.float64)
    (brute.learned_colour(mt, centre, zt, Pt) * torch.tensor(Gc)).sum().backward()
    dirs = scene.means[:, idx].astype(np.float64).T - centre
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x = oracle.mlp_inputs(zt.detach().numpy(), dirs[:, None, :])
    # the kernel's direction is FP32: widen the input bound of the SH half
    ex = np.concatenate([np.zeros((len(idx), 16)), (U + 1e-5) * np.abs(x[:, 16:]) + 1e-6], axis=1)
    bP, bdx, massP = bwd_bounds(x, P, Gc, ex=ex)
    got_z = grads["latents"].cpu().numpy().astype(np.float64)
    assert (got_z[~live] == 0).all()
    _check_grads("learned colour", grads["mlp"].cpu().numpy().astype(np.float64), Pt.grad.numpy(), bP,
                 got_z[idx], zt.grad.numpy(), bdx[:, :16], massP)
    # means: geometry (1e-3 relative) + the direction share, whose error is at
    # most |grad Y_j| <= 10 on the unit sphere times the dL/dY bound, over |v|
    share = mt.grad.numpy()
    want_m = geo["means"].copy()
    want_m[:, idx] += share
    got_m = grads["means"].cpu().numpy().astype(np.float64)
    ref = np.maximum(np.abs(geo["means"]), 1e-3 * np.abs(geo["means"]).max())
    bound = 1e-3 * ref
    vlen = np.linalg.norm(scene.means[:, idx].astype(np.float64).T - centre, axis=1)
    bound[:, idx] += 1e-5 * np.abs(share) + (10 * bdx[:, 16:].sum(1) / vlen)[None, :]
    err = np.abs(got_m - want_m)
    assert (err[:, ok] <= bound[:, ok]).all(), (err[:, ok] / bound[:, ok]).max()
    say(f"  means: max err/bound {(err[:, ok] / bound[:, ok]).max():.3f}")

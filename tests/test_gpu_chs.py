"""Colour-hash sampling (Sec. IV-C.1), the approximate compositing mode, on
the GPU through the C ABI against the oracle (staged: the oracle takes the HIP
path's own FP32 records and lists):
  - buckets and group representatives of every list entry bit-exact, the
    bucket table's counts exact and its float sums within their FP32 bound;
  - the forward image, final_T and n_contrib as the oracle's walk over its
    per-entry records (near-threshold pixels resolved by branch, as in the
    exact mode's staged test), for the PLAIN and BALANCED work splits, which
    give the same bits;
  - the backward's record gradients (the aggregation's chain rule included)
    within 1e-3 relative against the oracle's;
  - the unsupported combinations are refused.
Scenes: the tiny and skewed workloads and the skewed scene with spatially
coherent colour (where most entries of dense tiles merge)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import (DEV, STAGED_MARGINS, check_render, conic_to_sigma_grad, fmt_flags, gpu_bin_sort, gpu_project,
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
        return scenes.config_scene(1), scenes.config_camera(1, bg=(0.2, 0.5, 0.8))
    if name == "skewed":
        return scenes.config_scene(2), scenes.config_camera(2)
    if name == "coherent":
        return scenes.coherent_colour(scenes.config_scene(2), 2077), scenes.config_camera(2)
    if name == "ragged":
        s = scenes.coherent_colour(scenes.skewed_scene(20000, 77, n_clusters=16, log_scale_mean=-3.6), 78)
        return s, scenes.pinhole(100, 70, 60.0, np.eye(3), (0.05, -0.02, 3.0), bg=(0.1, 0.0, 0.3))
    raise KeyError(name)


def _render(gs, n, out, pl, ranges, k, cam, schedule):
    cs = gs.camera_struct(cam)
    H, W = cam.height, cam.width
    image = torch.empty((3, H, W), dtype=torch.float32, device=DEV)
    fT = torch.empty((H, W), dtype=torch.float32, device=DEV)
    nc = torch.empty((H, W), dtype=torch.int32, device=DEV)
    ck = torch.empty(gs.render_ckpt_floats(k, cs), dtype=torch.float32, device=DEV)
    gs.render_fwd(n, out, pl, ranges, k, cs, image, fT, nc, ck, schedule=schedule | gs.RENDER_COLOUR_HASH)
    torch.cuda.synchronize()
    return image, fT, nc, ck


def _render_bwd(gs, n, out, pl, ranges, k, cam, fT, nc, ck, G, schedule):
    cs = gs.camera_struct(cam)
    g2d = torch.empty((gs.G2D, n), dtype=torch.float32, device=DEV)
    ws = torch.empty(max(gs.render_bwd_2d_workspace(n, k, cs, False), 1), dtype=torch.uint8, device=DEV)
    gs.render_bwd_2d(n, out, pl, ranges, k, cs, fT, nc, ck, G, g2d, ws, False,
                     schedule=schedule | gs.RENDER_COLOUR_HASH)
    torch.cuda.synchronize()
    return g2d.cpu().numpy().T.astype(np.float64)


@pytest.mark.parametrize("name", ["tiny", "ragged", "skewed", "coherent"])
def test_colour_hash_sampling_matches_oracle(gs, name):
    scene, cam = _case(name)
    n = scene.n
    say(f"[colour hash {name}] n={n} {cam.width}x{cam.height}")
    p, g, out = gpu_project(gs, scene, cam)
    h = proj_host(out)
    rec = h["rec"][:, :9].astype(np.float64)
    k, pl, ranges = gpu_bin_sort(gs, n, out, cam)
    o_pl = pl[:k].cpu().numpy().view(np.uint32)
    o_ranges = ranges.cpu().numpy().view(np.uint32)
    # buckets: from the FP32 colours of the HIP path's own records
    hashes = oracle.colour_hash(h["rec"][:, 6:9])
    agg = oracle.chs_aggregate(rec, o_pl, o_ranges, hashes, 256)

    # ---- bucket table, per-entry buckets and representatives
    cnt = torch.empty(gs.COLOUR_BUCKETS, dtype=torch.int32, device=DEV)
    sums = torch.empty((gs.COLOUR_BUCKETS, 4), dtype=torch.float32, device=DEV)
    bucket = torch.empty(max(k, 1), dtype=torch.int16, device=DEV)
    rep = torch.empty(max(k, 1), dtype=torch.int32, device=DEV)
    gs.colour_hash_table(n, out, pl, ranges, k, gs.camera_struct(cam), cnt, sums, bucket, rep)
    torch.cuda.synchronize()
    assert np.array_equal(bucket[:k].cpu().numpy().view(np.uint16), hashes[o_pl]), "buckets"
    assert np.array_equal(rep[:k].cpu().numpy().view(np.uint32).astype(np.int64), agg["rep"]), "representatives"
    got_cnt = cnt.cpu().numpy().view(np.uint32)
    assert np.array_equal(got_cnt, agg["tab_count"]), "bucket counts"
    # an FP32 sum of c positive terms errs by at most c 2^-24 of the sum
    got_sum = sums.cpu().numpy().astype(np.float64)
    bound = (got_cnt[:, None] * 2.0 ** -24 + 1e-6) * agg["tab_sum"] + 1e-30
    assert (np.abs(got_sum - agg["tab_sum"]) <= bound).all(), "bucket sums"
    merged = float((agg["rep"] != np.arange(k)).mean())
    say(f"  K={k}: {merged:.1%} of the entries merged into a representative, "
        f"{int((got_cnt > 0).sum())} buckets used")

    # ---- forward: the oracle's walk over its per-entry records
    image, fT, nc, ck = _render(gs, n, out, pl, ranges, k, cam, gs.SCHEDULE_BALANCED)
    ident = np.arange(k, dtype=np.uint32)
    _, _, _, flips, amb, st = check_render(image, fT, nc, agg["rec_e"], ident, o_ranges, cam)
    say(f"  forward: max err {st['max_err']:.2e}; " + fmt_flags(st))
    image_p, fT_p, nc_p, _ = _render(gs, n, out, pl, ranges, k, cam, gs.SCHEDULE_PLAIN)
    assert torch.equal(image, image_p) and torch.equal(fT, fT_p) and torch.equal(nc, nc_p)
    # the approximation against the exact method (reported)
    exact = oracle.render_fwd(rec, o_pl, o_ranges, cam)[0]
    mse = float(np.mean((np.clip(image.cpu().numpy(), 0, 1) - np.clip(exact, 0, 1)) ** 2))
    say(f"  PSNR of the sampled image against the exact one: {10 * np.log10(1.0 / max(mse, 1e-30)):.2f} dB")

    # ---- backward
    G = scenes.upstream_grad(cam, 1001)
    G[:, amb] = 0.0
    g_e, mass_e, cmass_e = oracle.render_bwd(agg["rec_e"], ident, o_ranges, cam, G, with_mass=True, flips=flips,
                                             margins=STAGED_MARGINS)
    want = conic_to_sigma_grad(rec, oracle.chs_route(rec, o_pl, o_ranges, 256, agg, g_e))
    m_e = mass_e.copy()
    m_e[:, 2:5] = cmass_e
    mass = oracle.chs_route(rec, o_pl, o_ranges, 256, agg, m_e)   # non-negative shares: routed term masses
    for sched in (gs.SCHEDULE_BALANCED, gs.SCHEDULE_PLAIN):
        got = _render_bwd(gs, n, out, pl, ranges, k, cam, fT, nc, ck, to_dev(G), sched)
        worst = 0.0
        for j, nm in enumerate("u v Sxx Sxy Syy o r g b".split()):
            worst = max(worst, grad_close(got[:, j], want[:, j], name=f"g2d.{nm}", mass=mass[:, j]))
        say(f"  backward (schedule {sched}): worst rel err {worst:.2e}")


def test_colour_hash_sampling_refuses_unsupported_modes(gs):
    scene, cam = _case("tiny")
    n = scene.n
    p, g, out = gpu_project(gs, scene, cam)
    k, pl, ranges = gpu_bin_sort(gs, n, out, cam)
    cs = gs.camera_struct(cam)
    H, W = cam.height, cam.width
    image = torch.empty((3, H, W), dtype=torch.float32, device=DEV)
    fT = torch.empty((H, W), dtype=torch.float32, device=DEV)
    nc = torch.empty((H, W), dtype=torch.int32, device=DEV)
    ck = torch.empty(gs.render_ckpt_floats(k, cs), dtype=torch.float32, device=DEV)
    with pytest.raises(gs.GsError) as e:
        gs.render_fwd(n, out, pl, ranges, k, cs, image, fT, nc, ck,
                      schedule=gs.SCHEDULE_MERGED | gs.RENDER_COLOUR_HASH)
    assert e.value.status == gs.GS_ERR_UNSUPPORTED
    with pytest.raises(gs.GsError) as e:
        gs.render_fwd(n, out, pl, ranges, k, cs, image, fT, nc, ck, schedule=0x200)
    assert e.value.status == gs.GS_ERR_INVALID_ARG
    gs.render_fwd(n, out, pl, ranges, k, cs, image, fT, nc, ck,
                  schedule=gs.SCHEDULE_BALANCED | gs.RENDER_COLOUR_HASH)
    g2d = torch.empty((gs.G2D, n), dtype=torch.float32, device=DEV)
    ws = torch.empty(gs.render_bwd_2d_workspace(n, k, cs, True), dtype=torch.uint8, device=DEV)
    with pytest.raises(gs.GsError) as e:
        gs.render_bwd_2d(n, out, pl, ranges, k, cs, fT, nc, ck, torch.zeros((3, H, W), device=DEV), g2d, ws, True,
                         schedule=gs.SCHEDULE_BALANCED | gs.RENDER_COLOUR_HASH)
    assert e.value.status == gs.GS_ERR_UNSUPPORTED
    torch.cuda.synchronize()

"""The training step around the splatting step (needs the GPU): densification
statistics accumulated by the backward, the fused Adam step over every
Gaussian parameter array, and a short training run through both."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import DEV, say, to_dev

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "quats", "logits", "sh")
LRS = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "logits": 5e-2, "sh_dc": 2.5e-3, "sh_rest": 1.25e-4}


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_14564_amd import gs as mod
    return mod


def test_densify_stats_accumulate_over_views(gs):
    """Three views: the backward adds |(dL/du, dL/dv)| and a visibility count
    per Gaussian; they must equal the NumPy accumulation of the same views'
    record gradients (deterministic reduction, the 2D-level call) and tile
    counts."""
    from paper_2510_14564_amd.raster import Rasterizer
    scene = scenes.config_scene(2, n=50000)
    n = scene.n
    # a 25-degree field of view sees 70-74 % of the scene from each of these
    # orbit positions, so visibility differs between Gaussians and views
    cams = [scenes.orbit_camera(k, 32, 400, 300, fov_x_deg=25.0) for k in (0, 3, 7)]
    say(f"[densify stats] n={n}, {len(cams)} views")
    p = {k: to_dev(v) for k, v in scene.arrays().items() if k in PARAMS}
    rast = Rasterizer(cams[0], scene.sh_degree, device=DEV, deterministic=True)
    stats = rast.enable_densify_stats(n)
    g2ds, vis = [], []
    for i, cam in enumerate(cams):
        rast.set_camera(cam)
        st = rast.forward(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"])
        G = to_dev(scenes.upstream_grad(cam, 500 + i))
        rast.backward(st, p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], G)
        g2d = torch.empty((gs.G2D, n), dtype=torch.float32, device=DEV)
        ws = torch.empty(gs.render_bwd_2d_workspace(n, st.k, st.cs, True), dtype=torch.uint8, device=DEV)
        gs.render_bwd_2d(n, st.proj, st.point_list, st.ranges, st.k, st.cs, st.final_T, st.n_contrib, st.t_ckpt,
                         G, g2d, ws, deterministic=True)
        torch.cuda.synchronize()
        g2ds.append(g2d.cpu().numpy().T.astype(np.float64))
        vis.append(st.proj.tiles_touched.cpu().numpy() > 0)
    want_sum, want_cnt = oracle.densify_stats(g2ds, vis)
    got_sum = stats[0].cpu().numpy().astype(np.float64)
    got_cnt = stats[1].cpu().numpy()
    assert np.array_equal(got_cnt, want_cnt)
    assert (got_cnt > 0).sum() > 0.5 * n and (got_cnt < len(cams)).any()
    err = np.abs(got_sum - want_sum)
    assert (err <= 4e-7 * want_sum + 1e-30).all(), (err / np.maximum(want_sum, 1e-30)).max()
    assert (got_sum[got_cnt == 0] == 0).all()
    say(f"  counts exact, sums within {(err / np.maximum(want_sum, 1e-30)).max():.1e} relative")


@pytest.mark.parametrize("deg,n", [(3, 4096), (0, 1001), (3, 999), (2, 20000)])
def test_adam_gaussians_matches_oracle(gs, deg, n):
    """Three fused Adam steps over every parameter array (group learning
    rates, degree-0 SH apart from the rest) against the oracle's FP64 step;
    sizes with n % 4 != 0 take the scalar path."""
    rng = np.random.default_rng(n + deg)
    nc = (deg + 1) ** 2
    shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n), "logits": (n,), "sh": (nc, 3, n)}
    P = {k: rng.normal(size=s).astype(np.float32) for k, s in shapes.items()}
    M = {k: np.zeros(s, np.float32) for k, s in shapes.items()}
    V = {k: np.zeros(s, np.float32) for k, s in shapes.items()}
    dp = {k: to_dev(v) for k, v in P.items()}
    dm = {k: to_dev(v) for k, v in M.items()}
    dv = {k: to_dev(v) for k, v in V.items()}
    Po = {k: v.astype(np.float64) for k, v in P.items()}
    Mo = {k: v.astype(np.float64) for k, v in M.items()}
    Vo = {k: v.astype(np.float64) for k, v in V.items()}
    say(f"[adam gaussians] deg={deg} n={n}")
    # the library receives the hyper-parameters as FP32: the oracle uses those
    # values, widened exactly (1 - 0.999f differs from 1 - 0.999 by 1.3e-5)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    lrs = {k: f32(v) for k, v in LRS.items()}
    b1, b2, eps = f32(0.9), f32(0.999), f32(1e-15)
    Mabs = {k: np.zeros(s) for k, s in shapes.items()}
    for step, scale in enumerate((1.0, 1e-3, 30.0), start=1):
        g = {k: (rng.normal(size=s) * scale).astype(np.float32) for k, s in shapes.items()}
        for k in PARAMS:
            Mabs[k] = b1 * Mabs[k] + (1.0 - b1) * np.abs(g[k].astype(np.float64))
        gs.adam_gaussians(n, deg, dp, {k: to_dev(v) for k, v in g.items()}, dm, dv, LRS, step, beta1=0.9,
                          beta2=0.999, eps=1e-15)
        for k in PARAMS:
            lr = lrs[k] if k != "sh" else np.where(np.arange(nc)[:, None, None] == 0, lrs["sh_dc"], lrs["sh_rest"])
            Po[k], Mo[k], Vo[k] = oracle.adam_step(Po[k], g[k], Mo[k], Vo[k], lr, step, beta1=b1, beta2=b2, eps=eps)
    torch.cuda.synchronize()
    for k in PARAMS:
        lr = LRS[k] if k != "sh" else max(LRS["sh_dc"], LRS["sh_rest"])
        # the first moment is a signed sum b1^2 (1-b1) g1 + b1 (1-b1) g2 + (1-b1) g3:
        # its FP32 rounding is relative to the sum of its terms' magnitudes
        # (Mabs), not to the sum itself, which may cancel; the second moment's
        # terms are all non-negative
        for name, got, want, scale, tol in (("p", dp[k], Po[k], np.abs(Po[k]), 1e-4 * lr),
                                            ("m", dm[k], Mo[k], Mabs[k], 0.0), ("v", dv[k], Vo[k], np.abs(Vo[k]), 0.0)):
            got = got.cpu().numpy().astype(np.float64)
            err = np.abs(got - want)
            bound = 4e-7 * scale + tol + 1e-30
            assert (err <= bound).all(), (k, name, float((err / bound).max()))


def test_training_steps_reduce_the_loss(gs):
    """Twenty training iterations -- rasterize, L1, backward, fused Adam --
    on the skewed scene towards the render of a perturbed copy of it: the L1
    loss falls, and the densification statistics count every iteration that
    sees a Gaussian."""
    from paper_2510_14564_amd.raster import Rasterizer, l1_loss, rasterize
    scene = scenes.config_scene(2, n=50000)
    cam = scenes.config_camera(2)
    n = scene.n
    rng = np.random.default_rng(9)
    target_scene = scenes.Scene(n, scene.sh_degree, scene.means, scene.log_scales, scene.quats,
                                (scene.logits + rng.normal(0, 0.5, n)).astype(np.float32),
                                (scene.sh + rng.normal(0, 0.05, scene.sh.shape)).astype(np.float32))
    rast = Rasterizer(cam, scene.sh_degree, device=DEV)
    tp = {k: to_dev(v) for k, v in target_scene.arrays().items() if k in PARAMS}
    with torch.no_grad():
        target = rasterize(tp["means"], tp["log_scales"], tp["quats"], tp["logits"], tp["sh"], rast).clone()
    p = {k: to_dev(v).requires_grad_(True) for k, v in scene.arrays().items() if k in PARAMS}
    m = {k: torch.zeros_like(v) for k, v in p.items()}
    v = {k: torch.zeros_like(t) for k, t in p.items()}
    stats = rast.enable_densify_stats(n)
    losses = []
    for it in range(1, 21):
        img = rasterize(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], rast)
        loss, dimg = l1_loss(img.detach(), target)
        img.backward(dimg)
        gs.adam_gaussians(n, scene.sh_degree, {k: t.detach() for k, t in p.items()},
                          {k: t.grad for k, t in p.items()}, m, v, LRS, it)
        for t in p.values():
            t.grad = None
        losses.append(loss.item())
    say(f"  L1 {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.8 * losses[0]
    cnt = stats[1].cpu().numpy()
    assert cnt.max() == 20 and set(np.unique(cnt)) <= set(range(21))

"""Density control (Sec. III-C) on the GPU through the C ABI against the
oracle: densities, classes, nearest neighbours, mean k-nearest distances and
the merge pairing bit-exact; the output set's size and order exact; kept and
new Gaussians bit-exact (copies and the FP32 offset formula); merged
Gaussians within FP32 rounding of their formulas.  A full comparison on a
20k-Gaussian skewed scene and on the tiny workload, and sampled checks on the
200k skewed workload (the oracle's brute force runs on sampled points)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import DEV, say, to_dev

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "quats", "logits", "sh")


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_14564_amd import gs as mod
    return mod


def _run(gs, scene, params, noise, capacity=None):
    n, deg = scene.n, scene.sh_degree
    p = {k: to_dev(v) for k, v in scene.arrays().items() if k in PARAMS}
    g = gs.gaussians_struct(p["means"], p["log_scales"], p["quats"], p["logits"], p["sh"], deg)
    cap = capacity if capacity is not None else 2 * n
    nc = (deg + 1) ** 2
    out = {"means": torch.zeros((3, cap), device=DEV), "log_scales": torch.zeros((3, cap), device=DEV),
           "quats": torch.zeros((4, cap), device=DEV), "logits": torch.zeros(cap, device=DEV),
           "sh": torch.zeros((nc, 3, cap), device=DEV)}
    pts = {"rho": torch.empty(n, dtype=torch.int32, device=DEV), "cls": torch.empty(n, dtype=torch.uint8, device=DEV),
           "nn": torch.empty(n, dtype=torch.int32, device=DEV), "dbar": torch.empty(n, device=DEV),
           "fate": torch.empty(n, dtype=torch.int32, device=DEV)}
    ws = torch.empty(gs.density_control_workspace(n), dtype=torch.uint8, device=DEV)
    rep = gs.density_control(g, params, to_dev(noise), out, cap, ws, points=pts)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in pts.items()}
    outs = {k: v.cpu().numpy()[..., :rep["n_out"]].astype(np.float64) for k, v in out.items()}
    return rep, host, outs


def _prm(r, **kw):
    d = dict(radius=r, alpha=1.0, beta=1.0, knn=3, spread=1.5, jitter=0.1 * r, gamma=1.0)
    d.update(kw)
    return d


def _oracle_prm(d):
    f = lambda x: float(np.float32(x))  # noqa: E731  (the library takes FP32 parameters)
    return np.array([f(d["radius"]), f(d["alpha"]), f(d["beta"]), d["knn"], f(d["spread"]), f(d["jitter"]),
                     f(d["gamma"])])


@pytest.mark.parametrize("case", ["skewed20k", "tiny", "skewed20k_k5", "far_split", "far_whole"])
def test_density_control_matches_oracle(gs, case):
    if case == "tiny":
        scene, r, kw = scenes.config_scene(1), scenes.DENSITY_RADIUS[1], {}
    elif case.startswith("far"):
        # a radius far below the spacing of uniform points: every query is
        # still open after eight rings of cells and goes to the far search --
        # split over point ranges (3,000 queries) or one workgroup per query
        # over every point (20,000 queries, more than the split's 16,384 slots)
        n = 3000 if case == "far_split" else 20000
        scene, r, kw = scenes.uniform_scene(n, 91, sh_degree=1), 0.002, {}
    else:
        scene = scenes.skewed_scene(20000, 2077, n_clusters=16, log_scale_mean=-4.0, sh_degree=2)
        r, kw = 0.04, ({"knn": 5, "alpha": 0.5, "gamma": 0.5} if case.endswith("k5") else {})
    n = scene.n
    say(f"[density {case}] n={n} r={r}")
    prm = _prm(r, **kw)
    noise = scenes.density_noise(n, 77)
    rep, pts, out = _run(gs, scene, prm, noise)
    o = oracle.density_control(scene, _oracle_prm(prm), noise)
    assert np.array_equal(pts["rho"], o["rho"]), "densities"
    st = o["stats"]
    assert rep["rho_mean"] == st["mu"] and rep["rho_std"] == st["sigma"]
    assert rep["rho_low"] == st["rho_low"] and rep["rho_high"] == st["rho_high"]
    assert np.array_equal(pts["cls"].astype(np.int8), o["cls"]), "classes"
    assert np.array_equal(pts["nn"].astype(np.int64), o["nn"]), "nearest neighbours"
    assert np.array_equal(pts["dbar"], o["dbar"]), "mean k-nearest distances"
    # d_merge: FP64 sums in another order (relative 1e-12); a pair whose
    # distance lies that close to it may merge on one side only
    assert rep["d_merge"] == pytest.approx(st["d_merge"], rel=1e-12)
    dnn = np.sqrt(oracle.knn(scene.means, 1)[1][:, 0].astype(np.float64))
    near = np.abs(dnn - st["d_merge"]) <= 1e-9 * st["d_merge"]
    assert not near.any(), "a nearest distance lies at d_merge: the pairing is not determined"
    assert np.array_equal(pts["fate"].astype(np.int64), o["fate"]), "merge pairing / output order"
    assert rep["n_out"] == o["n_out"] and rep["n_new"] == int((o["cls"] == 1).sum())
    merged = np.zeros(rep["n_out"], bool)
    removed = np.flatnonzero(o["fate"] < 0)
    for i in np.flatnonzero(o["fate"] >= 0):
        if o["nn"][i] in removed and o["fate"][o["nn"][i]] < 0 and o["nn"][o["nn"][i]] == i:
            merged[o["fate"][i]] = True
    for k in PARAMS:
        got, want = out[k], o[k]
        assert np.array_equal(got[..., ~merged], want[..., ~merged]), f"{k}: copies and new points"
        if merged.any():
            err = np.abs(got[..., merged] - want[..., merged])
            assert (err <= 4e-6 * np.abs(want[..., merged]) + 4e-6).all(), (k, err.max())
    say(f"  rho mean {rep['rho_mean']:.2f} std {rep['rho_std']:.2f}; {rep['n_new']} new, {rep['n_merged']} merged, "
        f"{rep['n_out']} out")


def test_density_control_sampled_at_the_skewed_workload(gs):
    scene = scenes.config_scene(2)
    n, r = scene.n, scenes.DENSITY_RADIUS[2]
    say(f"[density skewed] n={n} r={r}")
    prm = _prm(r)
    noise = scenes.density_noise(n, 2078)
    rep, pts, out = _run(gs, scene, prm, noise)
    rng = np.random.default_rng(5)
    q = np.concatenate([rng.choice(n, 3000, replace=False), np.flatnonzero(pts["fate"] < 0)[:300]])
    assert np.array_equal(pts["rho"][q], oracle.density(scene.means, r, q)), "sampled densities"
    idx, d2 = oracle.knn(scene.means, 3, q)
    assert np.array_equal(pts["nn"][q], idx[:, 0]), "sampled nearest neighbours"
    s = np.zeros(len(q), np.float32)
    for m in range(3):
        s = (s + np.sqrt(d2[:, m])).astype(np.float32)
    assert np.array_equal(pts["dbar"][q], (s / np.float32(3)).astype(np.float32)), "sampled mean distances"
    # thresholds from the (sampled-exact) densities, exactly as the definition states
    rho = pts["rho"].astype(np.int64)
    S1, S2 = int(rho.sum()), int((rho * rho).sum())
    mu = S1 / n
    sigma = np.sqrt(max(S2 / n - mu * mu, 0.0))
    assert rep["rho_mean"] == mu and rep["rho_std"] == sigma
    assert rep["rho_low"] == mu - 1.0 * sigma and rep["rho_high"] == mu + 1.0 * sigma
    cls = np.where(rho < rep["rho_low"], 1, np.where(rho > rep["rho_high"], 2, 0))
    assert np.array_equal(pts["cls"], cls)
    # the pairing: mutual nearest high pairs within d_merge, the higher index removed
    nn = pts["nn"].astype(np.int64)
    i = np.arange(n)
    dq = np.sqrt(oracle.knn(scene.means, 1, i[pts["fate"] < 0])[1][:, 0].astype(np.float64))
    assert (dq <= rep["d_merge"] * (1 + 1e-12)).all()
    pair = (cls == 2) & (cls[nn] == 2) & (nn[nn] == i)
    removed = pts["fate"] < 0
    assert (removed <= (pair & (nn < i))).all()
    cand = np.flatnonzero(pair & (nn < i))
    dc = np.sqrt(oracle.knn(scene.means, 1, cand)[1][:, 0].astype(np.float64))
    inside = dc < rep["d_merge"] * (1 - 1e-9)
    assert removed[cand[inside]].all() and not removed[cand[dc > rep["d_merge"] * (1 + 1e-9)]].any()
    assert rep["n_out"] == n - int((pts["fate"] < 0).sum()) + int((cls == 1).sum())
    say(f"  rho mean {rep['rho_mean']:.2f} std {rep['rho_std']:.2f}; {rep['n_new']} new, {rep['n_merged']} merged")


def test_density_control_reports_capacity(gs):
    scene = scenes.config_scene(1)
    prm = _prm(scenes.DENSITY_RADIUS[1])
    noise = scenes.density_noise(scene.n, 9)
    rep, _, _ = _run(gs, scene, prm, noise)
    with pytest.raises(gs.GsError) as e:
        _run(gs, scene, prm, noise, capacity=rep["n_out"] - 1)
    assert e.value.status == gs.GS_ERR_CAPACITY and e.value.report["n_out"] == rep["n_out"]

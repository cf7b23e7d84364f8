"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: closed forms,
invariants, textbook tables, library routines (scipy, Python's sort), brute
force by torch.autograd, or central finite differences.  Paper passages:
Sec. II-A (G(x), EWA projection, front-to-back blending), Sec. IV-C.1 (16x16
tiles).
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import brute
from paper_2510_14564_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit(rng, n):
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ------------------------------------------------------------------ SH basis

def test_sh_basis_matches_textbook_table():
    rng = np.random.default_rng(1)
    for d in _unit(rng, 50):
        Y, _ = oracle.sh_basis(3, d)
        T = brute.sh_table(3, torch.tensor(d)).numpy()
        np.testing.assert_allclose(Y, T, rtol=0, atol=1e-14)


def test_sh_basis_matches_scipy_complex_harmonics():
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(2)
    for d in _unit(rng, 20):
        theta = math.acos(d[2]); phi = math.atan2(d[1], d[0])
        Y, _ = oracle.sh_basis(3, d)
        j = 0
        for l in range(4):
            for m in range(-l, l + 1):
                c = complex(sp.sph_harm_y(l, abs(m), theta, phi))   # Condon-Shortley phase included
                ref = c.real if m == 0 else (math.sqrt(2) * c.real if m > 0 else math.sqrt(2) * c.imag)
                assert abs(Y[j] - ref) < 1e-13, (l, m)
                j += 1


def test_sh_orthonormal_under_exact_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi is exact for degree <= 6 products
    xs, ws = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        s = math.sqrt(1 - x * x)
        for k in range(nphi):
            phi = 2 * math.pi * k / nphi
            Y, _ = oracle.sh_basis(3, [s * math.cos(phi), s * math.sin(phi), x])
            G += np.outer(Y, Y) * w * (2 * math.pi / nphi)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_sh_degree0_colour():
    # D = 0: colour = Y0 f0 + 1/2 with Y0 = 1/(2 sqrt(pi)), independent of the view
    s = scenes.uniform_scene(32, 3, sh_degree=0)
    cam = scenes.front_camera(64, 64)
    pr = oracle.project(s, cam)
    live = pr["radius"] > 0
    y0 = 0.5 / math.sqrt(math.pi)
    want = np.maximum(0.0, y0 * s.sh[0].astype(np.float64).T + 0.5)
    np.testing.assert_allclose(pr["rec"][live, 6:9], want[live], atol=1e-15)


def test_sh_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    for d in _unit(rng, 10):
        _, G = oracle.sh_basis(3, d)
        h = 1e-6
        for k in range(3):
            e = np.zeros(3); e[k] = h
            fd = (oracle.sh_basis(3, d + e)[0] - oracle.sh_basis(3, d - e)[0]) / (2 * h)
            np.testing.assert_allclose(G[:, k], fd, atol=1e-8)


# ----------------------------------------------------- closed-form renders

def _single(scale, o, colour, pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), log_scales=None, deg=0):
    y0 = 0.5 / math.sqrt(math.pi)
    nc = (deg + 1) ** 2
    sh = np.zeros((nc, 3, 1), np.float32)
    sh[0, :, 0] = (np.asarray(colour) - 0.5) / y0
    ls = np.full((3, 1), math.log(scale), np.float32) if log_scales is None else np.asarray(log_scales, np.float32).reshape(3, 1)
    logit = math.log(o / (1 - o))
    return scenes.Scene(1, deg, np.asarray(pos, np.float32).reshape(3, 1), ls,
                        np.asarray(quat, np.float32).reshape(4, 1), np.array([logit], np.float32), sh)


def test_single_isotropic_gaussian_closed_form():
    cam = scenes.front_camera(96, 80, 3.0, 60.0, bg=(0.2, 0.5, 0.8))
    colour = np.array([0.9, 0.3, 0.6])
    s = _single(0.05, 0.3, colour)
    f = oracle.forward(s, cam)
    o = 1.0 / (1.0 + math.exp(-float(s.logits[0])))
    sig2x = (cam.fx * 0.05 / 3.0) ** 2 + 0.3
    sig2y = (cam.fy * 0.05 / 3.0) ** 2 + 0.3
    ys, xs = np.mgrid[0:80, 0:96] + 0.5
    c = np.asarray(s.sh[0, :, 0], np.float64) * (0.5 / math.sqrt(math.pi)) + 0.5
    # s is stored in float32: use the widened values exactly as the oracle does
    sc = float(np.exp(np.float64(s.log_scales[0, 0])))
    sig2x = (np.float64(np.float32(cam.fx)) * sc / 3.0) ** 2 + 0.3
    sig2y = (np.float64(np.float32(cam.fy)) * sc / 3.0) ** 2 + 0.3
    dx = cam.cx - xs; dy = cam.cy - ys
    a = o * np.exp(-0.5 * (dx * dx / sig2x + dy * dy / sig2y))
    a = np.where(a >= 1.0 / 255.0, a, 0.0)
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    want = c[:, None, None] * a[None] + (1 - a)[None] * bg[:, None, None]
    np.testing.assert_allclose(f["image"], want, atol=1e-12)
    np.testing.assert_allclose(f["final_T"], 1 - a, atol=1e-12)


def test_ewa_area_and_second_moment():
    # rotated anisotropic Gaussian on the optical axis: the image of alpha integrates to
    # 2 pi sqrt(det S') (o - 1/255) and its normalised second moment is kappa S'
    # with S' = (f/tz)^2 Sigma_xy + 0.3 I, Sigma = R diag(s^2) R^T.
    from scipy.spatial.transform import Rotation
    q = np.array([0.9, 0.2, -0.3, 0.25]); q /= np.linalg.norm(q)
    ls = np.log([0.05, 0.02, 0.035])
    cam = scenes.front_camera(256, 256, 3.0, 60.0)
    s = _single(1.0, 0.8, (1.0, 1.0, 1.0), quat=q, log_scales=ls)
    f = oracle.forward(s, cam)
    img = f["image"][0]
    Rm = Rotation.from_quat(np.asarray(s.quats[[1, 2, 3, 0], 0], np.float64)).as_matrix()
    Sig = Rm @ np.diag(np.exp(2 * s.log_scales[:, 0].astype(np.float64))) @ Rm.T
    fx = np.float64(np.float32(cam.fx))
    Sp = (fx / 3.0) ** 2 * Sig[:2, :2] + 0.3 * np.eye(2)
    o = 1.0 / (1.0 + math.exp(-float(s.logits[0])))
    area = 2 * math.pi * math.sqrt(np.linalg.det(Sp)) * (o - 1 / 255)
    assert abs(img.sum() - area) / area < 2e-3
    ys, xs = np.mgrid[0:256, 0:256] + 0.5
    dx = xs - cam.cx; dy = ys - cam.cy
    w = img / img.sum()
    M = np.array([[np.sum(w * dx * dx), np.sum(w * dx * dy)], [np.sum(w * dx * dy), np.sum(w * dy * dy)]])
    a2 = 2 * math.log(255 * o)
    kappa = (2 - (a2 + 2) * math.exp(-a2 / 2)) / (2 * (1 - math.exp(-a2 / 2)))
    np.testing.assert_allclose(M, kappa * Sp, rtol=5e-3, atol=5e-3 * np.abs(Sp).max())


def _white_scene(n, seed, deg=3):
    s = scenes.skewed_scene(n, seed, n_clusters=4, log_scale_mean=-3.0, sh_degree=deg)
    s.sh[:] = 0.0
    s.sh[0] = 0.5 / (0.5 / math.sqrt(math.pi))    # colour exactly 1 in FP64 up to one rounding
    return s


def test_partition_of_unity_and_transmittance_bounds():
    s = _white_scene(400, 11)
    cam = scenes.front_camera(80, 72, 3.0, 60.0)
    f = oracle.forward(s, cam)
    c = f["proj"]["rec"][:, 6:9]
    live = f["proj"]["radius"] > 0
    assert np.abs(c[live] - 1.0).max() < 1e-6
    # out = sum c alpha T; with c == c0 exactly per Gaussian, out / c0 = 1 - T_final
    c0 = c[live][0, 0]
    np.testing.assert_allclose(f["image"] / c0, np.broadcast_to(1 - f["final_T"], f["image"].shape), atol=1e-12)
    assert f["final_T"].min() >= 1e-4 and f["final_T"].max() <= 1.0
    nt = (f["ranges"][:, 1] - f["ranges"][:, 0]).reshape(cam.tiles_y, cam.tiles_x)
    ntp = np.kron(nt, np.ones((16, 16), np.int64))[:cam.height, :cam.width]
    assert (f["n_contrib"] <= ntp).all()
    assert (f["final_T"] < 1).sum() > 100


def _records_at_pixel(n, alpha, px, py):
    rec = np.zeros((n, 9))
    rec[:, 0] = px + 0.5; rec[:, 1] = py + 0.5
    rec[:, 2] = 0.01; rec[:, 3] = 0.0; rec[:, 4] = 0.01
    rec[:, 5] = alpha; rec[:, 6:9] = 1.0
    return rec


def _load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return rows


def test_termination_counts_golden():
    cam = scenes.front_camera(32, 32, 3.0, 60.0)
    for alpha, want in _load_golden("termination_counts.txt"):
        n = 200
        rec = _records_at_pixel(n, alpha, 5, 7)
        depth = np.arange(1, n + 1, dtype=np.float32)
        radius = np.full(n, 3, np.int32)
        pl, ranges, _, _ = oracle.bin_sort(rec[:, 0], rec[:, 1], radius, depth, 32, 32)
        _, fT, nc, _ = oracle.render_fwd(rec, pl, ranges, cam)
        assert nc[7, 5] == int(want), alpha
        assert abs(fT[7, 5] - (1 - alpha) ** int(want)) < 1e-15
        # closed form floor(ln 1e-4 / ln(1 - alpha))
        assert int(want) == math.floor(math.log(1e-4) / math.log(1 - alpha))


def test_skip_below_alpha_min_and_clamp_at_099():
    cam = scenes.front_camera(48, 48, 3.0, 60.0, bg=(0.2, 0.5, 0.8))
    s = _single(0.1, 0.003, (0.9, 0.1, 0.4))        # o < 1/255: never blended
    f = oracle.forward(s, cam)
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    np.testing.assert_allclose(f["image"], np.broadcast_to(bg[:, None, None], f["image"].shape), atol=0)
    assert (f["n_contrib"] == 0).all() and (f["final_T"] == 1).all()
    # o e^power >= 0.99 near the centre: alpha clamps, out = 0.99 c + 0.01 bg, dL/do = 0 there
    s = _single(1.0, 0.999, (0.9, 0.1, 0.4))
    f = oracle.forward(s, cam)
    c = f["proj"]["rec"][0, 6:9]
    want = 0.99 * c + 0.01 * bg
    np.testing.assert_allclose(f["image"][:, 24, 24], want, atol=1e-14)
    G = np.zeros((3, 48, 48)); G[:, 24, 24] = 1.0
    g2d = oracle.render_bwd(f["proj"]["rec"], f["point_list"], f["ranges"], cam, G)
    assert g2d[0, 5] == 0.0 and g2d[0, 0] == 0.0


def _walk_at(rec, cam, px, py, flips=0, margins=None, G=None):
    """Render records stacked on one pixel (depth = order) with a near-decision
    mask at that pixel; returns the pixel's colour, T, n_contrib, flags, near
    count and, with an upstream gradient G at the pixel, the record gradients."""
    n = len(rec)
    depth = np.arange(1, n + 1, dtype=np.float32)
    radius = np.full(n, 3, np.int32)
    pl, ranges, _, _ = oracle.bin_sort(rec[:, 0], rec[:, 1], radius, depth, cam.width, cam.height)
    fl = np.zeros((cam.height, cam.width), np.uint8)
    fl[py, px] = flips
    img, fT, nc, flags, nn = oracle.render_fwd(rec, pl, ranges, cam, margins=margins, flips=fl, with_near=True)
    g2d = None
    if G is not None:
        Gi = np.zeros((3, cam.height, cam.width))
        Gi[:, py, px] = G
        g2d = oracle.render_bwd(rec, pl, ranges, cam, Gi, margins=margins, flips=fl)
    return img[:, py, px], fT[py, px], int(nc[py, px]), int(flags[py, px]), int(nn[py, px]), g2d


def test_near_decision_flips_match_nudged_inputs():
    """Taking the other branch of a near-threshold decision (the masks that
    locate FP32/FP64 splits) gives the plain walk of an input nudged across the
    threshold, forward and backward; bits follow the walk order."""
    cam = scenes.front_camera(32, 32, 3.0, 60.0, bg=(0.2, 0.5, 0.8))
    px, py = 5, 7
    G = np.array([0.7, -0.4, 1.1])
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    # alpha vs 1/255: a single entry at the pixel centre (power 0, alpha = o)
    up = _records_at_pixel(1, (1 + 1e-7) / 255, px, py)
    dn = _records_at_pixel(1, (1 - 1e-7) / 255, px, py)
    c0, T0, n0, f0, k0, _ = _walk_at(up, cam, px, py)
    assert (n0, f0, k0) == (1, 1, 1)
    c1, T1, n1, _, _, _ = _walk_at(up, cam, px, py, flips=1)
    cd, Td, nd, fd, _, _ = _walk_at(dn, cam, px, py)
    assert (n1, nd, fd) == (0, 0, 1) and T1 == Td == 1.0
    np.testing.assert_allclose(c1, bg, atol=0) and np.testing.assert_allclose(cd, bg, atol=0)
    assert _walk_at(up, cam, px, py, margins=(0.0, 0.0, 0.0))[3] == 0
    # two near entries: bit k flips the k-th near decision met by the walk
    two = np.concatenate([up, dn])
    assert _walk_at(two, cam, px, py)[2:5] == (1, 1, 2)
    for mask, want_nc, want_T in ((1, 0, 1.0), (2, 2, (1 - up[0, 5]) * (1 - dn[0, 5])), (3, 2, 1 - dn[0, 5])):
        _, T, nc, _, _, _ = _walk_at(two, cam, px, py, flips=mask)
        assert nc == want_nc and abs(T - want_T) < 1e-15, mask
    # T' vs 1e-4: identical entries whose 14th blend lands just below / above 1e-4
    a_lo = 1 - (1e-4 * (1 - 1e-9)) ** (1 / 14)
    a_hi = 1 - (1e-4 * (1 + 1e-9)) ** (1 / 14)
    lo = _records_at_pixel(20, a_lo, px, py)
    hi = _records_at_pixel(20, a_hi, px, py)
    c0, T0, n0, f0, k0, g0 = _walk_at(lo, cam, px, py, G=G)
    assert n0 == 13 and f0 & 2 and k0 == 1
    c1, T1, n1, _, _, g1 = _walk_at(lo, cam, px, py, flips=1, G=G)
    ch, Th, nh, _, _, gh = _walk_at(hi, cam, px, py, G=G)
    assert n1 == nh == 14
    np.testing.assert_allclose(c1, ch, rtol=1e-7)
    np.testing.assert_allclose(T1, Th, rtol=1e-7)
    np.testing.assert_allclose(g1, gh, rtol=1e-6, atol=1e-12)
    assert not g0[13].any() and np.abs(g1[13]).max() > 0   # the 14th entry's gradient exists only when blended
    # o e^power vs 0.99: clamped (dL/do = 0) or not
    cl = _records_at_pixel(1, 0.99 * (1 + 1e-7), px, py)
    un = _records_at_pixel(1, 0.99 * (1 - 1e-7), px, py)
    _, _, _, f0, k0, g0 = _walk_at(cl, cam, px, py, G=G)
    assert f0 == 4 and k0 == 1 and g0[0, 5] == 0.0
    _, _, _, _, _, g1 = _walk_at(cl, cam, px, py, flips=1, G=G)
    _, _, _, _, _, gu = _walk_at(un, cam, px, py, G=G)
    assert gu[0, 5] != 0.0
    np.testing.assert_allclose(g1, gu, rtol=1e-6, atol=1e-15)


def test_record_gradients_match_finite_differences():
    """Every record channel of the render backward -- centre (u, v), the conic
    entries A, B, C as they enter the power (B once), opacity and colour --
    against central differences of the FP64 render in that record entry, at
    entries where no pixel's decisions move."""
    s = _tiny_scene(24)
    cam = scenes.pinhole(40, 36, 60.0, np.eye(3), (0.05, 0.0, 3.0), bg=(0.2, 0.5, 0.8))
    f = oracle.forward(s, cam)
    rec, pl, ranges = f["proj"]["rec"], f["point_list"], f["ranges"]
    G = scenes.upstream_grad(cam, 8)
    g2d = oracle.render_bwd(rec, pl, ranges, cam, G)
    checked = 0
    for i in np.argsort(-np.abs(g2d[:, 5]))[:8]:
        for ch in range(9):
            h = 1e-5 * max(abs(rec[i, ch]), 1e-3)
            vals = []
            for sgn in (1, -1):
                r2 = rec.copy()
                r2[i, ch] += sgn * h
                img, _, nc, _ = oracle.render_fwd(r2, pl, ranges, cam)
                vals.append((float(np.sum(G * img)), nc))
            if not (np.array_equal(vals[0][1], f["n_contrib"]) and np.array_equal(vals[1][1], f["n_contrib"])):
                continue
            fd = (vals[0][0] - vals[1][0]) / (2 * h)
            scale = np.abs(g2d[:, ch]).max()
            assert abs(fd - g2d[i, ch]) <= 1e-5 * max(abs(g2d[i, ch]), 1e-3 * scale), (i, ch, fd, g2d[i, ch])
            checked += 1
    assert checked >= 60


# ------------------------------------------------------------------ binning

def _py_bin_sort(u, v, r, depth, W, H):
    tx = (W + 15) // 16
    ntiles = tx * ((H + 15) // 16)
    entries = []
    bits = np.asarray(depth, np.float32).view(np.uint32)
    for i in range(len(u)):
        rc = brute._rect(float(u[i]), float(v[i]), int(r[i]), W, H)
        if rc is None:
            continue
        x0, x1, y0, y1 = rc
        for y in range(y0, y1 + 1):
            for x in range(x0, x1 + 1):
                entries.append((y * tx + x, int(bits[i]), i))
    entries.sort()
    pl = np.array([e[2] for e in entries], np.uint32)
    tiles = np.array([e[0] for e in entries], np.int64)
    starts = np.searchsorted(tiles, np.arange(ntiles), side="left")
    ends = np.searchsorted(tiles, np.arange(ntiles), side="right")
    return pl, np.stack([starts, ends], 1).astype(np.uint32)


def test_bin_sort_matches_python_sort_with_ties_and_offscreen():
    rng = np.random.default_rng(5)
    n, W, H = 3000, 100, 70          # ragged: 7 x 5 tiles, the last row and column partial
    u = rng.uniform(-60, 160, n).astype(np.float32).astype(np.float64)
    v = rng.uniform(-60, 130, n).astype(np.float32).astype(np.float64)
    r = rng.integers(0, 40, n).astype(np.int32)
    depth = rng.choice(np.float32([1.0, 1.5, 2.25, 3.0, 7.0]), n)       # many exact ties
    pl, ranges, tt, off = oracle.bin_sort(u, v, r, depth, W, H)
    want_pl, want_ranges = _py_bin_sort(u, v, r, depth, W, H)
    assert np.array_equal(pl, want_pl)
    assert np.array_equal(ranges, want_ranges)
    assert tt.sum() == len(pl) and off[-1] + tt[-1] == len(pl)
    # rectangles and per-tile counts against the Python rectangles and sort
    rect, counts, K = oracle.bin_rects(u, v, r, W, H)
    assert K == len(want_pl)
    assert np.array_equal(counts, (want_ranges[:, 1] - want_ranges[:, 0]).astype(np.int64))
    for i in range(n):
        rc = brute._rect(float(u[i]), float(v[i]), int(r[i]), W, H)
        assert (rect[i, 1] < rect[i, 0]) if rc is None else tuple(rect[i]) == rc, i
    # a tile mask keeps exactly the selected tiles' lists, in the same order
    mask = np.zeros(len(want_ranges), np.uint8)
    mask[[0, 3, 4, 11, 34]] = 1
    mpl, mranges, _, _ = oracle.bin_sort(u, v, r, depth, W, H, tile_mask=mask)
    m = 0
    for t in range(len(mask)):
        s, e = mranges[t]
        if mask[t]:
            assert s == m and np.array_equal(mpl[s:e], want_pl[want_ranges[t, 0]:want_ranges[t, 1]]), t
            m = e
        else:
            assert s == e == m, t
    assert m == len(mpl)


def test_tile_rect_integer_form_avoids_fp32_round_up():
    # u = 0.99999994f, r = 15: u + r rounds to 16.0 in FP32, but the square
    # [u - 15, u + 15] ends below 16, so only tile column 0 is touched.
    u = float(np.float32(0.99999994))
    assert np.float32(u) + np.float32(15) == np.float32(16.0)
    cnt, rect = oracle.tile_rect(u, 8.0, 15, 64, 64)
    assert rect[0] == 0 and rect[1] == 0
    cnt, rect = oracle.tile_rect(-15.0, 8.0, 15, 64, 64)       # touches x = 0 exactly
    assert cnt > 0 and rect[1] == 0
    cnt, rect = oracle.tile_rect(-15.5, 8.0, 15, 64, 64)       # square ends at -0.5: off-screen
    assert cnt == 0
    cnt, rect = oracle.tile_rect(float("nan"), 8.0, 15, 64, 64)
    assert cnt == 0


def test_culling_special_cases():
    cam = scenes.front_camera(40, 40, 3.0, 60.0, bg=(0.1, 0.2, 0.3))
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    empty = scenes.uniform_scene(0, 1)
    behind = scenes.uniform_scene(50, 2)
    behind.means[2] = -5.0                                   # tz = -2 <= near
    nan = scenes.uniform_scene(50, 3)
    nan.means[0, :] = np.nan
    for s in (empty, behind, nan):
        f = oracle.forward(s, cam)
        assert len(f["point_list"]) == 0
        np.testing.assert_array_equal(f["image"], np.broadcast_to(bg[:, None, None], (3, 40, 40)))
        assert (f["final_T"] == 1).all() and (f["n_contrib"] == 0).all()


def test_permutation_invariance():
    s = scenes.uniform_scene(300, 8, log_scale_mean=-3.0)
    cam = scenes.front_camera(64, 48, 3.0, 60.0)
    f = oracle.forward(s, cam)
    d = f["proj"]["depth"].astype(np.float32)
    assert len(np.unique(d)) == len(d)
    perm = np.random.default_rng(9).permutation(s.n)
    f2 = oracle.forward(s.subset(perm), cam)
    assert np.array_equal(f["image"], f2["image"])
    assert np.array_equal(f["final_T"], f2["final_T"])


# ---------------------------------------------------------------- rotation

def test_quaternion_sign_and_scale_invariance_and_isotropic_zero_grad():
    s = scenes.uniform_scene(64, 12, log_scale_mean=-3.0, sh_degree=1)
    cam = scenes.front_camera(64, 64, 3.0, 60.0)
    base = oracle.project(s, cam)["rec"]
    for factor in (-1.0, 4.0, 0.25, -2.0):   # exact in FP32
        s2 = scenes.Scene(s.n, s.sh_degree, s.means, s.log_scales, (s.quats * np.float32(factor)).astype(np.float32),
                          s.logits, s.sh)
        np.testing.assert_allclose(oracle.project(s2, cam)["rec"], base, rtol=1e-12, atol=1e-12)
    iso = scenes.Scene(s.n, s.sh_degree, s.means, np.repeat(s.log_scales[:1], 3, 0), s.quats, s.logits, s.sh)
    g2d = np.random.default_rng(1).standard_normal((s.n, 9))
    g = oracle.project_bwd(iso, cam, g2d)
    assert np.abs(g["quats"]).max() < 1e-9 * max(1.0, np.abs(g["log_scales"]).max())


# ------------------------------------------------------------------ gradients

def _tiny_scene(seed=21):
    s = scenes.skewed_scene(48, seed, n_clusters=3, log_scale_mean=-2.6, log_scale_std=0.3, sh_degree=3)
    s.means = (0.4 * s.means).astype(np.float32)
    return s


def test_oracle_matches_brute_force_image_and_autograd_gradients():
    s = _tiny_scene()
    cam = scenes.pinhole(50, 38, 60.0, np.eye(3), (0.1, -0.05, 3.0), bg=(0.2, 0.5, 0.8))
    f = oracle.forward(s, cam)
    img, params, pr = brute.render(s, cam, requires_grad=True)
    np.testing.assert_allclose(img.detach().numpy(), f["image"], atol=1e-12)
    G = scenes.upstream_grad(cam, 77)
    (img * torch.tensor(G.astype(np.float64))).sum().backward()
    g = oracle.backward(s, cam, f, G)
    for k in ("means", "log_scales", "quats", "logits", "sh"):
        ref = params[k].grad.numpy()
        np.testing.assert_allclose(g[k], ref, rtol=1e-9, atol=1e-11 * max(1.0, np.abs(ref).max()), err_msg=k)


def test_colour_gradient_is_exact_for_affine_dependence():
    s = _tiny_scene(22)
    cam = scenes.front_camera(40, 40, 3.0, 60.0)
    f = oracle.forward(s, cam)
    G = scenes.upstream_grad(cam, 5)
    g2d = oracle.render_bwd(f["proj"]["rec"], f["point_list"], f["ranges"], cam, G)
    rec = f["proj"]["rec"]
    for i in np.argsort(-np.abs(g2d[:, 6]))[:5]:
        for ch in range(3):
            r2 = rec.copy(); r2[i, 6 + ch] += 1.0
            img2, _, _, _ = oracle.render_fwd(r2, f["point_list"], f["ranges"], cam)
            dL = np.sum(G * (img2 - f["image"]))
            assert abs(dL - g2d[i, 6 + ch]) < 1e-12 * max(1, abs(dL))


def test_oracle_backward_matches_central_finite_differences():
    s = _tiny_scene(23)
    cam = scenes.pinhole(32, 32, 60.0, np.eye(3), (0.0, 0.0, 3.0))
    G = scenes.upstream_grad(cam, 6)
    f = oracle.forward(s, cam, margins=1e-3)
    g = oracle.backward(s, cam, f, G)

    def loss(sc):
        ff = oracle.forward(sc, cam)
        return float(np.sum(G * ff["image"])), ff

    rng = np.random.default_rng(0)
    checked = 0
    for k in ("means", "log_scales", "quats", "logits", "sh"):
        arr = getattr(s, k)
        flat_idx = rng.choice(arr.size, size=6, replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            x0 = float(arr[idx])
            h = 1e-6 * max(1.0, abs(x0))
            vals = []
            ok = True
            for sgn in (1, -1):
                s2 = scenes.Scene(s.n, s.sh_degree, *(np.asarray(getattr(s, a), np.float64).copy()
                                                      for a in ("means", "log_scales", "quats", "logits", "sh")))
                getattr(s2, k)[idx] = x0 + sgn * h
                L, ff = loss(s2)
                # only points whose discrete decisions do not move
                if (not np.array_equal(ff["n_contrib"], f["n_contrib"])
                        or not np.array_equal(ff["point_list"], f["point_list"])):
                    ok = False
                vals.append(L)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = g[k][idx]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.abs(g[k]).max(), 1e-9), (k, idx, fd, an)
            checked += 1
    assert checked >= 20

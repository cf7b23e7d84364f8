"""Pins of the oracle's colour-hash sampling mode (Sec. IV-C.1: colour
quantisation, hash-based grouping, bucket-wise aggregation) against what the
paper's formulas and plain arithmetic fix (CPU only): the quantisation against
the paper's floor formula in exact rational arithmetic, special values, the
grouping and aggregation against a brute-force Python grouping, the exact
method as the window-1 case, a closed form for co-located members, the bucket
table against a histogram, and the mode's backward against central finite
differences of its forward."""
from fractions import Fraction

import numpy as np

import oracle
from paper_2510_14564_amd import scenes


def _paper_level(v8: int) -> int:
    """c_q = floor(c / 256 * 16) for the 8-bit value c, exactly."""
    return int(Fraction(v8, 256) * 16 // 1)


def test_quantisation_matches_paper_formula_for_every_8bit_value():
    # the FP32 colour nearest to v8/255 maps back to v8, and its level is the
    # paper's floor(v8/256*16); the hash packs the three levels as R 256 + G 16 + B
    rng = np.random.default_rng(1)
    v = rng.integers(0, 256, size=(4000, 3))
    v[:256, 0] = np.arange(256)
    v[:256, 1] = np.arange(256)[::-1]
    v[:256, 2] = (np.arange(256) * 7) % 256
    rgb = (v / 255.0).astype(np.float32)
    got = oracle.colour_hash(rgb)
    want = np.array([_paper_level(a) * 256 + _paper_level(b) * 16 + _paper_level(c) for a, b, c in v])
    assert np.array_equal(got.astype(np.int64), want)
    # 16 levels of 16 eight-bit values each
    levels = [_paper_level(k) for k in range(256)]
    assert levels == [k // 16 for k in range(256)]


def test_quantisation_rounds_to_the_nearest_8bit_value():
    # colours half a step either side of an 8-bit value's centre: the level
    # changes exactly where the nearest 8-bit value crosses a multiple of 16
    for v8 in (15, 16, 31, 32, 127, 128, 239, 240):
        lo = np.float32((v8 - 0.49) / 255.0)
        hi = np.float32((v8 + 0.49) / 255.0)
        h = oracle.colour_hash(np.array([[lo, 0, 0], [hi, 0, 0]], np.float32))
        assert h[0] == h[1] == _paper_level(v8) * 256, (v8, h)


def test_quantisation_special_values():
    rgb = np.array([[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [-3, 7, np.nan], [np.inf, -np.inf, 1e-30]],
                   np.float32)
    h = oracle.colour_hash(rgb)
    assert h.tolist() == [0, 4095, 8 * 256 + 8 * 16 + 8, 15 * 16, 15 * 256]
    assert (oracle.colour_hash(np.random.default_rng(2).normal(0.5, 2.0, (10000, 3)).astype(np.float32)) < 4096).all()


def _lists(n_tiles, rng, n_gauss, max_len):
    """Random sorted-list structure: ranges over n_tiles tiles and a point list."""
    lens = rng.integers(0, max_len + 1, n_tiles)
    lens[0] = max_len
    ranges = np.zeros((n_tiles, 2), np.uint32)
    ranges[:, 1] = np.cumsum(lens)
    ranges[1:, 0] = ranges[:-1, 1]
    pl = rng.integers(0, n_gauss, int(lens.sum())).astype(np.uint32)
    return pl, ranges


def _py_aggregate(rec, pl, ranges, hashes, window):
    """Brute-force grouping: a dict per window from bucket to its members."""
    K = len(pl)
    rep = np.full(K, -1, np.int64)
    size = np.zeros(K, np.int64)
    rec_e = rec[pl].copy()
    for s, e in ranges:
        for w0 in range(int(s), int(e), window):
            groups = {}
            for m in range(w0, min(w0 + window, int(e))):
                groups.setdefault(int(hashes[pl[m]]), []).append(m)
            for members in groups.values():
                r = members[0]
                for m in members:
                    rep[m] = r
                    size[m] = len(members)
                    if m != r:
                        rec_e[m, 5] = 0.0
                rec_e[r, 6:9] = np.mean([rec[pl[m], 6:9] for m in members], axis=0)
                rec_e[r, 5] = 1.0 - np.prod([1.0 - rec[pl[m], 5] for m in members])
    return rep, size, rec_e


def test_aggregation_matches_brute_force_grouping():
    rng = np.random.default_rng(3)
    n = 300
    rec = rng.random((n, 9))
    rec[:, 5] = rng.uniform(0.01, 0.9, n)
    for n_buckets, window in ((5, 256), (40, 256), (3, 7), (4096, 256), (2, 1)):
        pl, ranges = _lists(9, rng, n, 600)
        hashes = rng.integers(0, n_buckets, n).astype(np.uint16)
        agg = oracle.chs_aggregate(rec, pl, ranges, hashes, window)
        rep, size, rec_e = _py_aggregate(rec, pl, ranges, hashes, window)
        assert np.array_equal(agg["rep"], rep)
        assert np.array_equal(agg["size"], size)
        assert np.allclose(agg["rec_e"], rec_e, rtol=1e-14, atol=1e-15)
        # bucket table: a histogram and sums over every list entry
        assert np.array_equal(agg["tab_count"], np.bincount(hashes[pl], minlength=4096))
        ts = np.zeros((4096, 4))
        np.add.at(ts, hashes[pl], rec[pl][:, [6, 7, 8, 5]])
        assert np.allclose(agg["tab_sum"], ts, rtol=1e-13, atol=0)


def _scene_lists(seed=31):
    s = scenes.skewed_scene(400, seed, n_clusters=4, log_scale_mean=-3.0, log_scale_std=0.4, sh_degree=1)
    s.means = (0.5 * s.means).astype(np.float32)
    cam = scenes.pinhole(64, 48, 60.0, np.eye(3), (0.0, 0.0, 3.0), bg=(0.2, 0.5, 0.8))
    f = oracle.forward(s, cam)
    rec = f["proj"]["rec"]
    return s, cam, f, rec, oracle.colour_hash(rec[:, 6:9].astype(np.float32))


def test_window_one_and_distinct_buckets_are_the_exact_method():
    s, cam, f, rec, h = _scene_lists()
    pl, ranges = f["point_list"], f["ranges"]
    exact = oracle.render_fwd(rec, pl, ranges, cam)
    for hashes, window in ((h, 1), (np.arange(rec.shape[0]).astype(np.uint16), 256)):
        img, fT, nc, _, agg = oracle.chs_render_fwd(rec, pl, ranges, cam, hashes, window)
        assert np.array_equal(agg["rep"], np.arange(len(pl)))
        assert np.array_equal(img, exact[0]) and np.array_equal(fT, exact[1]) and np.array_equal(nc, exact[2])
    # and a real window merges something on this scene
    agg = oracle.chs_aggregate(rec, pl, ranges, h, 256)
    assert (agg["rep"] != np.arange(len(pl))).sum() > 0


def test_co_located_members_composite_to_their_accumulated_opacity():
    # n Gaussians with one footprint centred on a pixel centre and one colour:
    # at that pixel (G = 1) the exact blend is c (1 - prod(1 - o_j)) + prod(1 - o_j) bg,
    # which is what their single representative composites to
    cam = scenes.pinhole(16, 16, 60.0, np.eye(3), (0.0, 0.0, 3.0), bg=(0.2, 0.5, 0.8))
    o = np.array([0.3, 0.5, 0.2, 0.4, 0.1])
    rec = np.zeros((5, 9))
    rec[:, 0] = 7.5; rec[:, 1] = 9.5
    rec[:, 2] = 0.05; rec[:, 3] = 0.01; rec[:, 4] = 0.07
    rec[:, 5] = o
    rec[:, 6:9] = (0.25, 0.6, 0.9)
    pl = np.arange(5, dtype=np.uint32)
    ranges = np.array([[0, 5]], np.uint32)
    h = oracle.colour_hash(rec[:, 6:9].astype(np.float32))
    assert (h == h[0]).all()
    img, fT, nc, _, agg = oracle.chs_render_fwd(rec, pl, ranges, cam, h, 256)
    keep = np.prod(1.0 - o)
    bg = np.array([0.2, 0.5, 0.8], np.float32).astype(np.float64)
    want = np.array([0.25, 0.6, 0.9]) * (1 - keep) + keep * bg
    assert np.allclose(img[:, 9, 7], want, rtol=0, atol=1e-15)
    assert abs(fT[9, 7] - keep) < 1e-15 and nc[9, 7] == 1
    exact = oracle.render_fwd(rec, pl, ranges, cam)
    assert np.allclose(exact[0][:, 9, 7], want, rtol=0, atol=1e-15)


def test_sampling_backward_matches_finite_differences():
    """Record gradients of the sampling mode (backward of the walk over the
    per-entry records, then the aggregation's chain rule) against central
    differences of the mode's forward in each Gaussian record entry, at
    entries where no decision moves (same n_contrib, same groups)."""
    s, cam, f, rec, h = _scene_lists(33)
    pl, ranges = f["point_list"], f["ranges"]
    G = scenes.upstream_grad(cam, 9)
    g2d = oracle.chs_render_bwd(rec, pl, ranges, cam, h, 256, G)
    _, _, nc0, _, agg0 = oracle.chs_render_fwd(rec, pl, ranges, cam, h, 256)
    merged = np.unique(pl[agg0["rep"] != np.arange(len(pl))])
    cand = list(merged[:6]) + list(np.argsort(-np.abs(g2d[:, 5]))[:6])
    checked = 0
    for i in cand:
        for ch in range(9):
            hh = 1e-5 * max(abs(rec[i, ch]), 1e-3)
            vals = []
            for sgn in (1, -1):
                r2 = rec.copy()
                r2[i, ch] += sgn * hh
                img, _, nc, _, agg = oracle.chs_render_fwd(r2, pl, ranges, cam, h, 256)
                vals.append((float(np.sum(G * img)), nc, agg["rep"]))
            if not all(np.array_equal(v[1], nc0) and np.array_equal(v[2], agg0["rep"]) for v in vals):
                continue
            fd = (vals[0][0] - vals[1][0]) / (2 * hh)
            scale = np.abs(g2d[:, ch]).max()
            assert abs(fd - g2d[i, ch]) <= 1e-5 * max(abs(g2d[i, ch]), 1e-3 * scale), (i, ch, fd, g2d[i, ch])
            checked += 1
    assert checked >= 60
    # members that are not representatives get colour and opacity gradients only
    non_rep = np.setdiff1d(merged, pl[agg0["rep"] == np.arange(len(pl))])
    assert non_rep.size and np.all(g2d[non_rep, :5] == 0)

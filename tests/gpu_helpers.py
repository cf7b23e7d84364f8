"""Shared helpers for the GPU parity tests: upload seeded inputs, run the HIP
stages through the C ABI, and compare against the FP64 oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

DEV = "cuda"

# tolerances
PIX_ATOL = 1e-4          # pixels and final_T, absolute
GRAD_RTOL = 1e-3         # gradients: |g - g*| <= 1e-3 max(|g*|, 1e-3 max|g*|, 1e-2 mass)
# mass = sum of |per-pair terms| of g*: an FP32 sum of n terms carries a
# rounding error up to n * 2^-24 of its mass (about sqrt(n) * 2^-24 in
# practice); the floor only matters for sums that cancel by more than 100x
MASS_FLOOR = 1e-2
PROJ_RTOL = 2e-5         # projected quantities, relative to the field's scale
# near-threshold margins of the oracle's walk when it composites the HIP
# path's own FP32 records (staged): alpha vs 1/255 and o e^power vs 0.99 at
# 1e-5 relative plus 8 units of 2^-24 of the pair's power-term magnitude (the
# FP32 evaluation error of the power, large for elongated footprints whose
# terms cancel), T' vs 1e-4 from 1e-4 relative plus the error a product of
# (1 - alpha) factors accumulates; from raw parameters (end to end) the
# records themselves differ by FP32 rounding, so the fixed margins are 1e-3
STAGED_MARGINS = (1e-5, 1e-4, 1e-5, oracle.POWER_ERR)
E2E_MARGINS = (1e-3, 1e-3, 1e-3, oracle.POWER_ERR)


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


def grad_close(got, want, rtol=GRAD_RTOL, name="", mass=None, stats=None, extra=None):
    """Relative error 1e-3 against max(|g*|, 1e-3 max|g*|) and, when the oracle's
    term mass is given, 1e-2 of it: a sum that cancels by more than 100x is
    judged against its terms, which is what its rounding error scales with.
    extra (absolute, per entry) is added to the bound: the response of g* to
    a known error of its inputs.  Returns the worst ratio to the plain
    (mass-free) relative bound."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = np.abs(want).max() if want.size else 0.0
    ref = np.maximum(np.abs(want), 1e-3 * scale)
    plain = rtol * ref
    bound = plain if mass is None else rtol * np.maximum(ref, MASS_FLOOR * np.asarray(mass, np.float64))
    if extra is not None:
        bound = bound + np.asarray(extra, np.float64)
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
    parameter sum_j |d param / d record_j| weights[:, j] over the HIP path's
    record channels j (Sigma' entries), from one oracle pass per channel j (a Gaussian's parameter gradient depends on its own
    record gradient only).  With weights = |g2d| this is the sum of the chain
    rule's per-channel terms, which the FP32 rounding of a cancelling
    parameter gradient scales with."""
    n = scene.n
    rec = oracle.project(scene, cam)["rec"]
    out = [None] * len(weights)
    for j in range(9):
        e = np.zeros((n, 9))
        e[:, j] = 1.0
        col = oracle.project_bwd(scene, cam, sigma_to_conic_grad(rec, e))
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
    ws = torch.empty(max(gs.render_bwd_2d_workspace(n, k, cs, deterministic), 1), dtype=torch.uint8, device=DEV)
    gs.render_bwd_2d(n, out, pl, ranges, k, cs, fT, nc, ck, G, g2d, ws, deterministic, schedule=schedule)
    torch.cuda.synchronize()
    return g2d


# ------------------------------------------------- record gradient forms
# The oracle returns the conic entries of a record gradient as they enter the
# power (dL/dA, dL/dB, dL/dC of K = [[A, B], [B, C]]); the HIP path hands the
# projection dL/dSigma' of the covariance Sigma' = K^-1 = [[a, b], [b, c]]
# (b counted in both off-diagonal places).  dK = -K dSigma' K links them.

def _sym(a, b, c):
    M = np.empty((len(a), 2, 2))
    M[:, 0, 0] = a
    M[:, 0, 1] = M[:, 1, 0] = b
    M[:, 1, 1] = c
    return M


def conic_to_sigma_grad(rec, g):
    """g[n][9] with conic entries -> the same with dL/dSigma' (FP64)."""
    g = np.asarray(g, np.float64)
    K = _sym(rec[:, 2], rec[:, 3], rec[:, 4])
    Gc = _sym(g[:, 2], 0.5 * g[:, 3], g[:, 4])
    GS = -K @ Gc @ K
    out = g.copy()
    out[:, 2], out[:, 3], out[:, 4] = GS[:, 0, 0], 2.0 * GS[:, 0, 1], GS[:, 1, 1]
    return out


def sigma_to_conic_grad(rec, g):
    """Inverse of conic_to_sigma_grad for the records' conics (rows whose conic
    is zero, i.e. culled, keep zero conic entries)."""
    g = np.asarray(g, np.float64)
    A, B, C = rec[:, 2], rec[:, 3], rec[:, 4]
    det = A * C - B * B
    live = det > 0
    inv = np.where(live, 1.0 / np.where(live, det, 1.0), 0.0)
    S = _sym(C * inv, -B * inv, A * inv)
    GS = _sym(g[:, 2], 0.5 * g[:, 3], g[:, 4])
    Gc = -S @ GS @ S
    out = g.copy()
    out[:, 2], out[:, 3], out[:, 4] = Gc[:, 0, 0], 2.0 * Gc[:, 0, 1], Gc[:, 1, 1]
    out[~live, 2:5] = 0.0
    return out


def record_sensitivity(rec, pl, ranges, cam, G, deltas, tile_mask=None, flips=None, margins=STAGED_MARGINS):
    """How far the oracle's record gradients (Sigma' form) move when the
    records move by their FP32 error: sum over record fields f of
    |g(rec + deltas[:, f] e_f) - g(rec)|, one oracle pass per field (every
    Gaussian's field f moved at once).  From raw parameters the two sides'
    records differ by FP32 rounding of the projection, so a gradient compared
    end to end may differ by this much on top of the staged tolerance (large
    only for sums that cancel: a small footprint's dL/du is a difference of
    its left and right pixels)."""
    g0 = oracle.render_bwd(rec, pl, ranges, cam, G, tile_mask=tile_mask, margins=margins, flips=flips)
    out = np.zeros_like(g0)
    for f in range(9):
        if not np.any(deltas[:, f]):
            continue
        r2 = rec.copy()
        r2[:, f] += deltas[:, f]
        g1 = oracle.render_bwd(r2, pl, ranges, cam, G, tile_mask=tile_mask, margins=margins, flips=flips)
        out += np.abs(conic_to_sigma_grad(rec, g1 - g0))
    return out


def oracle_render_bwd_sigma(rec, pl, ranges, cam, G, tile_mask=None, flips=None, margins=STAGED_MARGINS):
    """Oracle record gradients in the HIP path's form (dL/dSigma' entries) and
    their term masses (per-pixel terms carried to Sigma' before the sum)."""
    g, mass, cmass = oracle.render_bwd(rec, pl, ranges, cam, G, tile_mask=tile_mask, with_mass=True,
                                       margins=margins, flips=flips)
    gs_ = conic_to_sigma_grad(rec, g)
    m = mass.copy()
    m[:, 2:5] = cmass
    return g, gs_, m


# ------------------------------------------------- forward comparison

_POPCOUNT8 = np.array([bin(i).count("1") for i in range(256)], np.int64)


def check_render(image, fT, nc, rec, pl, ranges, cam, margins=STAGED_MARGINS, tile_mask=None, pix_mask=None,
                 t_rtol=5e-4, max_ambiguous=1e-4):
    """Compare the HIP forward with the oracle's on every pixel of pix_mask.

    The oracle flags each decision whose FP64 value lies within `margins` of its
    threshold (alpha vs 1/255, T' vs 1e-4, o e^power vs 0.99).  A flagged pixel
    is not skipped: the oracle walks it once per combination of branches of its
    near decisions, and the HIP pixel must be one of those outcomes -- equal
    n_contrib, colour within PIX_ATOL and final_T within t_rtol relative.  The
    branches of one alpha or stop decision differ by at least 1/255 in T or by
    n_contrib, but two flips can compensate each other, so the matching
    outcome with the fewest flips, then the closest transmittance, identifies
    the branch the HIP path took; the oracle then uses that branch (flips) for
    this pixel.  A pixel whose
    outcomes cannot be told apart (a clamp at 0.99 changes T by about 1e-5) is
    ambiguous: its colour is checked, and its upstream gradient must be zeroed.
    Afterwards every pixel must match the oracle with the resolved branches:
    colour and final_T within PIX_ATOL, n_contrib exact.
    Returns (o_img, o_T, o_nc, flips, ambiguous, stats)."""
    H, W = cam.height, cam.width
    img = image.cpu().numpy().astype(np.float64)
    T = fT.cpu().numpy().astype(np.float64)
    n = nc.cpu().numpy()
    sel = np.ones((H, W), bool) if pix_mask is None else np.asarray(pix_mask, bool)
    _, _, _, fl, nn = oracle.render_fwd(rec, pl, ranges, cam, margins=margins, tile_mask=tile_mask, with_near=True)
    flips = np.zeros((H, W), np.uint8)
    amb = np.zeros((H, W), bool)
    flagged = (fl != 0) & sel
    pix = np.flatnonzero(flagged)
    stats = dict(pixels=int(sel.sum()), flagged=int(flagged.sum()), alpha=int(((fl & 1) != 0)[sel].sum()),
                 t_stop=int(((fl & 2) != 0)[sel].sum()), clamp=int(((fl & 4) != 0)[sel].sum()),
                 other_branch=0, ambiguous=0)
    if pix.size:
        bits = np.minimum(nn.flat[pix].astype(np.int64) + 2, 6)   # a flip may reveal later near decisions
        pp = np.repeat(pix, 1 << bits)
        mm = np.concatenate([np.arange(1 << b) for b in bits]).astype(np.uint8)
        out, bT, bnc, _, bnn = oracle.render_pixels(rec, pl, ranges, cam, pp, mm, margins=margins)
        valid = (mm.astype(np.int64) >> bnn.astype(np.int64)) == 0   # no bit beyond the decisions met
        gimg = img.reshape(3, -1)[:, pp].T
        terr = np.abs(T.flat[pp] - bT) / bT
        ok = valid & (bnc == n.flat[pp]) & (np.abs(gimg - out).max(axis=1) <= PIX_ATOL) & (terr <= t_rtol)
        start = 0
        for p, b in zip(pix, bits):
            cnt = 1 << int(b)
            okp, ep = ok[start:start + cnt], terr[start:start + cnt]
            start += cnt
            cand = np.flatnonzero(okp)
            assert cand.size, (f"pixel {divmod(int(p), W)[::-1]} matches no branch of its near decisions: "
                               f"HIP n_contrib {n.flat[p]}, T {T.flat[p]!r}")
            # fewest flipped decisions first (FP32 takes a decision the other
            # way only when it lies very close to its threshold; two flips can
            # compensate in T and colour), then the closest transmittance
            nflip = _POPCOUNT8[cand]
            fewest = cand[nflip == nflip.min()]
            best = fewest[np.argmin(ep[fewest])]
            rest = fewest[fewest != best]
            flips.flat[p] = best
            if rest.size and ep[rest].min() <= 4 * ep[best] + 1e-6:
                amb.flat[p] = True
        stats["other_branch"] = int(((flips != 0) & ~amb).sum())
        stats["ambiguous"] = int(amb.sum())
    assert stats["ambiguous"] <= max_ambiguous * max(stats["pixels"], 1), stats
    o_img, o_T, o_nc, _ = oracle.render_fwd(rec, pl, ranges, cam, margins=margins, tile_mask=tile_mask, flips=flips)
    err_img = np.abs(img - o_img).max(axis=0)
    assert (err_img[sel] <= PIX_ATOL).all(), f"max pixel err {err_img[sel].max()}"
    terr = np.abs(T - o_T)
    assert (terr[sel] <= PIX_ATOL).all(), f"max final_T err {terr[sel].max()}"
    mism = (n != o_nc) & sel
    assert not mism.any(), f"{mism.sum()} n_contrib mismatches after branch resolution"
    stats["max_err"] = float(err_img[sel].max()) if sel.any() else 0.0
    return o_img, o_T, o_nc, flips, amb, stats


def fmt_flags(st):
    return (f"flagged {st['flagged']} of {st['pixels']} px (alpha {st['alpha']}, T' stop {st['t_stop']}, "
            f"clamp {st['clamp']}); HIP took the other branch at {st['other_branch']}, ambiguous {st['ambiguous']}")

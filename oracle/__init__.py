"""FP64 CPU oracle for the differentiable tile-splatting step (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP path: the C library in
``gs_oracle.c`` is compiled with gcc, and this module only marshals NumPy
arrays into it.  Every input arrives as FP32 from the seeded generators and
is widened exactly to FP64 here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

TILE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no fast-math, no contraction of
    products and sums into fused multiply-adds, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_bin_count.restype = ctypes.c_int64
        _lib.or_tile_rect.restype = ctypes.c_int64
        _lib.or_tile_rect.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    return _lib


def _p(a):
    """Address of a NumPy array for a C call.  The caller must keep `a` referenced
    until the call returns: never pass a temporary."""
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def cam_array(cam) -> np.ndarray:
    """Flatten a camera into the oracle's double[22] layout (exact widening)."""
    return np.concatenate([
        np.array([cam.fx, cam.fy, cam.cx, cam.cy, cam.near_z, cam.tan_half_fov_x, cam.tan_half_fov_y],
                 np.float32).astype(np.float64),
        np.asarray(cam.R_cw, np.float32).astype(np.float64).reshape(9),
        np.asarray(cam.t_cw, np.float32).astype(np.float64).reshape(3),
        np.asarray(cam.bg, np.float32).astype(np.float64).reshape(3)])


def num_threads() -> int:
    return int(_load().or_num_threads())


def sh_basis(deg: int, d) -> tuple[np.ndarray, np.ndarray]:
    """Real SH basis Y_j(d) (j < (deg+1)^2) and its gradient dY_j/dd."""
    d = _d(d).reshape(3)
    nc = (deg + 1) ** 2
    Y = np.zeros(nc)
    G = np.zeros((nc, 3))
    _load().or_sh_basis(ctypes.c_int(deg), _p(d), _p(Y), _p(G))
    return Y, G


def tile_rect(u: float, v: float, r: int, W: int, H: int):
    rect = np.zeros(4, np.int32)
    cnt = _load().or_tile_rect(float(u), float(v), int(r), int(W), int(H), _p(rect))
    return int(cnt), rect


def project(scene, cam):
    """Per-Gaussian projection in FP64.  Returns dict with rec[n][9]
    (u, v, A, B, C, o, r, g, b), depth, radius, rect[n][4], tiles_touched, flags."""
    n = scene.n
    means, ls, q, lg, sh = (_d(scene.means), _d(scene.log_scales), _d(scene.quats),
                            _d(scene.logits), _d(scene.sh))
    rec = np.zeros((n, 9))
    depth = np.zeros(n)
    radius = np.zeros(n, np.int32)
    rect = np.zeros((n, 4), np.int32)
    tt = np.zeros(n, np.int64)
    flags = np.zeros(n, np.uint8)
    ca = cam_array(cam)
    rc = _load().or_project(ctypes.c_int64(n), ctypes.c_int(scene.sh_degree), _p(means), _p(ls), _p(q),
                            _p(lg), _p(sh), _p(ca), ctypes.c_int(cam.width), ctypes.c_int(cam.height),
                            _p(rec), _p(depth), _p(radius), _p(rect), _p(tt), _p(flags))
    if rc != 0:
        raise ValueError(f"or_project failed: {rc}")
    return dict(rec=rec, depth=depth, radius=radius, rect=rect, tiles_touched=tt, flags=flags)


def bin_rects(u, v, radius, W: int, H: int):
    """Each Gaussian's tile rectangle int32[n][4] = (x0, x1, y0, y1), inclusive
    (x1 < x0: no tile), the per-tile entry counts int64[T] and their total K."""
    u = _d(u); v = _d(v)
    radius = np.ascontiguousarray(radius, np.int32)
    n = u.shape[0]
    rect = np.zeros((n, 4), np.int32)
    counts = np.zeros(((W + TILE - 1) // TILE) * ((H + TILE - 1) // TILE), np.int64)
    K = _load().or_bin_rects(ctypes.c_int64(n), _p(u), _p(v), _p(radius), ctypes.c_int(W), ctypes.c_int(H),
                             _p(rect), _p(counts))
    return rect, counts, int(K)


def bin_sort(u, v, radius, depth_f32, W: int, H: int, tile_mask=None):
    """Tile binning and (tile, depth bits, index) sort on FP32-valued inputs.
    Returns (point_list uint32[K], ranges uint32[T][2], tiles_touched int64[n], offsets int64[n]).
    With tile_mask (uint8[T]) only the selected tiles get lists; the others get
    empty ranges and K counts the selected tiles' entries."""
    u = _d(u); v = _d(v)
    radius = np.ascontiguousarray(radius, np.int32)
    bits = np.ascontiguousarray(np.asarray(depth_f32, np.float32)).view(np.uint32)
    n = u.shape[0]
    tt = np.zeros(n, np.int64)
    off = np.zeros(n, np.int64)
    lib = _load()
    K = lib.or_bin_count(ctypes.c_int64(n), _p(u), _p(v), _p(radius), ctypes.c_int(W), ctypes.c_int(H),
                         _p(tt), _p(off))
    ntiles = ((W + TILE - 1) // TILE) * ((H + TILE - 1) // TILE)
    tm = None
    if tile_mask is not None:
        tm = np.ascontiguousarray(tile_mask, np.uint8)
        assert tm.shape == (ntiles,)
        _, counts, _ = bin_rects(u, v, radius, W, H)
        K = int(counts[tm != 0].sum())
    pl = np.zeros(max(K, 1), np.uint32)
    ranges = np.zeros((ntiles, 2), np.uint32)
    rc = lib.or_bin_sort(ctypes.c_int64(n), _p(u), _p(v), _p(radius), _p(bits), ctypes.c_int(W),
                         ctypes.c_int(H), _p(tm), ctypes.c_int64(K), _p(pl), _p(ranges))
    if rc != 0:
        raise RuntimeError(f"or_bin_sort failed: {rc}")
    return pl[:K], ranges, tt, off


# near-threshold margins of the per-pixel walk: alpha vs 1/255 (relative),
# T' vs 1e-4 (relative, base value; grows along the walk), o e^power vs 0.99,
# and the coefficient of the pair's power-term magnitude added to the two
# alpha margins (8 units of 2^-24: the FP32 evaluation error of the power)
POWER_ERR = 8.0 * 2.0 ** -24
MARGINS = (1e-5, 1e-4, 1e-5, POWER_ERR)


def _margins(m):
    """Four margins; a scalar or three values get no power-term margin."""
    m = np.asarray(m if m is not None else MARGINS, np.float64).reshape(-1)
    if m.size == 1:
        m = np.repeat(m, 3)
    if m.size == 3:
        m = np.append(m, 0.0)
    return np.ascontiguousarray(m[:4])


def render_fwd(rec, point_list, ranges, cam, margins=None, tile_mask=None, flips=None, with_near=False):
    """Front-to-back compositing per pixel.  Returns image[3][H][W], final_T[H][W],
    n_contrib[H][W] (int32) and per-pixel decision flags (bit0 alpha near 1/255,
    bit1 T' near 1e-4, bit2 o e^power near 0.99); with_near=True also the number
    of near decisions per pixel.  flips[H][W] (uint8) takes the other branch of
    the pixel's near decisions whose bits are set (walk order)."""
    W, H = cam.width, cam.height
    rec = _d(rec)
    pl = np.ascontiguousarray(point_list, np.uint32)
    rg = np.ascontiguousarray(ranges, np.uint32)
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    mg = _margins(margins)
    image = np.zeros((3, H, W))
    fT = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    fl = np.zeros((H, W), np.uint8)
    nn = np.zeros((H, W), np.uint8)
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, np.uint8)
    fp = None if flips is None else np.ascontiguousarray(flips, np.uint8)
    assert fp is None or fp.shape == (H, W)
    if not pl.size:
        pl = np.zeros(1, np.uint32)
    _load().or_render_fwd(ctypes.c_int(W), ctypes.c_int(H), _p(rec), _p(pl), _p(rg), _p(bg), _p(mg), _p(tm),
                          _p(fp), _p(image), _p(fT), _p(nc), _p(fl), _p(nn))
    return (image, fT, nc, fl, nn) if with_near else (image, fT, nc, fl)


def render_pixels(rec, point_list, ranges, cam, pix, flips, margins=None):
    """The per-pixel walk for (pixel, flips) pairs: pix int64[m] = y W + x,
    flips uint8[m].  Returns colour[m][3] (with background), final_T[m],
    n_contrib[m], flags[m] and near counts[m]."""
    W, H = cam.width, cam.height
    rec = _d(rec)
    pl = np.ascontiguousarray(point_list, np.uint32)
    rg = np.ascontiguousarray(ranges, np.uint32)
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    mg = _margins(margins)
    pix = np.ascontiguousarray(pix, np.int64)
    fp = np.ascontiguousarray(flips, np.uint8)
    m = pix.shape[0]
    assert fp.shape == (m,)
    out = np.zeros((m, 3))
    fT = np.zeros(m)
    nc = np.zeros(m, np.int32)
    fl = np.zeros(m, np.uint8)
    nn = np.zeros(m, np.uint8)
    if not pl.size:
        pl = np.zeros(1, np.uint32)
    rc = _load().or_render_pixels(ctypes.c_int(W), ctypes.c_int(H), _p(rec), _p(pl), _p(rg), _p(bg), _p(mg),
                                  ctypes.c_int64(m), _p(pix), _p(fp), _p(out), _p(fT), _p(nc), _p(fl), _p(nn))
    if rc != 0:
        raise ValueError(f"or_render_pixels failed: {rc}")
    return out, fT, nc, fl, nn


def render_bwd(rec, point_list, ranges, cam, dL_dimage, tile_mask=None, with_mass=False, margins=None, flips=None):
    """Gradient of sum(dL_dimage * image) w.r.t. the records: g2d[n][9] in
    record order (u, v, A, B, C, o, r, g, b), the conic entries as they enter
    the power (B once).  with_mass=True also returns the per-entry sum of
    |per-pixel terms| (mass[n][9]) and the same sum for the per-pixel conic
    gradient carried to the 2D covariance (cov_mass[n][3], (a, b, c)).
    flips as for render_fwd."""
    W, H = cam.width, cam.height
    rec = _d(rec)
    n = rec.shape[0]
    pl = np.ascontiguousarray(point_list, np.uint32)
    rg = np.ascontiguousarray(ranges, np.uint32)
    bg = np.asarray(cam.bg, np.float32).astype(np.float64)
    G = _d(dL_dimage)
    mg = _margins(margins)
    g2d = np.zeros((n, 9))
    mass = np.zeros((n, 9)) if with_mass else None
    cmass = np.zeros((n, 3)) if with_mass else None
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, np.uint8)
    fp = None if flips is None else np.ascontiguousarray(flips, np.uint8)
    assert fp is None or fp.shape == (H, W)
    if not pl.size:
        pl = np.zeros(1, np.uint32)
    _load().or_render_bwd(ctypes.c_int(W), ctypes.c_int(H), ctypes.c_int64(n), _p(rec),
                          _p(pl), _p(rg), _p(bg), _p(G), _p(tm), _p(mg), _p(fp), _p(g2d), _p(mass), _p(cmass))
    return (g2d, mass, cmass) if with_mass else g2d


def project_bwd(scene, cam, g2d):
    """Chain rule from record gradients g2d[n][9] (record order, conic entries as
    returned by render_bwd) to the raw parameters."""
    n = scene.n
    means, ls, q, lg, sh = (_d(scene.means), _d(scene.log_scales), _d(scene.quats),
                            _d(scene.logits), _d(scene.sh))
    g = dict(means=np.zeros_like(means), log_scales=np.zeros_like(ls), quats=np.zeros_like(q),
             logits=np.zeros_like(lg), sh=np.zeros_like(sh))
    ca = cam_array(cam)
    g2d = _d(g2d)
    if g2d.shape != (n, 9):
        raise ValueError(f"g2d must be [n][9], got {g2d.shape}")
    rc = _load().or_project_bwd(ctypes.c_int64(n), ctypes.c_int(scene.sh_degree), _p(means), _p(ls), _p(q),
                                _p(lg), _p(sh), _p(ca), _p(g2d), _p(g["means"]), _p(g["log_scales"]),
                                _p(g["quats"]), _p(g["logits"]), _p(g["sh"]))
    if rc != 0:
        raise ValueError(f"or_project_bwd failed: {rc}")
    return g


def forward(scene, cam, margins=None):
    """Whole forward in FP64: project -> bin/sort on the FP64 projection -> render.
    The sort key is the FP64 depth rounded to FP32 bits (the binning reading)."""
    pr = project(scene, cam)
    rec = pr["rec"]
    pl, ranges, tt, off = bin_sort(rec[:, 0], rec[:, 1], pr["radius"], pr["depth"].astype(np.float32),
                                   cam.width, cam.height)
    image, fT, nc, fl = render_fwd(rec, pl, ranges, cam, margins)
    return dict(proj=pr, point_list=pl, ranges=ranges, image=image, final_T=fT, n_contrib=nc, pix_flags=fl)


def backward(scene, cam, fwd, dL_dimage):
    """Whole backward in FP64 from dL/dimage to the raw parameters."""
    g2d = render_bwd(fwd["proj"]["rec"], fwd["point_list"], fwd["ranges"], cam, dL_dimage)
    grads = project_bwd(scene, cam, g2d)
    grads["g2d"] = g2d
    return grads


# ------------------------------------------------------------ learned colour

MLP_PARAMS = 6467
MLP_SLICES = {"W1": (0, (64, 32)), "b1": (2048, (64,)), "W2": (2112, (64, 64)), "b2": (6208, (64,)),
              "W3": (6272, (3, 64)), "b3": (6464, (3,))}


def mlp_inputs(z, dirs):
    """x[n*per][32] = [z_i; Y_0..15(d_ik)] for latents z[n][16] and unit directions dirs[n][per][3]."""
    z = _d(z)
    dirs = _d(dirs)
    n, per = dirs.shape[0], dirs.shape[1]
    x = np.zeros((n * per, 32))
    _load().or_mlp_inputs(ctypes.c_int64(n), ctypes.c_int(per), _p(z), _p(dirs), _p(x))
    return x


def mlp_fwd(x, params, with_hidden=False):
    """Decoder colours c[S][3] (and hidden activations) for inputs x[S][32]."""
    x = _d(x)
    P = _d(params)
    assert P.shape == (MLP_PARAMS,)
    S = x.shape[0]
    out = np.zeros((S, 3))
    h1 = np.zeros((S, 64)) if with_hidden else None
    h2 = np.zeros((S, 64)) if with_hidden else None
    _load().or_mlp_fwd(ctypes.c_int64(S), _p(x), _p(P), _p(out), _p(h1), _p(h2))
    return (out, h1, h2) if with_hidden else out


def mlp_bwd(x, params, dL_dc, with_dx=True):
    """(dL/dparams[6467], dL/dx[S][32]) of sum(dL_dc * c(x))."""
    x = _d(x)
    P = _d(params)
    G = _d(dL_dc)
    S = x.shape[0]
    dP = np.zeros(MLP_PARAMS)
    dx = np.zeros((S, 32)) if with_dx else None
    _load().or_mlp_bwd(ctypes.c_int64(S), _p(x), _p(P), _p(G), _p(dP), _p(dx))
    return dP, dx


def sh_colour(sh, deg, dirs):
    """SH colour max(0, sum Y f + 1/2) of every Gaussian at its directions dirs[n][per][3]."""
    sh = _d(sh)
    dirs = _d(dirs)
    n, per = dirs.shape[0], dirs.shape[1]
    out = np.zeros((n, per, 3))
    _load().or_sh_colour(ctypes.c_int64(n), ctypes.c_int(deg), _p(sh), _p(dirs), ctypes.c_int(per), _p(out))
    return out


# ------------------------------------------------------------ optimiser step

def adam_step(p, g, m, v, lr, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One bias-corrected Adam step in FP64 (Kingma & Ba, Algorithm 1), the
    optimiser of 3DGS training: returns the new (p, m, v).
      m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2
      p = p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
    lr may be an array broadcast against p (one rate per parameter group)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - np.asarray(lr, np.float64) * mh / (np.sqrt(vh) + eps), m, v


def densify_stats(g2d_views, visible_views):
    """Densification statistics over views: per Gaussian, the sum of
    |(dL/du, dL/dv)| over the views that see it and the number of those
    views.  g2d_views: record gradients [n][9] per view (u, v first);
    visible_views: bool [n] per view."""
    gsum = None
    cnt = None
    for g, vis in zip(g2d_views, visible_views):
        g = np.asarray(g, np.float64)
        vis = np.asarray(vis, bool)
        term = np.where(vis, np.hypot(g[:, 0], g[:, 1]), 0.0)
        gsum = term if gsum is None else gsum + term
        cnt = vis.astype(np.int64) if cnt is None else cnt + vis
    return gsum, cnt


# ------------------------------------------------- colour-hash sampling

CHS_BUCKETS = 4096


def colour_hash(rgb):
    """Bucket (Sec. IV-C.1) of each FP32 colour rgb[n][3]: 4-bit levels of the
    channels' 8-bit values, hashed as R_q 256 + G_q 16 + B_q.  uint16[n]."""
    rgb = np.ascontiguousarray(np.asarray(rgb, np.float32).reshape(-1, 3))
    n = rgb.shape[0]
    h = np.zeros(max(n, 1), np.uint16)
    _load().or_colour_hash(ctypes.c_int64(n), _p(rgb), _p(h))
    return h[:n]


def chs_aggregate(rec, point_list, ranges, hashes, window):
    """Per-entry records of the colour-hash sampling mode: dict with rec_e[K][9],
    rep[K] (list position of each entry's representative), size[K] (its
    group's size), tab_count[4096] and tab_sum[4096][4] (r, g, b, opacity)."""
    rec = _d(rec)
    pl = np.ascontiguousarray(point_list, np.uint32)
    rg = np.ascontiguousarray(ranges, np.uint32)
    hs = np.ascontiguousarray(hashes, np.uint16)
    K = pl.shape[0]
    rec_e = np.zeros((max(K, 1), 9))
    rep = np.zeros(max(K, 1), np.int64)
    size = np.zeros(max(K, 1), np.int32)
    tc = np.zeros(CHS_BUCKETS, np.uint32)
    ts = np.zeros((CHS_BUCKETS, 4))
    if not pl.size:
        pl = np.zeros(1, np.uint32)
    rc = _load().or_chs_aggregate(ctypes.c_int64(rg.shape[0]), _p(rg), _p(pl), _p(rec), _p(hs), ctypes.c_int(window),
                                  _p(rec_e), _p(rep), _p(size), _p(tc), _p(ts))
    if rc != 0:
        raise ValueError(f"or_chs_aggregate failed: {rc}")
    return dict(rec_e=rec_e[:K], rep=rep[:K], size=size[:K], tab_count=tc, tab_sum=ts)


def chs_render_fwd(rec, point_list, ranges, cam, hashes, window, margins=None, tile_mask=None, agg=None):
    """Forward compositing in the colour-hash sampling mode: the plain walk over
    the per-entry records of chs_aggregate (point list 0..K-1, same ranges).
    Returns (image, final_T, n_contrib, flags, agg); n_contrib counts list
    positions, as in the exact mode."""
    if agg is None:
        agg = chs_aggregate(rec, point_list, ranges, hashes, window)
    K = agg["rec_e"].shape[0]
    ident = np.arange(K, dtype=np.uint32)
    image, fT, nc, fl = render_fwd(agg["rec_e"], ident, ranges, cam, margins, tile_mask=tile_mask)
    return image, fT, nc, fl, agg


def chs_render_bwd(rec, point_list, ranges, cam, hashes, window, dL_dimage, tile_mask=None, agg=None,
                   margins=None):
    """Record gradients g2d[n][9] of sum(dL_dimage * image) in the colour-hash
    sampling mode: the backward of the walk over the per-entry records, then
    the chain rule of the aggregation (or_chs_route)."""
    rec = _d(rec)
    if agg is None:
        agg = chs_aggregate(rec, point_list, ranges, hashes, window)
    K = agg["rec_e"].shape[0]
    ident = np.arange(K, dtype=np.uint32)
    g_e = render_bwd(agg["rec_e"], ident, ranges, cam, dL_dimage, tile_mask=tile_mask, margins=margins)
    return chs_route(rec, point_list, ranges, window, agg, g_e)


def chs_route(rec, point_list, ranges, window, agg, g_e):
    """The aggregation's chain rule (or_chs_route): per-entry record gradients
    g_e[K][9] of the sampling mode's records -> per-Gaussian g2d[n][9]."""
    rec = _d(rec)
    K = agg["rec_e"].shape[0]
    n = rec.shape[0]
    g2d = np.zeros((n, 9))
    pl = np.ascontiguousarray(point_list, np.uint32)
    rg = np.ascontiguousarray(ranges, np.uint32)
    g_e = np.ascontiguousarray(_d(g_e))
    if not pl.size:
        pl = np.zeros(1, np.uint32)
        g_e = np.zeros((1, 9))
    rep = np.ascontiguousarray(agg["rep"]) if K else np.zeros(1, np.int64)
    size = np.ascontiguousarray(agg["size"]) if K else np.zeros(1, np.int32)
    rc = _load().or_chs_route(ctypes.c_int64(n), ctypes.c_int64(rg.shape[0]), _p(rg), _p(pl), _p(rec),
                              ctypes.c_int(window), _p(rep), _p(size), _p(g_e), _p(g2d))
    if rc != 0:
        raise ValueError(f"or_chs_route failed: {rc}")
    return g2d


# ---------------------------------------------------- density control (T1)

# (r, alpha, beta, k, a, delta, gamma): neighbour radius, threshold factors,
# k of the mean neighbour distance, spread factor (> 1), perturbation
# half-width, merge-radius factor
DENSITY_DEFAULTS = dict(alpha=1.0, beta=1.0, k=3, spread=1.5, jitter_frac=0.1, gamma=1.0)


def density_params(r, alpha=1.0, beta=1.0, k=3, spread=1.5, jitter=None, gamma=1.0):
    """Parameter vector of or_density_control (jitter defaults to r / 10)."""
    return np.array([r, alpha, beta, k, spread, 0.1 * r if jitter is None else jitter, gamma], np.float64)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def density(means, r, query=None):
    """rho of the queried points (all if None): other points within r (FP32 distance decision)."""
    m = _f32(means).reshape(3, -1)
    n = m.shape[1]
    q = np.arange(n, dtype=np.int64) if query is None else np.ascontiguousarray(query, np.int64)
    rho = np.zeros(max(len(q), 1), np.int32)
    _load().or_density(ctypes.c_int64(n), _p(m), ctypes.c_float(r), ctypes.c_int64(len(q)), _p(q), _p(rho))
    return rho[:len(q)]


def knn(means, k, query=None):
    """(idx[nq][k], d2[nq][k]): the k nearest other points by (FP32 d2, index)."""
    m = _f32(means).reshape(3, -1)
    n = m.shape[1]
    q = np.arange(n, dtype=np.int64) if query is None else np.ascontiguousarray(query, np.int64)
    idx = np.zeros((max(len(q), 1), k), np.int64)
    d2 = np.zeros((max(len(q), 1), k), np.float32)
    rc = _load().or_knn(ctypes.c_int64(n), _p(m), ctypes.c_int(k), ctypes.c_int64(len(q)), _p(q), _p(idx), _p(d2))
    if rc != 0:
        raise ValueError(f"or_knn failed: {rc}")
    return idx[:len(q)], d2[:len(q)]


def density_control(scene, prm, noise):
    """One round of density control (Sec. III-C) in the oracle.  prm from
    density_params, noise[6][n] (z rows then e rows).  Returns a dict with the
    new parameter arrays (FP64, n_out columns), per-point rho, cls (1 low,
    2 high), nn, dbar, fate (-1 removed, else output index) and the
    statistics."""
    n, deg = scene.n, scene.sh_degree
    nc = (deg + 1) ** 2
    cap = max(2 * n, 1)
    arrs = [_f32(a) for a in (scene.means, scene.log_scales, scene.quats, scene.logits, scene.sh)]
    nz = _f32(noise).reshape(6, n)
    out = dict(means=np.zeros((3, cap)), log_scales=np.zeros((3, cap)), quats=np.zeros((4, cap)),
               logits=np.zeros(cap), sh=np.zeros((nc, 3, cap)))
    rho = np.zeros(max(n, 1), np.int32)
    cls = np.zeros(max(n, 1), np.int8)
    nn = np.zeros(max(n, 1), np.int64)
    dbar = np.zeros(max(n, 1), np.float32)
    fate = np.zeros(max(n, 1), np.int64)
    stats = np.zeros(8)
    prm = np.ascontiguousarray(prm, np.float64)
    _load().or_density_control(ctypes.c_int64(n), ctypes.c_int(deg), *(_p(a) for a in arrs), _p(prm), _p(nz),
                               _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]), _p(out["logits"]),
                               _p(out["sh"]), _p(rho), _p(cls), _p(nn), _p(dbar), _p(fate), _p(stats))
    n_out = int(stats[7])
    res = {k: v[..., :n_out] for k, v in out.items()}
    res.update(rho=rho[:n], cls=cls[:n], nn=nn[:n], dbar=dbar[:n], fate=fate[:n], n_out=n_out,
               stats=dict(zip(("mu", "sigma", "rho_low", "rho_high", "mu_d", "sigma_d", "d_merge"), stats[:7])))
    return res

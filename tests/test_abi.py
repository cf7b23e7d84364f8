"""C ABI checks that need no GPU: the library loads, exports every symbol that
include/gsplat.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_14564_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gs():
    from paper_2510_14564_amd import gs as mod
    return mod


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "gsplat.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gs_\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported(gs):
    decl = _declared_symbols()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(gs._lib, name), name
    assert set(decl) == set(gs.EXPORTS)


def test_version_and_empty_error(gs):
    assert "gfx950" in gs.version()
    # every entry point clears the error message first (an earlier test in
    # the same process may have left one)
    assert gs.mlp_bwd_workspace(16, 1) > 0
    assert gs.last_error() == ""


def _cam(gs, **over):
    c = gs.camera_struct(scenes.config_camera(1))
    for k, v in over.items():
        setattr(c, k, v)
    return c


def _gauss(gs, n=10, deg=0, mode=0, null=False):
    g = gs.Gaussians()
    g.n, g.sh_degree, g.colour_mode = n, deg, mode
    p = None if null else ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    g.means = g.log_scales = g.quats = g.logits = g.sh = p
    return g


def _proj(gs):
    p = gs.Projected()
    p.records = p.depth = p.radius = p.tiles_touched = ctypes.c_void_p(0x1000)
    return p


NULL = ctypes.c_void_p(0)


@pytest.mark.parametrize("case", ["neg_n", "deg4", "mode7", "null_arrays", "cam_w0", "cam_nan", "cam_fx0"])
def test_project_rejects_bad_arguments(gs, case):
    g, c = _gauss(gs), _cam(gs)
    if case == "neg_n":
        g.n = -1
    elif case == "deg4":
        g.sh_degree = 4
    elif case == "mode7":
        g.colour_mode = 7
    elif case == "null_arrays":
        g = _gauss(gs, null=True)
    elif case == "cam_w0":
        c.width = 0
    elif case == "cam_nan":
        c.fx = float("nan")
    elif case == "cam_fx0":
        c.fx = 0.0
    st = gs._lib.gs_project(ctypes.byref(g), ctypes.byref(c), ctypes.byref(_proj(gs)), NULL)
    assert st == gs.GS_ERR_INVALID_ARG
    assert gs.last_error() != ""


def test_null_descriptors_rejected(gs):
    c = _cam(gs)
    assert gs._lib.gs_project(None, ctypes.byref(c), ctypes.byref(_proj(gs)), NULL) == gs.GS_ERR_INVALID_ARG
    assert gs._lib.gs_project(ctypes.byref(_gauss(gs)), None, ctypes.byref(_proj(gs)), NULL) == gs.GS_ERR_INVALID_ARG


def test_workspace_queries_are_host_only(gs):
    c = _cam(gs)
    b = ctypes.c_size_t(0)
    assert gs._lib.gs_bin_sort_workspace(4096, 20000, ctypes.byref(c), ctypes.byref(b)) == gs.GS_OK
    assert b.value > 4 * 20000
    b2 = ctypes.c_size_t(0)
    assert gs._lib.gs_bin_sort_workspace(4096, 40000, ctypes.byref(c), ctypes.byref(b2)) == gs.GS_OK
    assert b2.value > b.value
    assert gs._lib.gs_bin_sort_workspace(-1, 0, ctypes.byref(c), ctypes.byref(b)) == gs.GS_ERR_INVALID_ARG
    assert gs._lib.gs_render_bwd_2d_workspace(10, 10, ctypes.byref(c), 0, ctypes.byref(b)) == gs.GS_OK
    # the deterministic reduction holds a 36-byte row per entry
    d1, d2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert gs._lib.gs_render_bwd_2d_workspace(1000, 100000, ctypes.byref(c), 1, ctypes.byref(d1)) == gs.GS_OK
    assert gs._lib.gs_render_bwd_2d_workspace(1000, 200000, ctypes.byref(c), 1, ctypes.byref(d2)) == gs.GS_OK
    assert d2.value - d1.value >= 36 * 100000
    assert gs._lib.gs_render_bwd_2d_workspace(1000, 100000, ctypes.byref(c), 0, ctypes.byref(b)) == gs.GS_OK
    assert d1.value > b.value
    # the full backward: the 2D workspace, plus the record gradients g2d[9][n]
    # where the projection cannot read the accumulator rows (deterministic
    # mode, learned colour), plus the decoder backward's workspace
    for det, mode in ((0, 0), (1, 0), (0, 1)):
        f = ctypes.c_size_t(0)
        g = _gauss(gs, n=1000, deg=3, mode=mode)
        g.latents = g.mlp = ctypes.c_void_p(0x1000)
        assert gs._lib.gs_render_bwd_workspace(ctypes.byref(g), 100000, ctypes.byref(c), det, ctypes.byref(f)) == \
            gs.GS_OK
        two_d = d1.value if det else b.value
        assert f.value >= two_d + (0 if (det, mode) == (0, 0) else 36 * 1000), (det, mode)
    bad = _gauss(gs, n=1000, deg=5)
    assert gs._lib.gs_render_bwd_workspace(ctypes.byref(bad), 10, ctypes.byref(c), 0, ctypes.byref(b)) == \
        gs.GS_ERR_INVALID_ARG


def test_bin_sort_rejects_small_workspace_and_bad_alignment(gs):
    c = _cam(gs)
    k = ctypes.c_int64(0)
    st = gs._lib.gs_bin_sort(10, ctypes.byref(_proj(gs)), ctypes.byref(c), ctypes.c_void_p(0x1000), 16,
                             ctypes.c_void_p(0x1000), 100, ctypes.c_void_p(0x1000), ctypes.byref(k), NULL)
    assert st == gs.GS_ERR_INVALID_ARG
    st = gs._lib.gs_bin_sort(10, ctypes.byref(_proj(gs)), ctypes.byref(c), ctypes.c_void_p(0x1004), 1 << 30,
                             ctypes.c_void_p(0x1000), 100, ctypes.c_void_p(0x1000), ctypes.byref(k), NULL)
    assert st == gs.GS_ERR_INVALID_ARG


def test_render_calls_reject_nulls(gs):
    c = _cam(gs)
    st = gs._lib.gs_render_fwd(10, ctypes.byref(_proj(gs)), NULL, NULL, 5, ctypes.byref(c), NULL, NULL, NULL, NULL,
                               0, NULL)
    assert st == gs.GS_ERR_INVALID_ARG
    st = gs._lib.gs_render_bwd_2d(10, ctypes.byref(_proj(gs)), NULL, NULL, 5, ctypes.byref(c), NULL, NULL, NULL,
                                  NULL, NULL, NULL, 0, 0, 0, NULL)
    assert st == gs.GS_ERR_INVALID_ARG
    p = ctypes.c_void_p(0x1000)
    gr = gs.GaussiansGrad()
    gr.means = gr.log_scales = gr.quats = gr.logits = gr.sh = p
    g = _gauss(gs)
    ws = ctypes.c_void_p(0x100000)

    def full(grad, stats=None, ws_bytes=1 << 40, sched=1, ranges=p, wsp=ws):
        return gs._lib.gs_render_bwd(ctypes.byref(g), ctypes.byref(c), ctypes.byref(_proj(gs)), p, ranges, 5, p, p,
                                     p, p, ctypes.byref(grad), stats, wsp, ws_bytes, 0, sched, NULL)
    assert full(gr, ranges=NULL) == gs.GS_ERR_INVALID_ARG
    nog = gs.GaussiansGrad()
    nog.means = nog.log_scales = nog.quats = nog.logits = p
    assert full(nog) == gs.GS_ERR_INVALID_ARG and "gradient" in gs.last_error()       # sh gradient missing
    half = gs.DensifyStats()
    half.grad_norm_sum = p
    assert full(gr, stats=ctypes.byref(half)) == gs.GS_ERR_INVALID_ARG and "statistics" in gs.last_error()
    assert full(gr, ws_bytes=16) == gs.GS_ERR_INVALID_ARG and "workspace" in gs.last_error()
    assert full(gr, wsp=ctypes.c_void_p(0x100010)) == gs.GS_ERR_INVALID_ARG and "aligned" in gs.last_error()
    assert full(gr, sched=5) == gs.GS_ERR_INVALID_ARG and "schedule" in gs.last_error()
    # an unknown schedule, and the balanced schedule without its plan storage
    p = ctypes.c_void_p(0x1000)
    for sched, ck in ((3, p), (-1, p), (gs.SCHEDULE_BALANCED, NULL), (gs.SCHEDULE_MERGED, NULL)):
        st = gs._lib.gs_render_fwd(10, ctypes.byref(_proj(gs)), p, p, 5, ctypes.byref(c), p, p, p, ck, sched, NULL)
        assert st == gs.GS_ERR_INVALID_ARG, sched
        assert "schedule" in gs.last_error()
    assert gs._lib.gs_l1_loss(NULL, NULL, 0, NULL, NULL, NULL, NULL) == gs.GS_ERR_INVALID_ARG


def test_adam_gaussians_argument_checks(gs):
    """The fused Gaussian Adam step rejects bad hyper-parameters and missing
    arrays before any device work."""
    p = ctypes.c_void_p(0x1000)
    arr = gs.ParamArrays()
    arr.means = arr.log_scales = arr.quats = arr.logits = arr.sh = p
    gr = gs.GaussiansGrad()
    gr.means = gr.log_scales = gr.quats = gr.logits = gr.sh = p

    def call(cfg, n=10, deg=3, params=arr, grad=gr):
        return gs._lib.gs_adam_gaussians(n, deg, ctypes.byref(params), ctypes.byref(grad), ctypes.byref(arr),
                                         ctypes.byref(arr), ctypes.byref(cfg), NULL)

    def cfg(**over):
        c = gs.AdamConfig()
        c.lr_means = c.lr_log_scales = c.lr_quats = c.lr_logits = c.lr_sh_dc = c.lr_sh_rest = 1e-3
        c.beta1, c.beta2, c.eps, c.step = 0.9, 0.999, 1e-15, 1
        for k, v in over.items():
            setattr(c, k, v)
        return c
    for bad in (dict(step=0), dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0), dict(lr_quats=float("inf"))):
        assert call(cfg(**bad)) == gs.GS_ERR_INVALID_ARG, bad
    assert call(cfg(), deg=4) == gs.GS_ERR_INVALID_ARG
    assert call(cfg(), n=-1) == gs.GS_ERR_INVALID_ARG
    holey = gs.ParamArrays()
    holey.means = holey.log_scales = holey.quats = holey.logits = p
    assert call(cfg(), params=holey) == gs.GS_ERR_INVALID_ARG
    assert call(cfg(), n=0) == gs.GS_OK            # nothing to do, no device work


def test_camera_struct_layout_matches_header(gs):
    # int32 x2 + float x7 + R[9] + t[3] + bg[3] = 2*4 + 22*4 bytes
    assert ctypes.sizeof(gs.Camera) == 8 + 22 * 4
    assert ctypes.sizeof(gs.Gaussians) == 8 + 4 + 4 + 7 * 8


def test_bin_sort_async_argument_checks(gs):
    """Host-side rejections of the no-wait bin/sort: a NULL K buffer, a small
    workspace, and a frame whose per-chunk tables exceed LDS (2400 x 1000 px,
    150 x 63 tiles), which must use gs_bin_sort -- all before device work."""
    c = _cam(gs)
    fake = ctypes.c_void_p(0x1000)
    st = gs._lib.gs_bin_sort_async(10, ctypes.byref(_proj(gs)), ctypes.byref(c), fake, 1 << 30, fake, 100, fake,
                                   NULL, NULL)
    assert st == gs.GS_ERR_INVALID_ARG
    st = gs._lib.gs_bin_sort_async(10, ctypes.byref(_proj(gs)), ctypes.byref(c), fake, 16, fake, 100, fake, fake,
                                   NULL)
    assert st == gs.GS_ERR_INVALID_ARG
    wide = gs.camera_struct(scenes.pinhole(4800, 1000, 70.0, np.eye(3), (0.0, 0.0, 3.0)))   # 18,900 tiles
    st = gs._lib.gs_bin_sort_async(10, ctypes.byref(_proj(gs)), ctypes.byref(wide), fake, 1 << 40, fake, 100, fake,
                                   fake, NULL)
    assert st == gs.GS_ERR_UNSUPPORTED
    assert "gs_bin_sort" in gs.last_error()


@pytest.mark.parametrize("case", ["r0", "r_nan", "k0", "k9", "alpha_neg", "jitter_neg", "null_noise", "null_out",
                                  "small_ws", "mode1"])
def test_density_control_rejects_bad_arguments(gs, case):
    g = _gauss(gs, n=100, deg=1)
    prm = gs.DensityParams(0.05, 1.0, 1.0, 3, 1.5, 0.005, 1.0)
    out = gs.ParamArrays()
    out.means = out.log_scales = out.quats = out.logits = out.sh = ctypes.c_void_p(0x1000)
    noise = ctypes.c_void_p(0x1000)
    need = gs.density_control_workspace(100)
    ws, nbytes = ctypes.c_void_p(0x100000), need
    if case == "r0":
        prm.radius = 0.0
    elif case == "r_nan":
        prm.radius = float("nan")
    elif case == "k0":
        prm.knn = 0
    elif case == "k9":
        prm.knn = 9
    elif case == "alpha_neg":
        prm.alpha = -1.0
    elif case == "jitter_neg":
        prm.jitter = -0.1
    elif case == "null_noise":
        noise = None
    elif case == "null_out":
        out.sh = None
    elif case == "small_ws":
        nbytes = need - 1
    elif case == "mode1":
        g.colour_mode = 1
        g.latents = g.mlp = ctypes.c_void_p(0x1000)
    rep = gs.DensityReport()
    st = gs._lib.gs_density_control(ctypes.byref(g), ctypes.byref(prm), noise, ctypes.byref(out), 200, ws, nbytes,
                                    ctypes.byref(rep), None, NULL)
    assert st == gs.GS_ERR_INVALID_ARG, case
    assert gs.last_error() != ""


def test_density_control_workspace_grows_with_n(gs):
    a, b = gs.density_control_workspace(1000), gs.density_control_workspace(100000)
    assert b > a > 0 and b - a >= 60 * 99000

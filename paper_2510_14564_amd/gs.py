"""ctypes binding of libgsplat.so (include/gsplat.h).

Argument marshalling only: every step runs in the HIP kernels behind the C ABI.
Tensors are PyTorch device tensors (ROCm); PyTorch provides device memory and
the current HIP stream.  Importing this module loads the library and raises
if it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsplat.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_14564_amd.build` "
                      "(or __graft_entry__.build()) before using the HIP path")

_lib = ctypes.CDLL(LIB_PATH)

TILE = 16
REC_FLOATS = 12
G2D = 9
L1_PARTIALS = 1024
MLP_PARAMS = 6467
MLP_PACKED_BYTES = 31244

SCHEDULE_PLAIN, SCHEDULE_BALANCED, SCHEDULE_MERGED = 0, 1, 2
# or-ed into a compositing call's schedule: the approximate colour-hash sampling mode
RENDER_COLOUR_HASH = 0x100
COLOUR_BUCKETS = 4096
GS_OK, GS_ERR_INVALID_ARG, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
STATUS_NAMES = {0: "GS_OK", -1: "GS_ERR_INVALID_ARG", -2: "GS_ERR_CAPACITY", -3: "GS_ERR_HIP",
                -4: "GS_ERR_UNSUPPORTED"}

# every symbol declared in include/gsplat.h
EXPORTS = ("gs_last_error", "gs_version", "gs_project", "gs_bin_sort_workspace", "gs_bin_sort", "gs_bin_sort_async",
           "gs_render_fwd", "gs_render_count", "gs_colour_hash_table", "gs_render_ckpt_floats", "gs_render_bwd_workspace", "gs_render_bwd",
           "gs_render_bwd_2d_workspace", "gs_render_bwd_2d", "gs_project_bwd", "gs_project_bwd_workspace",
           "gs_adam_gaussians", "gs_density_control_workspace", "gs_density_control", "gs_l1_loss", "gs_l1_loss_static", "gs_mlp_pack", "gs_mlp_fwd", "gs_mlp_bwd_workspace", "gs_mlp_bwd",
           "gs_sh_colour", "gs_adam_step", "gs_kernel_timer_start", "gs_kernel_timer_stop")


class DensityParams(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("alpha", ctypes.c_float), ("beta", ctypes.c_float),
                ("knn", ctypes.c_int32), ("spread", ctypes.c_float), ("jitter", ctypes.c_float),
                ("gamma", ctypes.c_float)]


class DensityReport(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int64), ("n_merged", ctypes.c_int64), ("n_new", ctypes.c_int64),
                ("n_out", ctypes.c_int64), ("rho_mean", ctypes.c_double), ("rho_std", ctypes.c_double),
                ("rho_low", ctypes.c_double), ("rho_high", ctypes.c_double), ("d_mean", ctypes.c_double),
                ("d_std", ctypes.c_double), ("d_merge", ctypes.c_double)]


class DensityPoints(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("cls", ctypes.c_void_p), ("nn", ctypes.c_void_p),
                ("dbar", ctypes.c_void_p), ("fate", ctypes.c_void_p)]


class GsError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("near_z", ctypes.c_float), ("tan_half_fov_x", ctypes.c_float), ("tan_half_fov_y", ctypes.c_float),
                ("R_cw", ctypes.c_float * 9), ("t_cw", ctypes.c_float * 3), ("bg", ctypes.c_float * 3)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("colour_mode", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("logits", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("latents", ctypes.c_void_p),
                ("mlp", ctypes.c_void_p)]


class Projected(ctypes.Structure):
    _fields_ = [("records", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("radius", ctypes.c_void_p),
                ("tiles_touched", ctypes.c_void_p), ("colour_grad", ctypes.c_void_p)]


class GaussiansGrad(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("logits", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("latents", ctypes.c_void_p),
                ("mlp", ctypes.c_void_p)]


class DensifyStats(ctypes.Structure):
    _fields_ = [("grad_norm_sum", ctypes.c_void_p), ("visible_count", ctypes.c_void_p)]


class ParamArrays(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("logits", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class AdamConfig(ctypes.Structure):
    _fields_ = [("lr_means", ctypes.c_float), ("lr_log_scales", ctypes.c_float), ("lr_quats", ctypes.c_float),
                ("lr_logits", ctypes.c_float), ("lr_sh_dc", ctypes.c_float), ("lr_sh_rest", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step", ctypes.c_int32)]


_vp, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_P = ctypes.POINTER
_sigs = {
    "gs_last_error": ([], ctypes.c_char_p),
    "gs_version": ([], ctypes.c_char_p),
    "gs_project": ([_P(Gaussians), _P(Camera), _P(Projected), _vp], ctypes.c_int),
    "gs_bin_sort_workspace": ([_i64, _i64, _P(Camera), _P(_sz)], ctypes.c_int),
    "gs_bin_sort": ([_i64, _P(Projected), _P(Camera), _vp, _sz, _vp, _i64, _vp, _P(_i64), _vp], ctypes.c_int),
    "gs_bin_sort_async": ([_i64, _P(Projected), _P(Camera), _vp, _sz, _vp, _i64, _vp, _vp, _vp], ctypes.c_int),
    "gs_render_fwd": ([_i64, _P(Projected), _vp, _vp, _i64, _P(Camera), _vp, _vp, _vp, _vp, _i32, _vp],
                      ctypes.c_int),
    "gs_render_ckpt_floats": ([_i64, _P(Camera), _P(_sz)], ctypes.c_int),
    "gs_render_count": ([_i64, _P(Projected), _vp, _vp, _i64, _P(Camera), _vp, _vp], ctypes.c_int),
    "gs_colour_hash_table": ([_i64, _P(Projected), _vp, _vp, _i64, _P(Camera), _vp, _vp, _vp, _vp, _vp],
                             ctypes.c_int),
    "gs_render_bwd_workspace": ([_P(Gaussians), _i64, _P(Camera), _i32, _P(_sz)], ctypes.c_int),
    "gs_render_bwd": ([_P(Gaussians), _P(Camera), _P(Projected), _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                       _P(GaussiansGrad), _P(DensifyStats), _vp, _sz, _i32, _i32, _vp], ctypes.c_int),
    "gs_render_bwd_2d_workspace": ([_i64, _i64, _P(Camera), _i32, _P(_sz)], ctypes.c_int),
    "gs_render_bwd_2d": ([_i64, _P(Projected), _vp, _vp, _i64, _P(Camera), _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32,
                          _i32, _vp], ctypes.c_int),
    "gs_kernel_timer_start": ([], ctypes.c_int),
    "gs_kernel_timer_stop": ([ctypes.c_char_p, _sz, _P(_sz)], ctypes.c_int),
    "gs_adam_gaussians": ([_i64, _i32, _P(ParamArrays), _P(GaussiansGrad), _P(ParamArrays), _P(ParamArrays),
                           _P(AdamConfig), _vp], ctypes.c_int),
    "gs_project_bwd_workspace": ([_P(Gaussians), _P(_sz)], ctypes.c_int),
    "gs_density_control_workspace": ([_i64, _P(_sz)], ctypes.c_int),
    "gs_density_control": ([_P(Gaussians), _P(DensityParams), _vp, _P(ParamArrays), _i64, _vp, _sz,
                            _P(DensityReport), _P(DensityPoints), _vp], ctypes.c_int),
    "gs_project_bwd": ([_P(Gaussians), _P(Camera), _P(Projected), _vp, _P(GaussiansGrad), _vp, _sz, _vp],
                       ctypes.c_int),
    "gs_l1_loss": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "gs_l1_loss_static": ([_vp, _vp, _i64, _vp, _vp, _vp], ctypes.c_int),
    "gs_mlp_pack": ([_vp, _vp, _vp], ctypes.c_int),
    "gs_mlp_fwd": ([_i64, _i32, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "gs_mlp_bwd_workspace": ([_i64, _i32, _P(_sz)], ctypes.c_int),
    "gs_mlp_bwd": ([_i64, _i32, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, _vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
    "gs_sh_colour": ([_i64, _i32, _i64, _i32, _vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "gs_adam_step": ([_i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      _i32, _vp], ctypes.c_int),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def version() -> str:
    return _lib.gs_version().decode()


def last_error() -> str:
    return _lib.gs_last_error().decode()


def _check(status: int, fn: str):
    if status != GS_OK:
        raise GsError(status, fn, last_error())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def camera_struct(cam) -> Camera:
    """ctypes camera from a scenes.Camera (or any object with the same fields)."""
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.near_z = float(cam.near_z)
    c.tan_half_fov_x, c.tan_half_fov_y = float(cam.tan_half_fov_x), float(cam.tan_half_fov_y)
    for i, v in enumerate(list(map(float, cam.R_cw.reshape(9)))):
        c.R_cw[i] = v
    for i in range(3):
        c.t_cw[i] = float(cam.t_cw[i])
        c.bg[i] = float(cam.bg[i])
    return c


def n_tiles(cam) -> int:
    return ((cam.width + TILE - 1) // TILE) * ((cam.height + TILE - 1) // TILE)


def _check_f32(name, t, shape=None):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")


def gaussians_struct(means, log_scales, quats, logits, sh, sh_degree: int) -> Gaussians:
    n = means.shape[1]
    _check_f32("means", means, (3, n))
    _check_f32("log_scales", log_scales, (3, n))
    _check_f32("quats", quats, (4, n))
    _check_f32("logits", logits, (n,))
    _check_f32("sh", sh, ((sh_degree + 1) ** 2, 3, n))
    g = Gaussians()
    g.n, g.sh_degree, g.colour_mode = n, sh_degree, 0
    g.means, g.log_scales, g.quats, g.logits, g.sh = (_ptr(means), _ptr(log_scales), _ptr(quats),
                                                      _ptr(logits), _ptr(sh))
    return g


class ProjectedBuffers:
    """Device buffers written by gs_project."""

    def __init__(self, n: int, device, colour_grad: bool = True):
        self.n = n
        self.records = torch.empty((n, REC_FLOATS), dtype=torch.float32, device=device)
        self.depth = torch.empty(n, dtype=torch.float32, device=device)
        self.radius = torch.empty(n, dtype=torch.int32, device=device)
        self.tiles_touched = torch.empty(n, dtype=torch.int32, device=device)
        # d colour / d direction and the clamp mask for the backward (SH colour)
        self.colour_grad = torch.empty((10, n), dtype=torch.float32, device=device) if colour_grad else None

    def struct(self) -> Projected:
        p = Projected()
        p.records, p.depth, p.radius, p.tiles_touched = (_ptr(self.records), _ptr(self.depth), _ptr(self.radius),
                                                         _ptr(self.tiles_touched))
        p.colour_grad = _ptr(self.colour_grad)
        return p


# ------------------------------------------------------------------ entry points

def project(gauss: Gaussians, cam: Camera, out: ProjectedBuffers, stream=None):
    _check(_lib.gs_project(ctypes.byref(gauss), ctypes.byref(cam), ctypes.byref(out.struct()), _stream(stream)),
           "gs_project")


def bin_sort_workspace(n: int, capacity: int, cam: Camera) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.gs_bin_sort_workspace(n, capacity, ctypes.byref(cam), ctypes.byref(b)), "gs_bin_sort_workspace")
    return int(b.value)


def bin_sort(n: int, proj: ProjectedBuffers, cam: Camera, ws, point_list, ranges, stream=None) -> int:
    """Returns K; raises GsError(GS_ERR_CAPACITY) with .required = K if point_list is too small."""
    k = ctypes.c_int64(0)
    st = _lib.gs_bin_sort(n, ctypes.byref(proj.struct()), ctypes.byref(cam), _ptr(ws), ws.numel() * ws.element_size(),
                          _ptr(point_list), point_list.numel(), _ptr(ranges), ctypes.byref(k), _stream(stream))
    if st == GS_ERR_CAPACITY:
        e = GsError(st, "gs_bin_sort", last_error())
        e.required = int(k.value)
        raise e
    _check(st, "gs_bin_sort")
    return int(k.value)


def bin_sort_async(n: int, proj: ProjectedBuffers, cam: Camera, ws, point_list, ranges, k_dev, stream=None):
    """bin_sort without the host wait: K and the look-back flag go to k_dev
    (int64[2]: a device tensor, or a pinned host tensor, which the kernels
    write directly so that no copy is queued); the lists are valid only if
    k_dev[0] <= point_list.numel() and k_dev[1] == 0."""
    assert k_dev.dtype == torch.int64 and k_dev.numel() >= 2 and (k_dev.is_cuda or k_dev.is_pinned())
    _check(_lib.gs_bin_sort_async(n, ctypes.byref(proj.struct()), ctypes.byref(cam), _ptr(ws),
                                  ws.numel() * ws.element_size(), _ptr(point_list), point_list.numel(), _ptr(ranges),
                                  _ptr(k_dev), _stream(stream)), "gs_bin_sort_async")


def render_fwd(n: int, proj: ProjectedBuffers, point_list, ranges, k: int, cam: Camera, image, final_T, n_contrib,
               t_ckpt=None, schedule=None, stream=None):
    """schedule: SCHEDULE_BALANCED when t_ckpt is given, else SCHEDULE_PLAIN, unless set."""
    if schedule is None:
        schedule = SCHEDULE_BALANCED if t_ckpt is not None else SCHEDULE_PLAIN
    _check(_lib.gs_render_fwd(n, ctypes.byref(proj.struct()), _ptr(point_list), _ptr(ranges), k, ctypes.byref(cam),
                              _ptr(image), _ptr(final_T), _ptr(n_contrib), _ptr(t_ckpt), int(schedule),
                              _stream(stream)), "gs_render_fwd")


def render_count(n: int, proj: ProjectedBuffers, point_list, ranges, k: int, cam: Camera, counts, stream=None):
    """counts: device int64[2] <- (pairs examined, pairs blended) of the forward."""
    _check(_lib.gs_render_count(n, ctypes.byref(proj.struct()), _ptr(point_list), _ptr(ranges), k, ctypes.byref(cam),
                                _ptr(counts), _stream(stream)), "gs_render_count")


def colour_hash_table(n: int, proj: ProjectedBuffers, point_list, ranges, k: int, cam: Camera, count=None, sums=None,
                      bucket=None, rep=None, stream=None):
    """Colour-hash sampling statistics of a binned frame: count uint32[4096],
    sums float[4096][4] (r, g, b, opacity), bucket uint16[k] and rep uint32[k]
    (device tensors, each optional, overwritten)."""
    _check(_lib.gs_colour_hash_table(n, ctypes.byref(proj.struct()), _ptr(point_list), _ptr(ranges), k,
                                     ctypes.byref(cam), _ptr(count), _ptr(sums), _ptr(bucket), _ptr(rep),
                                     _stream(stream)), "gs_colour_hash_table")


def render_ckpt_floats(k: int, cam: Camera) -> int:
    f = ctypes.c_size_t(0)
    _check(_lib.gs_render_ckpt_floats(k, ctypes.byref(cam), ctypes.byref(f)), "gs_render_ckpt_floats")
    return int(f.value)


def render_bwd_2d_workspace(n: int, k: int, cam: Camera, deterministic: bool) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.gs_render_bwd_2d_workspace(n, k, ctypes.byref(cam), int(deterministic), ctypes.byref(b)),
           "gs_render_bwd_2d_workspace")
    return int(b.value)


def render_bwd_2d(n: int, proj: ProjectedBuffers, point_list, ranges, k: int, cam: Camera, final_T, n_contrib, t_ckpt,
                  dL_dimage, g2d, ws, deterministic: bool = False, schedule=SCHEDULE_BALANCED, stream=None):
    """Compositing backward only: record gradients g2d[9][n] (Sigma' form)."""
    _check(_lib.gs_render_bwd_2d(n, ctypes.byref(proj.struct()), _ptr(point_list), _ptr(ranges), k,
                                 ctypes.byref(cam), _ptr(final_T), _ptr(n_contrib), _ptr(t_ckpt), _ptr(dL_dimage),
                                 _ptr(g2d), _ptr(ws), ws.numel() * ws.element_size(), int(deterministic),
                                 int(schedule), _stream(stream)), "gs_render_bwd_2d")


def render_bwd_workspace(gauss: Gaussians, k: int, cam: Camera, deterministic: bool) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.gs_render_bwd_workspace(ctypes.byref(gauss), k, ctypes.byref(cam), int(deterministic),
                                        ctypes.byref(b)), "gs_render_bwd_workspace")
    return int(b.value)


def _grad_struct(grads: dict) -> GaussiansGrad:
    gg = GaussiansGrad()
    gg.means, gg.log_scales, gg.quats, gg.logits = (_ptr(grads["means"]), _ptr(grads["log_scales"]),
                                                    _ptr(grads["quats"]), _ptr(grads["logits"]))
    gg.sh, gg.latents, gg.mlp = _ptr(grads.get("sh")), _ptr(grads.get("latents")), _ptr(grads.get("mlp"))
    return gg


def render_bwd(gauss: Gaussians, cam: Camera, proj: ProjectedBuffers, point_list, ranges, k: int, final_T, n_contrib,
               t_ckpt, dL_dimage, grads: dict, ws, stats=None, deterministic: bool = False,
               schedule=SCHEDULE_BALANCED, stream=None):
    """Full backward, dL/dimage -> parameter gradients (grads keyed like
    project_bwd's).  stats: optional (grad_norm_sum float32[n],
    visible_count int32[n]) accumulated in place."""
    st = None
    if stats is not None:
        st = DensifyStats()
        st.grad_norm_sum, st.visible_count = _ptr(stats[0]), _ptr(stats[1])
    _check(_lib.gs_render_bwd(ctypes.byref(gauss), ctypes.byref(cam), ctypes.byref(proj.struct()), _ptr(point_list),
                              _ptr(ranges), k, _ptr(final_T), _ptr(n_contrib), _ptr(t_ckpt), _ptr(dL_dimage),
                              ctypes.byref(_grad_struct(grads)), ctypes.byref(st) if st is not None else None,
                              _ptr(ws), _nbytes(ws), int(deterministic), int(schedule), _stream(stream)),
           "gs_render_bwd")


def _param_struct(d: dict) -> ParamArrays:
    pa = ParamArrays()
    pa.means, pa.log_scales, pa.quats, pa.logits, pa.sh = (_ptr(d["means"]), _ptr(d["log_scales"]),
                                                           _ptr(d["quats"]), _ptr(d["logits"]), _ptr(d["sh"]))
    return pa


def adam_gaussians(n: int, sh_degree: int, params: dict, grads: dict, m: dict, v: dict, lrs: dict, step: int,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, stream=None):
    """One fused Adam step over every parameter array (updated in place).
    lrs: learning rates keyed means, log_scales, quats, logits, sh_dc, sh_rest."""
    cfg = AdamConfig()
    cfg.lr_means, cfg.lr_log_scales, cfg.lr_quats = lrs["means"], lrs["log_scales"], lrs["quats"]
    cfg.lr_logits, cfg.lr_sh_dc, cfg.lr_sh_rest = lrs["logits"], lrs["sh_dc"], lrs["sh_rest"]
    cfg.beta1, cfg.beta2, cfg.eps, cfg.step = beta1, beta2, eps, int(step)
    _check(_lib.gs_adam_gaussians(n, sh_degree, ctypes.byref(_param_struct(params)),
                                  ctypes.byref(_grad_struct(grads)), ctypes.byref(_param_struct(m)),
                                  ctypes.byref(_param_struct(v)), ctypes.byref(cfg), _stream(stream)),
           "gs_adam_gaussians")


def density_control_workspace(n: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.gs_density_control_workspace(n, ctypes.byref(b)), "gs_density_control_workspace")
    return int(b.value)


def density_control(gauss: Gaussians, params: dict, noise, out: dict, capacity: int, ws, points: dict = None,
                    stream=None) -> dict:
    """One round of density control (gs_density_control).  params: radius,
    alpha, beta, knn, spread, jitter, gamma; out: parameter arrays with
    `capacity` columns; points: optional per-Gaussian outputs (rho, cls, nn,
    dbar, fate).  Returns the report as a dict; raises GsError (with .report)
    on failure, e.g. GS_ERR_CAPACITY when the output needs more columns."""
    prm = DensityParams(params["radius"], params.get("alpha", 1.0), params.get("beta", 1.0),
                        int(params.get("knn", 3)), params.get("spread", 1.5),
                        params.get("jitter", 0.1 * params["radius"]), params.get("gamma", 1.0))
    rep = DensityReport()
    pts = None
    if points:
        pts = DensityPoints(*(_ptr(points.get(k)) for k in ("rho", "cls", "nn", "dbar", "fate")))
    st = _lib.gs_density_control(ctypes.byref(gauss), ctypes.byref(prm), _ptr(noise),
                                 ctypes.byref(_param_struct(out)), capacity, _ptr(ws), _nbytes(ws), ctypes.byref(rep),
                                 ctypes.byref(pts) if pts is not None else None, _stream(stream))
    report = {f: getattr(rep, f) for f, _ in DensityReport._fields_}
    if st != GS_OK:
        e = GsError(st, "gs_density_control", _lib.gs_last_error().decode())
        e.report = report
        raise e
    return report


def project_bwd_workspace(gauss: Gaussians) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.gs_project_bwd_workspace(ctypes.byref(gauss), ctypes.byref(b)), "gs_project_bwd_workspace")
    return int(b.value)


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def project_bwd(gauss: Gaussians, cam: Camera, g2d, grads: dict, proj: ProjectedBuffers = None, ws=None,
                stream=None):
    """grads: device tensors keyed like the parameters ("sh" for SH colour,
    "latents" [n][16] and "mlp" [MLP_PARAMS] FP32 for the learned colour)."""
    ps = ctypes.byref(proj.struct()) if proj is not None else None
    _check(_lib.gs_project_bwd(ctypes.byref(gauss), ctypes.byref(cam), ps, _ptr(g2d),
                               ctypes.byref(_grad_struct(grads)), _ptr(ws), _nbytes(ws), _stream(stream)),
           "gs_project_bwd")


def l1_loss(img, target, loss, grad, partials, stream=None):
    _check(_lib.gs_l1_loss(_ptr(img), _ptr(target), img.numel(), _ptr(loss), _ptr(grad), _ptr(partials),
                           _stream(stream)), "gs_l1_loss")


def l1_loss_static(img, target, loss, grad, stream=None):
    """gs_l1_loss with the library's static scratch (allocates nothing)."""
    _check(_lib.gs_l1_loss_static(_ptr(img), _ptr(target), img.numel(), _ptr(loss), _ptr(grad), _stream(stream)),
           "gs_l1_loss_static")


# ------------------------------------------------------------ learned colour

def mlp_pack(params_bf16, packed, stream=None):
    """params_bf16: device int16/uint16 tensor of MLP_PARAMS bf16 bit patterns."""
    _check(_lib.gs_mlp_pack(_ptr(params_bf16), _ptr(packed), _stream(stream)), "gs_mlp_pack")


def mlp_fwd(S: int, per: int, latents_bf16, dirs, packed, rgb, stream=None):
    _check(_lib.gs_mlp_fwd(S, per, _ptr(latents_bf16), _ptr(dirs), _ptr(packed), _ptr(rgb), _stream(stream)),
           "gs_mlp_fwd")


def gaussians_struct_mlp(means, log_scales, quats, logits, latents_bf16, packed) -> Gaussians:
    n = means.shape[1]
    _check_f32("means", means, (3, n))
    _check_f32("log_scales", log_scales, (3, n))
    _check_f32("quats", quats, (4, n))
    _check_f32("logits", logits, (n,))
    if tuple(latents_bf16.shape) != (n, 16) or latents_bf16.element_size() != 2:
        raise ValueError("latents: expected a [n][16] 16-bit tensor of bf16 bit patterns")
    g = Gaussians()
    g.n, g.sh_degree, g.colour_mode = n, 0, 1
    g.means, g.log_scales, g.quats, g.logits = _ptr(means), _ptr(log_scales), _ptr(quats), _ptr(logits)
    g.sh = None
    g.latents, g.mlp = _ptr(latents_bf16), _ptr(packed)
    return g


def mlp_bwd_workspace(S: int, per: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.gs_mlp_bwd_workspace(S, per, ctypes.byref(b)), "gs_mlp_bwd_workspace")
    return int(b.value)


def mlp_bwd(S: int, per: int, latents_bf16, dirs, packed, dlatents, dparams, ws, dL_drgb=None, target=None,
            scale: float = 1.0, loss=None, stream=None):
    """Decoder backward: dL/drgb given, or the distillation loss
    scale * sum |rgb - target|^2 (value into `loss`)."""
    _check(_lib.gs_mlp_bwd(S, per, _ptr(latents_bf16), _ptr(dirs), _ptr(packed), _ptr(dL_drgb), _ptr(target),
                           float(scale), _ptr(dlatents), _ptr(dparams), _ptr(loss), _ptr(ws), _nbytes(ws),
                           _stream(stream)), "gs_mlp_bwd")


def sh_colour(S: int, per: int, n: int, sh_degree: int, sh, dirs, rgb, clamp01: bool = True, stream=None):
    _check(_lib.gs_sh_colour(S, per, n, sh_degree, _ptr(sh), _ptr(dirs), int(clamp01), _ptr(rgb), _stream(stream)),
           "gs_sh_colour")


def adam_step(param, grad, m, v, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
              param_bf16=None, stream=None):
    _check(_lib.gs_adam_step(param.numel(), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), _ptr(param_bf16), float(lr),
                             float(beta1), float(beta2), float(eps), int(step), _stream(stream)), "gs_adam_step")


# ------------------------------------------------------------ measurement

def kernel_timer_start():
    """Time every kernel the library launches from this thread (HIP events
    on the launch stream) until kernel_timer_stop."""
    _check(_lib.gs_kernel_timer_start(), "gs_kernel_timer_start")


def kernel_timer_stop() -> dict:
    """Stop the timer: {kernel name: (launches, total ms)} in first-launch order."""
    size = 1 << 20
    buf = ctypes.create_string_buffer(size)
    need = ctypes.c_size_t(0)
    _check(_lib.gs_kernel_timer_stop(buf, size, ctypes.byref(need)), "gs_kernel_timer_stop")
    if need.value > size:
        raise RuntimeError("kernel timer report truncated")
    out = {}
    for line in buf.value.decode().splitlines():
        name, count, ms = line.rsplit(" ", 2)
        out[name] = (int(count), float(ms))
    return out



"""Differentiable tile rasterisation as a torch.autograd.Function over the C ABI.

forward : gs_project -> gs_bin_sort -> gs_render_fwd
backward: gs_render_bwd -> gs_project_bwd
The saved state per call is the projection, the sorted list, the tile ranges,
the final transmittance and per-pixel contributor counts; nothing per
(pixel, Gaussian) pair is stored -- the backward recomputes transmittance.
Buffers are kept in a Rasterizer and reused across iterations; the (tile,
Gaussian) capacity grows on demand (the library reports the size it needs).
The colour comes from SH coefficients (a tensor) or from the learned decoder
(a decoder.LearnedColour: BF16 latents + packed weights, colour_mode 1).
"""
from __future__ import annotations

import contextlib
import dataclasses

import torch

from . import gs
from .decoder import LearnedColour


@dataclasses.dataclass
class FrameState:
    n: int
    k: int
    proj: gs.ProjectedBuffers
    point_list: torch.Tensor
    ranges: torch.Tensor
    image: torch.Tensor
    final_T: torch.Tensor
    n_contrib: torch.Tensor
    t_ckpt: torch.Tensor


class Rasterizer:
    """Holds device buffers for one camera resolution and one Gaussian count."""

    def __init__(self, cam, sh_degree: int, device="cuda", deterministic: bool = False, capacity: int | None = None,
                 schedule: int = gs.SCHEDULE_BALANCED):
        self.cam = cam
        self.schedule = schedule
        self.cs = gs.camera_struct(cam)
        self.sh_degree = sh_degree
        self.device = torch.device(device)
        self.deterministic = deterministic
        self.ntiles = gs.n_tiles(cam)
        self._cap = capacity
        self._n = None
        self.proj = None
        self.point_list = None
        self.bin_ws = None
        self.bwd_ws = None
        self.pbwd_ws = None
        self.t_ckpt = None
        H, W = cam.height, cam.width
        self.ranges = torch.empty((self.ntiles, 2), dtype=torch.int32, device=self.device)
        self.image = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        self.final_T = torch.empty((H, W), dtype=torch.float32, device=self.device)
        self.n_contrib = torch.empty((H, W), dtype=torch.int32, device=self.device)
        self.last_k = 0
        self.timer = None          # optional callable(stage_name) -> context manager

    def _stage(self, name):
        return self.timer(name) if self.timer is not None else contextlib.nullcontext()

    def _ensure(self, n: int):
        if self._n != n:
            self._n = n
            self.proj = gs.ProjectedBuffers(n, self.device)
            if self._cap is None:
                self._cap = max(1024, 8 * n)
            self._alloc_lists(self._cap)

    def _alloc_lists(self, cap: int):
        self._cap = cap
        self.point_list = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        ws = gs.bin_sort_workspace(self._n, cap, self.cs)
        self.bin_ws = torch.empty(ws, dtype=torch.uint8, device=self.device)

    def set_camera(self, cam):
        assert cam.width == self.cam.width and cam.height == self.cam.height
        self.cam = cam
        self.cs = gs.camera_struct(cam)

    def _gauss(self, means, log_scales, quats, logits, colour) -> gs.Gaussians:
        if isinstance(colour, LearnedColour):
            return gs.gaussians_struct_mlp(means, log_scales, quats, logits, colour.latents_bf16, colour.packed)
        return gs.gaussians_struct(means, log_scales, quats, logits, colour, self.sh_degree)

    def forward(self, means, log_scales, quats, logits, colour) -> FrameState:
        n = means.shape[1]
        self._ensure(n)
        g = self._gauss(means, log_scales, quats, logits, colour)
        with self._stage("project"):
            gs.project(g, self.cs, self.proj)
        while True:
            try:
                with self._stage("bin_sort"):
                    k = gs.bin_sort(n, self.proj, self.cs, self.bin_ws, self.point_list, self.ranges)
                break
            except gs.GsError as e:
                if e.status != gs.GS_ERR_CAPACITY:
                    raise
                self._alloc_lists(int(e.required * 1.25) + 1024)
        self.last_k = k
        need = gs.render_ckpt_floats(k, self.cs)
        if self.t_ckpt is None or self.t_ckpt.numel() < need:
            self.t_ckpt = torch.empty(int(need * 1.25), dtype=torch.float32, device=self.device)
        with self._stage("render_fwd"):
            gs.render_fwd(n, self.proj, self.point_list, self.ranges, k, self.cs, self.image, self.final_T,
                          self.n_contrib, self.t_ckpt, schedule=self.schedule)
        return FrameState(n, k, self.proj, self.point_list, self.ranges, self.image, self.final_T, self.n_contrib,
                          self.t_ckpt)

    def backward(self, st: FrameState, means, log_scales, quats, logits, colour, dL_dimage, g2d=None):
        n = st.n
        dL_dimage = dL_dimage.contiguous()
        need = gs.render_bwd_workspace(n, st.k, self.cs, self.deterministic)
        if self.bwd_ws is None or self.bwd_ws.numel() < need:
            self.bwd_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        if g2d is None:
            g2d = torch.empty((gs.G2D, n), dtype=torch.float32, device=self.device)
        with self._stage("render_bwd"):
            gs.render_bwd(n, st.proj, st.point_list, st.ranges, st.k, self.cs, st.final_T, st.n_contrib, st.t_ckpt,
                          dL_dimage, g2d, self.bwd_ws, self.deterministic, schedule=self.schedule)
        grads = {k: torch.empty_like(v) for k, v in
                 (("means", means), ("log_scales", log_scales), ("quats", quats), ("logits", logits))}
        g = self._gauss(means, log_scales, quats, logits, colour)
        ws = None
        if isinstance(colour, LearnedColour):
            grads["latents"] = torch.empty((n, 16), dtype=torch.float32, device=self.device)
            grads["mlp"] = torch.empty(gs.MLP_PARAMS, dtype=torch.float32, device=self.device)
            need = gs.project_bwd_workspace(g)
            if self.pbwd_ws is None or self.pbwd_ws.numel() < need:
                self.pbwd_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            ws = self.pbwd_ws
        else:
            grads["sh"] = torch.empty_like(colour)
        with self._stage("project_bwd"):
            gs.project_bwd(g, self.cs, g2d, grads, proj=st.proj, ws=ws)
        return grads, g2d


class _RasterizeFn(torch.autograd.Function):
    """Inputs: the geometry tensors, then the colour's tensors -- (sh, None) for
    SH colour, (latents FP32, weights FP32) for the learned colour, whose BF16
    copies and packed weights come in `learned` (kept in sync by the caller)."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, logits, c0, c1, rast: Rasterizer, learned):
        colour = learned if learned is not None else c0
        st = rast.forward(means, log_scales, quats, logits, colour)
        ctx.rast, ctx.st, ctx.colour = rast, st, colour
        ctx.save_for_backward(means, log_scales, quats, logits)
        # the rasterizer reuses its image buffer next call: hand autograd a copy
        return st.image.clone()

    @staticmethod
    def backward(ctx, dL_dimage):
        means, log_scales, quats, logits = ctx.saved_tensors
        grads, _ = ctx.rast.backward(ctx.st, means, log_scales, quats, logits, ctx.colour, dL_dimage)
        if isinstance(ctx.colour, LearnedColour):
            gc0, gc1 = grads["latents"], grads["mlp"]
        else:
            gc0, gc1 = grads["sh"], None
        return grads["means"], grads["log_scales"], grads["quats"], grads["logits"], gc0, gc1, None, None


def rasterize(means, log_scales, quats, logits, sh, rast: Rasterizer):
    """Differentiable render of the Gaussians with the rasterizer's camera: image[3][H][W]."""
    return _RasterizeFn.apply(means, log_scales, quats, logits, sh, None, rast, None)


def rasterize_learned(means, log_scales, quats, logits, dec, rast: Rasterizer):
    """Same with the learned colour of a decoder.Decoder: gradients flow to
    dec.latents and dec.params (FP32 masters) when they require grad."""
    return _RasterizeFn.apply(means, log_scales, quats, logits, dec.latents, dec.params, rast, dec.colour())


def l1_loss(img, target, partials=None):
    """(loss device scalar, dL/dimg) from the library's L1 kernel."""
    loss = torch.empty(1, dtype=torch.float32, device=img.device)
    grad = torch.empty_like(img)
    if partials is None:
        partials = torch.empty(gs.L1_PARTIALS, dtype=torch.float32, device=img.device)
    gs.l1_loss(img.contiguous(), target.contiguous(), loss, grad, partials)
    return loss, grad

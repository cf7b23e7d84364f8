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
                 schedule: int = gs.SCHEDULE_BALANCED, async_k: bool = False):
        self.cam = cam
        # async_k: bin with gs_bin_sort_async (no host wait inside a frame) once
        # a frame's K is known; each frame's K is checked at the next forward
        # (or by check_async), which raises GsError if that frame's lists did
        # not fit -- its outputs are then invalid and the capacity has grown
        self.async_k = async_k
        self.k_dev = None       # int64[2] on the device, K and the look-back flag
        self.k_host = None      # its pinned host copy
        self._k_event = None
        self._k_cap = 0
        self.last_k = None
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
        k = None
        if self.async_k and self.last_k is not None:
            self.check_async()
            if self.k_dev is None:
                self.k_dev = torch.zeros(2, dtype=torch.int64, device=self.device)
                self.k_host = torch.zeros(2, dtype=torch.int64, pin_memory=True)
            try:
                with self._stage("bin_sort"):
                    gs.bin_sort_async(n, self.proj, self.cs, self.bin_ws, self.point_list, self.ranges, self.k_dev)
                self.k_host.copy_(self.k_dev, non_blocking=True)
                self._k_event = torch.cuda.Event()
                self._k_event.record()
                k = self._k_cap = self._cap   # an upper bound serves every later layout
            except gs.GsError as e:
                if e.status != gs.GS_ERR_UNSUPPORTED:
                    raise
                self.async_k = False           # frame too large for the direct emission
        while k is None:
            try:
                with self._stage("bin_sort"):
                    k = gs.bin_sort(n, self.proj, self.cs, self.bin_ws, self.point_list, self.ranges)
            except gs.GsError as e:
                if e.status != gs.GS_ERR_CAPACITY:
                    raise
                self._alloc_lists(int(e.required * 1.25) + 1024)
            else:
                self.last_k = k
        need = gs.render_ckpt_floats(k, self.cs)
        if self.t_ckpt is None or self.t_ckpt.numel() < need:
            self.t_ckpt = torch.empty(int(need * 1.25), dtype=torch.float32, device=self.device)
        with self._stage("render_fwd"):
            gs.render_fwd(n, self.proj, self.point_list, self.ranges, k, self.cs, self.image, self.final_T,
                          self.n_contrib, self.t_ckpt, schedule=self.schedule)
        return FrameState(n, k, self.proj, self.point_list, self.ranges, self.image, self.final_T, self.n_contrib,
                          self.t_ckpt)

    def check_async(self) -> int | None:
        """Check the last frame binned without a host wait: returns its K, or
        raises GsError (GS_ERR_CAPACITY with .required = K, after growing the
        capacity; GS_ERR_HIP if its depth sort did not complete)."""
        if self._k_event is None:
            return self.last_k
        self._k_event.synchronize()
        self._k_event = None
        K, flag = int(self.k_host[0]), int(self.k_host[1])
        if flag:
            raise gs.GsError(gs.GS_ERR_HIP, "gs_bin_sort_async", "depth sort look-back did not complete")
        if K > self._k_cap:
            self._alloc_lists(int(K * 1.25) + 1024)
            e = gs.GsError(gs.GS_ERR_CAPACITY, "gs_bin_sort_async",
                           f"a frame needed {K} entries, the capacity was {self._k_cap}")
            e.required = K
            raise e
        self.last_k = K
        return K

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

"""Differentiable tile rasterisation as a torch.autograd.Function over the C ABI.

forward : gs_project -> gs_bin_sort -> gs_render_fwd
backward: gs_render_bwd (compositing backward + projection backward)
The saved state per call is the projection, the sorted list, the tile ranges,
the final transmittance, per-pixel contributor counts and the batch-boundary
transmittance checkpoints; nothing per (pixel, Gaussian) pair is stored --
the backward recomputes transmittance.  Each forward gets its own output
buffers (from PyTorch's caching allocator, so no device allocation once warm)
and its camera; the Rasterizer keeps the scratch workspaces and the (tile,
Gaussian) capacity, which grows on demand (the library reports the size it
needs).
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
    """One forward's outputs, kept for its backward.  Every frame owns its
    buffers and its camera, so several frames can be alive at once (views
    summed into one loss); the rasterizer only shares scratch workspaces,
    which each call uses on the stream and leaves."""
    n: int
    k: int
    cs: gs.Camera
    proj: gs.ProjectedBuffers
    point_list: torch.Tensor
    ranges: torch.Tensor
    image: torch.Tensor
    final_T: torch.Tensor
    n_contrib: torch.Tensor
    t_ckpt: torch.Tensor
    schedule: int = gs.SCHEDULE_BALANCED   # work split (and sampling flag) of the forward; the backward uses it


class Rasterizer:
    """Buffers and settings for one camera resolution and one Gaussian count."""

    def __init__(self, cam, sh_degree: int, device="cuda", deterministic: bool = False, capacity: int | None = None,
                 schedule: int = gs.SCHEDULE_BALANCED, async_k: bool = False):
        """schedule: a work split, optionally or-ed with gs.RENDER_COLOUR_HASH
        (the approximate colour-hash sampling mode, forward and backward)."""
        self.cam = cam
        # async_k: bin with gs_bin_sort_async (no host wait inside a frame) once
        # a frame's K is known; each frame's K is checked at the next forward
        # (or by check_async), which raises GsError if that frame's lists did
        # not fit -- its outputs are then invalid and the capacity has grown
        self.async_k = async_k
        self.k_host = None      # int64[2] in pinned host memory: K and the look-back flag
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
        self._ckpt_floats = 0
        self.bin_ws = None
        self.bwd_ws = None
        self.stats = None          # optional (grad_norm_sum, visible_count), see enable_densify_stats
        self.timer = None          # optional callable(stage_name) -> context manager
        self.last_frame = None     # the latest forward's FrameState (for inspection)

    def _stage(self, name):
        return self.timer(name) if self.timer is not None else contextlib.nullcontext()

    def _ensure(self, n: int):
        if self._n != n:
            self._n = n
            if self._cap is None:
                self._cap = max(1024, 8 * n)
            self._alloc_lists(self._cap)

    def _alloc_lists(self, cap: int):
        self._cap = cap
        ws = gs.bin_sort_workspace(self._n, cap, self.cs)
        self.bin_ws = torch.empty(ws, dtype=torch.uint8, device=self.device)

    def set_camera(self, cam):
        assert cam.width == self.cam.width and cam.height == self.cam.height
        self.cam = cam
        self.cs = gs.camera_struct(cam)

    def enable_densify_stats(self, n: int):
        """Accumulate densification statistics over the following backwards:
        (sum over views of |dL/d(u, v)|, number of views that see the
        Gaussian).  Returns the two tensors (zeroed)."""
        self.stats = (torch.zeros(n, dtype=torch.float32, device=self.device),
                      torch.zeros(n, dtype=torch.int32, device=self.device))
        return self.stats

    def _gauss(self, means, log_scales, quats, logits, colour) -> gs.Gaussians:
        if isinstance(colour, LearnedColour):
            return gs.gaussians_struct_mlp(means, log_scales, quats, logits, colour.latents_bf16, colour.packed)
        return gs.gaussians_struct(means, log_scales, quats, logits, colour, self.sh_degree)

    def forward(self, means, log_scales, quats, logits, colour) -> FrameState:
        n = means.shape[1]
        self._ensure(n)
        dev = self.device
        cs = self.cs
        g = self._gauss(means, log_scales, quats, logits, colour)
        proj = gs.ProjectedBuffers(n, dev)
        with self._stage("project"):
            gs.project(g, cs, proj)
        ranges = torch.empty((self.ntiles, 2), dtype=torch.int32, device=dev)
        k = None
        point_list = None
        if self.async_k and self.last_k is not None:
            self.check_async()
            if self.k_host is None:
                # pinned: the bin/sort kernels write K and the flag here directly
                self.k_host = torch.zeros(2, dtype=torch.int64, pin_memory=True)
            point_list = torch.empty(max(self._cap, 1), dtype=torch.int32, device=dev)
            try:
                with self._stage("bin_sort"):
                    gs.bin_sort_async(n, proj, cs, self.bin_ws, point_list, ranges, self.k_host)
                self._k_event = torch.cuda.Event()
                self._k_event.record()
                k = self._k_cap = self._cap   # an upper bound serves every later layout
            except gs.GsError as e:
                if e.status != gs.GS_ERR_UNSUPPORTED:
                    raise
                self.async_k = False           # frame too large for the direct emission
        while k is None:
            if point_list is None or point_list.numel() < self._cap:
                point_list = torch.empty(max(self._cap, 1), dtype=torch.int32, device=dev)
            try:
                with self._stage("bin_sort"):
                    k = gs.bin_sort(n, proj, cs, self.bin_ws, point_list, ranges)
            except gs.GsError as e:
                if e.status != gs.GS_ERR_CAPACITY:
                    raise
                self._alloc_lists(int(e.required * 1.25) + 1024)
            else:
                self.last_k = k
        need = gs.render_ckpt_floats(k, cs)
        if need > self._ckpt_floats:
            self._ckpt_floats = int(need * 1.25)
        H, W = self.cam.height, self.cam.width
        image = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        final_T = torch.empty((H, W), dtype=torch.float32, device=dev)
        n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
        t_ckpt = torch.empty(self._ckpt_floats, dtype=torch.float32, device=dev)
        with self._stage("render_fwd"):
            gs.render_fwd(n, proj, point_list, ranges, k, cs, image, final_T, n_contrib, t_ckpt,
                          schedule=self.schedule)
        self.last_frame = FrameState(n, k, cs, proj, point_list, ranges, image, final_T, n_contrib, t_ckpt,
                                     self.schedule)
        return self.last_frame

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

    def backward(self, st: FrameState, means, log_scales, quats, logits, colour, dL_dimage) -> dict:
        """Parameter gradients of sum(dL_dimage * image) for frame st."""
        n = st.n
        dL_dimage = dL_dimage.contiguous()
        g = self._gauss(means, log_scales, quats, logits, colour)
        need = gs.render_bwd_workspace(g, st.k, st.cs, self.deterministic)
        if self.bwd_ws is None or self.bwd_ws.numel() < need:
            self.bwd_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        grads = {k: torch.empty_like(v) for k, v in
                 (("means", means), ("log_scales", log_scales), ("quats", quats), ("logits", logits))}
        if isinstance(colour, LearnedColour):
            grads["latents"] = torch.empty((n, 16), dtype=torch.float32, device=self.device)
            grads["mlp"] = torch.empty(gs.MLP_PARAMS, dtype=torch.float32, device=self.device)
        else:
            grads["sh"] = torch.empty_like(colour)
        stats = self.stats if (self.stats is not None and self.stats[0].numel() == n) else None
        with self._stage("render_bwd"):
            gs.render_bwd(g, st.cs, st.proj, st.point_list, st.ranges, st.k, st.final_T, st.n_contrib, st.t_ckpt,
                          dL_dimage, grads, self.bwd_ws, stats=stats, deterministic=self.deterministic,
                          schedule=st.schedule)
        return grads


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
        return st.image

    @staticmethod
    def backward(ctx, dL_dimage):
        means, log_scales, quats, logits = ctx.saved_tensors
        grads = ctx.rast.backward(ctx.st, means, log_scales, quats, logits, ctx.colour, dL_dimage)
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

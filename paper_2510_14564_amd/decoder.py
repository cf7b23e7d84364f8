"""Learned colour decoder: parameters, Adam state and distillation from SH colours.

Not part of the paper's method.  The decoder replaces the SH colour read of
the projection (Sec. I and Sec. II-A: colour from SH coefficients) with a
shared MLP on a 16-value BF16 latent per Gaussian and the real SH encoding of
the view direction (32 -> 64 -> 64 -> 3, ReLU, sigmoid).  It is trained by
distillation: per Gaussian, `per` fixed directions on the sphere, target =
the SH colour there clamped to [0, 1], loss = mean over Gaussians and
directions of the squared colour error.

Every step runs in the library's kernels (gs_sh_colour for the targets,
gs_mlp_bwd for the fused forward + loss + backward, gs_adam_step, gs_mlp_pack);
this module only owns the buffers.  FP32 master copies are updated by Adam,
which also writes the BF16 copies the forward reads.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import gs, scenes

N_LATENT = 16
# parameter blocks in the library's order (row-major), with their fan-in
_LAYOUT = (("W1", (64, 32)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (3, 64)), ("b3", (3,)))


def init_params(seed: int) -> np.ndarray:
    """Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases, as BF16 bits."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in _LAYOUT:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shape[1])
            out.append(rng.uniform(-bound, bound, int(np.prod(shape))))
        else:
            out.append(np.zeros(int(np.prod(shape))))
    return scenes.bf16_bits(np.concatenate(out).astype(np.float32))


@dataclasses.dataclass
class LearnedColour:
    """What the projection reads in colour_mode 1."""
    latents_bf16: torch.Tensor   # int16 [n][16] (BF16 bit patterns)
    packed: torch.Tensor         # the packed operand image of gs_mlp_pack


class Decoder:
    """Decoder weights and per-Gaussian latents on the device, with Adam state."""

    def __init__(self, n: int, device="cuda", seed: int = 0, latents_bits: np.ndarray | None = None,
                 params_bits: np.ndarray | None = None):
        self.n = n
        self.device = torch.device(device)
        pb = init_params(seed) if params_bits is None else params_bits
        if latents_bits is None:
            latents_bits = scenes.bf16_bits(
                np.random.default_rng(seed + 1).normal(0.0, 0.1, (n, N_LATENT)).astype(np.float32))
        dev = self.device
        self.params_bf16 = torch.from_numpy(pb.view(np.int16).copy()).to(dev)
        self.params = torch.from_numpy(scenes.bf16_to_f32(pb)).to(dev)
        self.latents_bf16 = torch.from_numpy(latents_bits.view(np.int16).copy()).to(dev)
        self.latents = torch.from_numpy(scenes.bf16_to_f32(latents_bits)).to(dev)
        self.packed = torch.empty(gs.MLP_PACKED_BYTES // 4 + 4, dtype=torch.float32, device=dev)
        self.m_w, self.v_w = torch.zeros_like(self.params), torch.zeros_like(self.params)
        self.m_z, self.v_z = torch.zeros_like(self.latents), torch.zeros_like(self.latents)
        self.step_w = 0
        self.pack()

    def pack(self):
        gs.mlp_pack(self.params_bf16, self.packed)

    def colour(self) -> LearnedColour:
        return LearnedColour(self.latents_bf16, self.packed)

    def adam_weights(self, grad, lr: float):
        self.step_w += 1
        gs.adam_step(self.params, grad, self.m_w, self.v_w, lr, self.step_w, param_bf16=self.params_bf16)
        self.pack()

    def adam_latents(self, grad, lr: float, step: int, lo: int = 0, hi: int | None = None):
        hi = self.n if hi is None else hi
        gs.adam_step(self.latents[lo:hi], grad, self.m_z[lo:hi], self.v_z[lo:hi], lr, step,
                     param_bf16=self.latents_bf16[lo:hi])


class Distiller:
    """Distillation of a Decoder from a scene's SH colours at fixed directions."""

    def __init__(self, dec: Decoder, sh, sh_degree: int, per: int = 64, seed: int = 5001, batch: int = 16384):
        n = dec.n
        self.dec, self.per, self.batch = dec, per, batch
        dev = dec.device
        self.dirs = torch.from_numpy(scenes.view_dirs(n, per, seed).reshape(n * per, 3)).to(dev)
        self.target = torch.empty((n * per, 3), dtype=torch.float32, device=dev)
        gs.sh_colour(n * per, per, n, sh_degree, sh, self.dirs, self.target, clamp01=True)
        self.dlat = torch.empty((n, N_LATENT), dtype=torch.float32, device=dev)
        self.dP = torch.empty(gs.MLP_PARAMS, dtype=torch.float32, device=dev)
        nb = (n + batch - 1) // batch
        self.losses = torch.zeros((0, nb), dtype=torch.float32, device=dev)
        self.ws = torch.empty(gs.mlp_bwd_workspace(min(n, batch) * per, per), dtype=torch.uint8, device=dev)
        self.epoch = 0

    def run_epoch(self, lr_w: float = 1e-3, lr_z: float = 1e-2):
        """One pass over the Gaussians in batches: fused decoder forward, loss
        and backward, then Adam on the weights and on the batch's latents."""
        dec, per, B = self.dec, self.per, self.batch
        n = dec.n
        self.epoch += 1
        row = torch.empty((1, self.losses.shape[1]), dtype=torch.float32, device=dec.device)
        for j, lo in enumerate(range(0, n, B)):
            hi = min(n, lo + B)
            S = (hi - lo) * per
            gs.mlp_bwd(S, per, dec.latents_bf16[lo:hi], self.dirs[lo * per:hi * per], dec.packed,
                       self.dlat[lo:hi], self.dP, self.ws, target=self.target[lo * per:hi * per],
                       scale=1.0 / S, loss=row[0, j:j + 1])
            dec.adam_weights(self.dP, lr_w)
            dec.adam_latents(self.dlat[lo:hi], lr_z, self.epoch, lo, hi)
        self.losses = torch.cat([self.losses, row])

    def train(self, epochs: int, lr_w: float = 1e-3, lr_z: float = 1e-2, final_factor: float = 0.01):
        """`epochs` epochs with both learning rates decayed on a cosine from
        their base value to `final_factor` times it."""
        for e in range(epochs):
            f = final_factor + (1.0 - final_factor) * 0.5 * (1.0 + np.cos(np.pi * e / max(epochs - 1, 1)))
            self.run_epoch(lr_w * f, lr_z * f)

    def loss_history(self) -> np.ndarray:
        """Per-epoch mean squared colour error (weighted by batch size)."""
        L = self.losses.cpu().numpy().astype(np.float64)
        n, B = self.dec.n, self.batch
        w = np.array([min(n, lo + B) - lo for lo in range(0, n, B)], np.float64)
        return (L * w).sum(1) / n

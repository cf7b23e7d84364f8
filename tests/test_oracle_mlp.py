"""Pins of the oracle's learned colour decoder and distillation target (CPU).

The decoder is not in the paper; it replaces the SH colour read of the
projection (Sec. I / Sec. II-A colour from SH coefficients) with a small MLP
on a per-Gaussian latent and the SH encoding of the view direction.  Each pin
checks the oracle against something other than itself: torch.autograd on an
independent torch implementation, central finite differences, the W = 0
special case, the textbook SH table, and torch's own bfloat16 rounding.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import brute
from paper_2510_14564_amd import scenes


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0.0, scale, oracle.MLP_PARAMS)


def _torch_mlp(x, P):
    t = lambda a: torch.as_tensor(a)
    sl = {k: t(P[o:o + int(np.prod(s))]).reshape(s) for k, (o, s) in oracle.MLP_SLICES.items()}
    h1 = torch.relu(x @ sl["W1"].T + sl["b1"])
    h2 = torch.relu(h1 @ sl["W2"].T + sl["b2"])
    return torch.sigmoid(h2 @ sl["W3"].T + sl["b3"])


def _dirs(n, per, seed):
    d = np.random.default_rng(seed).normal(size=(n, per, 3))
    return d / np.linalg.norm(d, axis=2, keepdims=True)


def test_inputs_are_latent_then_textbook_sh():
    z = np.random.default_rng(1).normal(size=(7, 16))
    d = _dirs(7, 5, 2)
    x = oracle.mlp_inputs(z, d)
    assert x.shape == (35, 32)
    np.testing.assert_array_equal(x[:, :16], np.repeat(z, 5, axis=0))
    Y = brute.sh_table(3, torch.tensor(d.reshape(-1, 3))).numpy()
    np.testing.assert_allclose(x[:, 16:], Y, atol=1e-14)


def test_forward_and_gradients_match_torch_autograd():
    P = _params(3)
    x = np.random.default_rng(4).normal(size=(64, 32))
    c = oracle.mlp_fwd(x, P)
    xt = torch.tensor(x, requires_grad=True)
    Pt = torch.tensor(P, requires_grad=True)
    ct = _torch_mlp(xt, Pt)
    np.testing.assert_allclose(c, ct.detach().numpy(), atol=1e-14)
    G = np.random.default_rng(5).normal(size=c.shape)
    (ct * torch.tensor(G)).sum().backward()
    dP, dx = oracle.mlp_bwd(x, P, G)
    np.testing.assert_allclose(dP, Pt.grad.numpy(), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_gradients_match_central_finite_differences():
    P = _params(6)
    x = np.random.default_rng(7).normal(size=(16, 32))
    G = np.random.default_rng(8).normal(size=(16, 3))
    dP, dx = oracle.mlp_bwd(x, P, G)
    h = 1e-6
    rng = np.random.default_rng(9)
    for name, (off, shape) in oracle.MLP_SLICES.items():
        for k in rng.choice(int(np.prod(shape)), size=3, replace=False):
            i = off + k
            Pp, Pm = P.copy(), P.copy()
            Pp[i] += h
            Pm[i] -= h
            fd = (np.sum(G * oracle.mlp_fwd(x, Pp)) - np.sum(G * oracle.mlp_fwd(x, Pm))) / (2 * h)
            assert abs(fd - dP[i]) < 1e-6 * max(1.0, abs(fd)), (name, k, fd, dP[i])
    for s, j in ((0, 3), (5, 20), (11, 31)):
        xp, xm = x.copy(), x.copy()
        xp[s, j] += h
        xm[s, j] -= h
        fd = (np.sum(G * oracle.mlp_fwd(xp, P)) - np.sum(G * oracle.mlp_fwd(xm, P))) / (2 * h)
        assert abs(fd - dx[s, j]) < 1e-6 * max(1.0, abs(fd))


def test_zero_weights_give_sigmoid_of_output_bias():
    P = np.zeros(oracle.MLP_PARAMS)
    b3 = np.array([-1.0, 0.3, 2.0])
    P[oracle.MLP_SLICES["b3"][0]:] = b3
    P[oracle.MLP_SLICES["b1"][0]:oracle.MLP_SLICES["b1"][0] + 64] = 0.7   # hidden biases cannot leak through W = 0
    x = np.random.default_rng(10).normal(size=(9, 32))
    c = oracle.mlp_fwd(x, P)
    np.testing.assert_allclose(c, np.broadcast_to(1 / (1 + np.exp(-b3)), (9, 3)), atol=1e-15)


def test_sh_colour_matches_textbook_basis():
    s = scenes.skewed_scene(50, 3, n_clusters=2, sh_degree=3)
    d = _dirs(50, 4, 11)
    c = oracle.sh_colour(s.sh, 3, d)
    Y = brute.sh_table(3, torch.tensor(d)).numpy()                  # [n][per][16]
    want = np.maximum(0.0, np.einsum("npj,jcn->npc", Y, s.sh.astype(np.float64)) + 0.5)
    np.testing.assert_allclose(c, want, atol=1e-14)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(12).normal(0, 3, 10000).astype(np.float32)
    x[:4] = [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9]   # ties round to even
    bits = scenes.bf16_bits(x)
    want = torch.tensor(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(bits, want)
    back = scenes.bf16_to_f32(bits)
    assert np.all(np.abs(back - x) <= np.abs(x) * 2.0 ** -8)


def test_brute_learned_colour_matches_c_oracle_and_finite_differences():
    """The torch route (brute.learned_colour) agrees with the C oracle's inputs,
    forward and parameter/latent gradients, and its gradient in the means with
    central differences of the C oracle's forward."""
    rng = np.random.default_rng(13)
    n = 12
    means = rng.normal(size=(3, n))
    centre = np.array([0.3, -0.2, -4.0])
    z = rng.normal(0, 0.3, (n, 16))
    P = _params(14)
    G = rng.normal(size=(n, 3))
    mt = torch.tensor(means, requires_grad=True)
    zt = torch.tensor(z, requires_grad=True)
    Pt = torch.tensor(P, requires_grad=True)
    c = brute.learned_colour(mt, centre, zt, Pt)
    dirs = (means.T - centre) / np.linalg.norm(means.T - centre, axis=1, keepdims=True)
    x = oracle.mlp_inputs(z, dirs[:, None, :])
    np.testing.assert_allclose(c.detach().numpy(), oracle.mlp_fwd(x, P), atol=1e-14)
    (c * torch.tensor(G)).sum().backward()
    dP, dx = oracle.mlp_bwd(x, P, G)
    np.testing.assert_allclose(Pt.grad.numpy(), dP, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(zt.grad.numpy(), dx[:, :16], rtol=1e-10, atol=1e-13)

    def f(m):
        d = (m.T - centre) / np.linalg.norm(m.T - centre, axis=1, keepdims=True)
        return np.sum(G * oracle.mlp_fwd(oracle.mlp_inputs(z, d[:, None, :]), P))
    h = 1e-6
    for k, i in ((0, 0), (1, 5), (2, 11)):
        mp, mm = means.copy(), means.copy()
        mp[k, i] += h
        mm[k, i] -= h
        fd = (f(mp) - f(mm)) / (2 * h)
        assert abs(fd - mt.grad[k, i].item()) < 1e-6 * max(1.0, abs(fd)), (k, i, fd, mt.grad[k, i].item())

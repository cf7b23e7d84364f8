"""Pins of the oracle's training-step functions (CPU only): the Adam update
against torch.optim.Adam in FP64, and the densification statistics against
their definition on hand-made gradients."""
import numpy as np
import torch

import oracle


def test_adam_step_matches_torch_optim_adam():
    rng = np.random.default_rng(4)
    shape = (5, 37)
    p0 = rng.normal(size=shape)
    lrs = np.array([1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3])[:, None]   # one rate per row (parameter group)
    grads = [rng.normal(size=shape) * s for s in (1.0, 1e-3, 10.0, 0.5)]
    P, M, V = p0.copy(), np.zeros(shape), np.zeros(shape)
    tp = [torch.tensor(p0[r:r + 1], dtype=torch.float64, requires_grad=True) for r in range(shape[0])]
    opt = torch.optim.Adam([{"params": [t], "lr": float(lrs[r, 0])} for r, t in enumerate(tp)],
                           betas=(0.9, 0.999), eps=1e-15)
    for step, g in enumerate(grads, start=1):
        P, M, V = oracle.adam_step(P, g, M, V, lrs, step)
        for r, t in enumerate(tp):
            t.grad = torch.tensor(g[r:r + 1], dtype=torch.float64)
        opt.step()
        got = np.concatenate([t.detach().numpy() for t in tp])
        np.testing.assert_allclose(P, got, rtol=1e-13, atol=1e-15)
    # first step closed form: every value moves by lr against its gradient's sign
    P1, _, _ = oracle.adam_step(p0, grads[0], np.zeros(shape), np.zeros(shape), lrs, 1, eps=0.0)
    np.testing.assert_allclose(P1 - p0, -lrs * np.sign(grads[0]), rtol=1e-12, atol=1e-15)


def test_densify_stats_definition():
    g1 = np.zeros((3, 9)); g1[:, 0] = [3.0, 0.0, -1.0]; g1[:, 1] = [4.0, 2.0, 0.0]
    g2 = np.zeros((3, 9)); g2[:, 0] = [0.0, 6.0, 0.0]; g2[:, 1] = [1.0, 8.0, 5.0]
    s, c = oracle.densify_stats([g1, g2], [np.array([1, 1, 0], bool), np.array([0, 1, 1], bool)])
    np.testing.assert_allclose(s, [5.0, 2.0 + 10.0, 5.0])
    assert c.tolist() == [1, 2, 1]

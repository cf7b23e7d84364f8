"""Error bounds of the learned-colour decoder's matrix-core kernels, shared by
the GPU tests.  Both sides use the same BF16 latents and weights; the HIP path
carries the SH encoding of the direction and both hidden activations as
hi + lo BF16 pairs and accumulates in FP32.  The bounds are running error
bounds of exactly those roundings, propagated through |W| in FP64."""
import numpy as np

import oracle
from paper_2510_14564_amd import scenes
from gpu_helpers import say

U = 2.0 ** -8      # bf16 relative rounding bound (half an ulp = 2^-9, doubled for safety)
UA = 2.0 ** -16    # hi + lo pair of bf16 values (2^-17 + FP32 rounding, doubled)
G32 = 2.0 ** -22   # FP32 accumulation, per term, with margin


def kaiming_params(seed):
    """Kaiming-uniform weights and small biases, rounded to bf16 bit patterns."""
    rng = np.random.default_rng(seed)
    P = np.zeros(oracle.MLP_PARAMS, np.float32)
    for name, (off, shape) in oracle.MLP_SLICES.items():
        size = int(np.prod(shape))
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shape[1])
            P[off:off + size] = rng.uniform(-bound, bound, size)
        else:
            P[off:off + size] = rng.uniform(-0.1, 0.1, size)
    return scenes.bf16_bits(P)


F32 = 2.0 ** -23   # FP32 rounding, doubled


def _slices(P):
    return {k: P[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in oracle.MLP_SLICES.items()}


def fwd_bounds(x, P, ex=None):
    """Running error bound of the forward: pre-activation errors d1, d2, d3,
    post-activation (BF16-rounded) errors e1, e2, colour error dc; plus the
    FP64 quantities.  ex: bound on the input error (default: the SH half
    rounded to BF16, latents exact)."""
    sl = _slices(P)
    ax = np.abs(x)
    if ex is None:
        ex = np.concatenate([np.zeros_like(ax[:, :16]), UA * ax[:, 16:]], axis=1)
    W1, W2, W3 = np.abs(sl["W1"]), np.abs(sl["W2"]), np.abs(sl["W3"])
    a1 = x @ sl["W1"].T + sl["b1"]
    h1 = np.maximum(a1, 0)
    a2 = h1 @ sl["W2"].T + sl["b2"]
    h2 = np.maximum(a2, 0)
    a3 = h2 @ sl["W3"].T + sl["b3"]
    c = 1 / (1 + np.exp(-a3))
    # 2x the terms: every product is two accumulated MFMAs (hi, lo)
    d1 = ex @ W1.T + 64 * G32 * ((ax + ex) @ W1.T + np.abs(sl["b1"]))
    e1 = d1 + UA * (h1 + d1)
    d2 = e1 @ W2.T + 128 * G32 * ((h1 + e1) @ W2.T + np.abs(sl["b2"]))
    e2 = d2 + UA * (h2 + d2)
    d3 = e2 @ W3.T + 128 * G32 * ((h2 + e2) @ W3.T + np.abs(sl["b3"]))
    dc = 0.25 * d3 + 2e-6
    return dict(sl=sl, ax=ax, ex=ex, a1=a1, h1=h1, a2=a2, h2=h2, c=c, d1=d1, e1=e1, d2=d2, e2=e2, dc=dc)


def error_bound(x, P):
    """Per-sample, per-channel bound on |c_gpu - c_exact|."""
    return fwd_bounds(x, P)["dc"]


def bwd_bounds(x, P, G, eG=None, ex=None):
    """Bounds on |dP_gpu - dP*| [6467] and |dx_gpu - dx*| [S][32] for the
    backward of sum(G * c): the forward bound, BF16 rounding of every operand
    the kernel feeds to the matrix cores (gradients and activations), FP32
    accumulation, and -- where a pre-activation lies within its error bound of
    0 -- the whole value of a ReLU gate that may have flipped.  eG bounds the
    error of G itself (the distillation loss takes G from the kernel's own c)."""
    f = fwd_bounds(x, P, ex)
    sl, ax, ex, c, dc = f["sl"], f["ax"], f["ex"], f["c"], f["dc"]
    W1, W2, W3 = np.abs(sl["W1"]), np.abs(sl["W2"]), np.abs(sl["W3"])
    S = x.shape[0]
    if eG is None:
        eG = np.zeros_like(G)
    s3 = c * (1 - c)
    g3 = G * s3
    eg3 = np.abs(G) * (dc + dc * dc) + eG * (s3 + dc + dc * dc) + 1e-6 * np.abs(g3)
    eg3b = eg3 + UA * (np.abs(g3) + eg3)
    t2 = g3 @ sl["W3"]
    et2 = eg3b @ W3 + 3 * G32 * (np.abs(g3) + eg3b) @ W3
    g2 = t2 * (f["a2"] > 0)
    eg2 = np.where(np.abs(f["a2"]) <= f["d2"], np.abs(t2) + et2, et2)
    eg2b = eg2 + UA * (np.abs(g2) + eg2)
    t1 = g2 @ sl["W2"]
    et1 = eg2b @ W2 + 64 * G32 * (np.abs(g2) + eg2b) @ W2
    g1 = t1 * (f["a1"] > 0)
    eg1 = np.where(np.abs(f["a1"]) <= f["d1"], np.abs(t1) + et1, et1)
    eg1b = eg1 + UA * (np.abs(g1) + eg1)
    edx = eg1b @ W1 + 64 * G32 * (np.abs(g1) + eg1b) @ W1
    acc = (S / 16 + 256) * F32
    h1, h2 = f["h1"], f["h2"]
    # the weight-gradient products read hi + lo pairs (lo x lo dropped)
    e1 = f["e1"] + UA * (h1 + f["e1"])
    e2 = f["e2"] + UA * (h2 + f["e2"])
    ex = ex + np.concatenate([np.zeros_like(ax[:, :16]), UA * (ax[:, 16:] + ex[:, 16:])], axis=1)
    xs = ax + ex
    eP = np.zeros(oracle.MLP_PARAMS)

    def put(name, v):
        off, shape = oracle.MLP_SLICES[name]
        eP[off:off + int(np.prod(shape))] = v.reshape(-1)

    ag1, ag2, ag3 = np.abs(g1), np.abs(g2), np.abs(g3)
    # mass: the sum over samples of |per-sample terms| of each exact gradient
    mass = np.zeros(oracle.MLP_PARAMS)

    def put_mass(name, v):
        off, shape = oracle.MLP_SLICES[name]
        mass[off:off + int(np.prod(shape))] = v.reshape(-1)

    put_mass("W1", ag1.T @ ax)
    put_mass("W2", ag2.T @ h1)
    put_mass("W3", ag3.T @ h2)
    put_mass("b1", ag1.sum(0))
    put_mass("b2", ag2.sum(0))
    put_mass("b3", ag3.sum(0))
    put("W1", eg1b.T @ xs + ag1.T @ ex + acc * (ag1 + eg1b).T @ xs)
    put("W2", eg2b.T @ (h1 + e1) + ag2.T @ e1 + acc * (ag2 + eg2b).T @ (h1 + e1))
    put("W3", eg3b.T @ (h2 + e2) + ag3.T @ e2 + acc * (ag3 + eg3b).T @ (h2 + e2))
    put("b1", eg1.sum(0) + acc * (ag1 + eg1).sum(0))
    put("b2", eg2.sum(0) + acc * (ag2 + eg2).sum(0))
    put("b3", eg3.sum(0) + acc * (ag3 + eg3).sum(0))
    return eP + 1e-7, edx + 1e-7, mass


def reading18(got, want, floor=1e-2, mass=None):
    """Fraction of entries within floor * max(|g*|, 1e-3 max|g*|), and, when
    the term mass is given, 1e-2 of it (a sum over samples that cancels by more
    than 100x is judged against its terms, which its rounding scales with)."""
    ref = np.maximum(np.abs(want), 1e-3 * np.abs(want).max())
    if mass is not None:
        ref = np.maximum(ref, 1e-2 * mass)
    return float(np.mean(np.abs(got - want) <= floor * ref))


def _check_grads(label, got_P, want_P, bP, got_z, want_z, bz, massP=None):
    errP, errz = np.abs(got_P - want_P), np.abs(got_z - want_z)
    assert (errP <= bP).all(), f"{label} dP: worst err/bound {(errP / bP).max():.2f}"
    assert (errz <= bz).all(), f"{label} dz: worst err/bound {(errz / bz).max():.2f}"
    fP, fz = reading18(got_P, want_P, mass=massP), reading18(got_z, want_z)
    say(f"  {label}: max err/bound dP {(errP / bP).max():.3f} dz {(errz / bz).max():.3f}; "
        f"within 1e-2 rel: dP {fP:.4f} dz {fz:.4f}")
    assert fP >= 0.99 and fz >= 0.99

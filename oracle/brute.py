"""Brute-force reference renderer in plain PyTorch FP64 on the CPU (test infrastructure).

A second, independent route to the same image and gradients as the C oracle,
for tiny scenes only.  It follows the definitions directly and takes none of
the C oracle's shortcuts:
  - the projection uses library routines (quaternion -> matrix by the Hamilton
    product formula written with torch ops, eigenvalues via torch.linalg,
    the 2x2 inverse via torch.linalg.inv);
  - the SH basis is the standard Cartesian table of real spherical harmonics
    (Condon-Shortley phase kept), written out term by term;
  - per pixel, every Gaussian whose tile rectangle contains the pixel's tile is
    gathered and ordered by (depth, index) with a sort -- no prefix scan, no
    keys, no ranges;
  - gradients come from torch.autograd, not from hand-derived formulas.
Paper passages: Sec. II-A (G(x), Sigma' = J W Sigma W^T J^T, front-to-back
blending over the depth-sorted Gaussians); tiles of Sec. IV-C.1.
"""
from __future__ import annotations

import math

import numpy as np
import torch

TILE = 16
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def sh_table(deg: int, d: torch.Tensor) -> torch.Tensor:
    """Real SH basis from the textbook Cartesian table; d is [..., 3] unit vectors.
    Returns [..., (deg+1)^2] ordered l, then m = -l..l."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 * math.sqrt(1.0 / pi))]
    if deg >= 1:
        c = math.sqrt(3.0 / (4.0 * pi))
        out += [-c * y, c * z, -c * x]
    if deg >= 2:
        out += [0.5 * math.sqrt(15.0 / pi) * x * y,
                -0.5 * math.sqrt(15.0 / pi) * y * z,
                0.25 * math.sqrt(5.0 / pi) * (2 * z * z - x * x - y * y),
                -0.5 * math.sqrt(15.0 / pi) * x * z,
                0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if deg >= 3:
        out += [-0.25 * math.sqrt(35.0 / (2 * pi)) * y * (3 * x * x - y * y),
                0.5 * math.sqrt(105.0 / pi) * x * y * z,
                -0.25 * math.sqrt(21.0 / (2 * pi)) * y * (4 * z * z - x * x - y * y),
                0.25 * math.sqrt(7.0 / pi) * z * (2 * z * z - 3 * x * x - 3 * y * y),
                -0.25 * math.sqrt(21.0 / (2 * pi)) * x * (4 * z * z - x * x - y * y),
                0.25 * math.sqrt(105.0 / pi) * z * (x * x - y * y),
                -0.25 * math.sqrt(35.0 / (2 * pi)) * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=-1)


def _quat_matrix(q: torch.Tensor) -> torch.Tensor:
    """Rotation of unit quaternions q[n][4] (w, x, y, z): the matrix of v -> q v q*,
    built by applying the Hamilton product to the three basis vectors."""
    w, x, y, z = q.unbind(-1)

    def rotate(vx, vy, vz):
        # p = q * (0, v)
        pw = -x * vx - y * vy - z * vz
        px = w * vx + y * vz - z * vy
        py = w * vy + z * vx - x * vz
        pz = w * vz + x * vy - y * vx
        # r = p * conj(q)
        rx = -pw * x + px * w - py * z + pz * y
        ry = -pw * y + py * w - pz * x + px * z
        rz = -pw * z + pz * w - px * y + py * x
        return torch.stack([rx, ry, rz], -1)

    one, zero = torch.ones_like(w), torch.zeros_like(w)
    cols = [rotate(one, zero, zero), rotate(zero, one, zero), rotate(zero, zero, one)]
    return torch.stack(cols, -1)   # [n][3][3], column j = image of e_j


def project(params: dict, deg: int, cam) -> dict:
    """Differentiable FP64 projection of every Gaussian."""
    means, ls, quats, logits, sh = (params[k] for k in ("means", "log_scales", "quats", "logits", "sh"))
    Wm = torch.tensor(np.asarray(cam.R_cw, np.float64))
    tcw = torch.tensor(np.asarray(cam.t_cw, np.float64))
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    near = float(np.float32(cam.near_z))
    limx = 1.3 * float(np.float32(cam.tan_half_fov_x))
    limy = 1.3 * float(np.float32(cam.tan_half_fov_y))

    mu = means.T                                     # [n][3]
    o = torch.sigmoid(logits)
    qn = quats.T / torch.linalg.norm(quats.T, dim=1, keepdim=True)
    R = _quat_matrix(qn)
    S2 = torch.diag_embed(torch.exp(2.0 * ls.T))
    Sigma = R @ S2 @ R.transpose(1, 2)
    t = mu @ Wm.T + tcw
    tx, ty, tz = t.unbind(-1)
    sx = torch.clamp(tx / tz, -limx, limx)
    sy = torch.clamp(ty / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * sx / tz], -1),
                     torch.stack([zero, fy / tz, -fy * sy / tz], -1)], -2)   # [n][2][3]
    T = J @ Wm
    Sp = T @ Sigma @ T.transpose(1, 2) + 0.3 * torch.eye(2, dtype=torch.float64)
    conic = torch.linalg.inv(Sp)
    ev = torch.linalg.eigvalsh(Sp.detach())
    mid = 0.5 * (ev[:, 0] + ev[:, 1])
    disc = (0.5 * (ev[:, 1] - ev[:, 0])) ** 2
    lam = mid + torch.sqrt(torch.clamp(disc, min=0.1))
    radius = torch.ceil(3.0 * torch.sqrt(lam)).to(torch.int64)
    u = fx * tx / tz + cx
    v = fy * ty / tz + cy
    centre = -(Wm.T @ tcw)
    dvec = mu - centre
    d = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
    Y = sh_table(deg, d)                                        # [n][nc]
    raw = torch.einsum("nj,jcn->nc", Y, sh) + 0.5
    rgb = torch.clamp(raw, min=0.0)
    culled = ~(tz > near)
    return dict(u=u, v=v, A=conic[:, 0, 0], B=conic[:, 0, 1], C=conic[:, 1, 1], o=o, rgb=rgb,
                depth=tz, radius=torch.where(culled, torch.zeros_like(radius), radius))


def _rect(u, v, r, W, H):
    tx, ty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    if r <= 0 or not (math.isfinite(u) and math.isfinite(v)):
        return None
    if u < -r or u >= TILE * tx + r or v < -r or v >= TILE * ty + r:
        return None
    fu, fv = math.floor(u), math.floor(v)
    x0, x1 = max(0, (fu - r) // TILE), min(tx - 1, (fu + r) // TILE)
    y0, y1 = max(0, (fv - r) // TILE), min(ty - 1, (fv + r) // TILE)
    if x0 > x1 or y0 > y1:
        return None
    return x0, x1, y0, y1


def composite(pr: dict, cam, depth_key=None) -> torch.Tensor:
    """Per-tile, per-pixel front-to-back compositing over every Gaussian whose
    rectangle contains the tile, ordered by (depth, index).  depth_key (numpy)
    overrides the ordering key (e.g. the FP32-rounded depth)."""
    W, H = cam.width, cam.height
    tx, ty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    bg = torch.tensor(np.asarray(cam.bg, np.float32).astype(np.float64))
    u_np = pr["u"].detach().numpy(); v_np = pr["v"].detach().numpy()
    r_np = pr["radius"].numpy()
    key = pr["depth"].detach().numpy() if depth_key is None else np.asarray(depth_key, np.float64)
    n = u_np.shape[0]
    rects = [_rect(float(u_np[i]), float(v_np[i]), int(r_np[i]), W, H) for i in range(n)]
    rows = []
    for tyi in range(ty):
        row = []
        for txi in range(tx):
            members = [i for i in range(n) if rects[i] is not None
                       and rects[i][0] <= txi <= rects[i][1] and rects[i][2] <= tyi <= rects[i][3]]
            members.sort(key=lambda i: (key[i], i))
            ys = torch.arange(tyi * TILE, min(tyi * TILE + TILE, H), dtype=torch.float64) + 0.5
            xs = torch.arange(txi * TILE, min(txi * TILE + TILE, W), dtype=torch.float64) + 0.5
            py, px = torch.meshgrid(ys, xs, indexing="ij")
            T = torch.ones_like(px)
            acc = torch.zeros((3,) + px.shape, dtype=torch.float64)
            done = torch.zeros_like(px, dtype=torch.bool)
            for i in members:
                dx = pr["u"][i] - px
                dy = pr["v"][i] - py
                power = -0.5 * (pr["A"][i] * dx * dx + pr["C"][i] * dy * dy) - pr["B"][i] * dx * dy
                og = pr["o"][i] * torch.exp(power)
                alpha = torch.clamp(og, max=ALPHA_MAX)
                use = (power <= 0) & (alpha >= ALPHA_MIN) & ~done
                Tn = T * (1.0 - alpha)
                stop = use & (Tn < T_MIN)
                done = done | stop
                blend = use & ~stop
                a = torch.where(blend, alpha, torch.zeros_like(alpha))
                acc = acc + pr["rgb"][i][:, None, None] * (a * T)[None]
                T = torch.where(blend, Tn, T)
            row.append(acc + T[None] * bg[:, None, None])
        rows.append(torch.cat(row, dim=2))
    return torch.cat(rows, dim=1)


def render(scene, cam, requires_grad=False):
    """Image (and, with requires_grad, the parameter tensors for autograd)."""
    params = {k: torch.tensor(np.asarray(v, np.float32).astype(np.float64), requires_grad=requires_grad)
              for k, v in scene.arrays().items()}
    pr = project(params, scene.sh_degree, cam)
    key = pr["depth"].detach().numpy().astype(np.float32).astype(np.float64)
    img = composite(pr, cam, depth_key=key)
    return img, params, pr


MLP_LAYOUT = (("W1", (64, 32)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (3, 64)), ("b3", (3,)))


def mlp_torch(x: torch.Tensor, P: torch.Tensor) -> torch.Tensor:
    """Decoder colours sigmoid(W3 ReLU(W2 ReLU(W1 x + b1) + b2) + b3) for x[S][32],
    parameters P[6467] in the order W1, b1, W2, b2, W3, b3 (row-major)."""
    sl, off = {}, 0
    for name, shape in MLP_LAYOUT:
        size = int(np.prod(shape))
        sl[name] = P[off:off + size].reshape(shape)
        off += size
    h1 = torch.relu(x @ sl["W1"].T + sl["b1"])
    h2 = torch.relu(h1 @ sl["W2"].T + sl["b2"])
    return torch.sigmoid(h2 @ sl["W3"].T + sl["b3"])


def learned_colour(means: torch.Tensor, centre, z: torch.Tensor, P: torch.Tensor) -> torch.Tensor:
    """Per-Gaussian decoder colour c[n][3] at the unit camera-to-Gaussian
    direction: x = [z; Y_0..15(d)], d = (mean - centre) / |mean - centre|.
    means[3][n], z[n][16].  Differentiable in means, z and P."""
    v = means.T - torch.as_tensor(centre, dtype=means.dtype)
    d = v / torch.linalg.norm(v, dim=1, keepdim=True)
    x = torch.cat([z, sh_table(3, d)], dim=1)
    return mlp_torch(x, P)

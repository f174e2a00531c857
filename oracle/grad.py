"""Gradient oracle for the deform-then-splat render (training direction).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the product path
never imports it.

The forward is written out again in plain PyTorch FP64 CPU ops, from the
paper, and differentiated by torch.autograd (a library primitive):

  * deformation (Sec. 4.2, Eq. 7-8): align-corners bilinear queries of the six
    planes per scale (torch grid_sample, border padding), element-wise
    product over the planes, concatenation over scales; decoder h = ReLU(W1
    f_h + b1), linear heads; X + dX, exp(log s + ds), normalise(r + dr),
    sigmoid(logit [+ dalpha]), C [+ dC];
  * projection (Sec. 3.1, Eq. 2-3): Sigma = R S S^T R^T from the quaternion
    as given (the render input is unit), Sigma' = J W Sigma W^T J^T with J
    at the frustum-clamped camera-space mean, +0.3 on the diagonal, conic =
    inverse; SH colour (real SH up to degree 3, + 0.5, clamped at 0);
  * compositing (Eq. 1, Eq. 4): each pixel walks its tile's depth-ordered
    list; alpha = min(0.99, o exp(power)); entries with alpha < 1/255 are
    skipped and the walk stops before the entry that would take T below
    1e-4; C = sum c alpha T + T_final bg.

The discrete structure is not differentiable and is held fixed: the tile
lists (which Gaussians a tile holds, in depth order) are given by the
caller (the binary32 structure of the C oracle, which the kernels match bit
for bit), and the per-pixel skip / stop / clamp decisions are taken in FP64
inside the forward under no_grad.  Pixels whose binary32 decisions sit near
a threshold are the C oracle's flagged pixels; callers give them zero loss
weight, so that the gradient compared is the derivative of one and the same
piecewise-smooth function on every side.
"""
from __future__ import annotations

import math
import types

import numpy as np
import torch

_PLANES = ((0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3))   # (a, b) axes: xy xz yz xt yt zt
F64 = torch.float64


def _t(a, grad=False):
    x = torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=F64).clone()
    return x.requires_grad_(grad)


# ------------------------------------------------------------------ deform

def deform_torch(p, planes, mlp, t: float, bmin, bmax):
    """Sec. 4.2 + Eq. 7-8 in FP64 torch.  p: dict of tensors means [3][n],
    log_scales [3][n], quats [4][n], opacity_logits [n], sh [(d+1)^2][3][n];
    planes: list over scales of six tensors [n_b][n_a][F]; mlp: dict of
    tensors w1 b1 wx bx wr br ws bs (+ wc bc wa ba).  Returns a dict of the
    render-ready set (means, scales, quats, opacity, sh)."""
    means = p["means"]
    n = means.shape[1]
    lo = torch.as_tensor(np.asarray(bmin, np.float64), dtype=F64)[:, None]
    hi = torch.as_tensor(np.asarray(bmax, np.float64), dtype=F64)[:, None]
    u = 2.0 * (means - lo) / (hi - lo) - 1.0
    u = torch.cat([u, torch.full((1, n), 2.0 * t - 1.0, dtype=F64)], 0)
    feats = []
    for lv in planes:
        f = torch.ones((lv[0].shape[2], n), dtype=F64)
        for pl, (a, b) in zip(lv, _PLANES):
            grid = torch.stack([u[a], u[b]], -1)[None, None]               # [1, 1, n, 2] (x = a, y = b)
            img = pl.permute(2, 0, 1)[None]                                  # [1, F, n_b, n_a]
            q = torch.nn.functional.grid_sample(img, grid, mode="bilinear", padding_mode="border",
                                                align_corners=True)[0, :, 0, :]   # [F, n]
            f = f * q
        feats.append(f)
    fh = torch.cat(feats, 0).T                                               # [n, F L]
    h = torch.relu(fh @ mlp["w1"].T + mlp["b1"])
    dx = h @ mlp["wx"].T + mlp["bx"]
    dr = h @ mlp["wr"].T + mlp["br"]
    ds = h @ mlp["ws"].T + mlp["bs"]
    out_means = means + dx.T
    out_scales = torch.exp(p["log_scales"] + ds.T)
    q = p["quats"] + dr.T
    out_quats = q / torch.linalg.norm(q, dim=0, keepdim=True)
    logit = p["opacity_logits"]
    if mlp.get("wa") is not None:
        logit = logit + (h @ mlp["wa"].T + mlp["ba"])[:, 0]
    sh = p["sh"]
    if mlp.get("wc") is not None:
        dc = h @ mlp["wc"].T + mlp["bc"]                                     # [n, 3 (d+1)^2]
        sh = sh + dc.T.reshape(sh.shape)
    return {"means": out_means, "scales": out_scales, "quats": out_quats,
            "opacity": torch.sigmoid(logit), "sh": sh}


# ------------------------------------------------------------------ SH colour

def sh_basis_cartesian(deg: int, d):
    """Real SH basis up to degree deg at unit directions d [3][n], as
    polynomials in (x, y, z) (index l^2 + l + m, Condon-Shortley phase):
    the expansion of K_l^m P_l^|m|(z) {cos, sin}(|m| phi) times r^l."""
    x, y, z = d[0], d[1], d[2]
    c0 = 0.5 / math.sqrt(math.pi)
    out = [torch.full_like(x, c0)]
    if deg >= 1:
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if deg >= 2:
        c2a = 0.5 * math.sqrt(15.0 / math.pi)
        c2b = 0.25 * math.sqrt(5.0 / math.pi)
        c2c = 0.25 * math.sqrt(15.0 / math.pi)
        out += [c2a * x * y, -c2a * y * z, c2b * (2 * z * z - x * x - y * y), -c2a * x * z,
                c2c * (x * x - y * y)]
    if deg >= 3:
        c3a = 0.25 * math.sqrt(35.0 / (2.0 * math.pi))
        c3b = 0.5 * math.sqrt(105.0 / math.pi)
        c3c = 0.25 * math.sqrt(21.0 / (2.0 * math.pi))
        c3d = 0.25 * math.sqrt(7.0 / math.pi)
        c3e = 0.25 * math.sqrt(105.0 / math.pi)
        out += [-c3a * y * (3 * x * x - y * y), c3b * x * y * z, -c3c * y * (4 * z * z - x * x - y * y),
                c3d * z * (2 * z * z - 3 * x * x - 3 * y * y), -c3c * x * (4 * z * z - x * x - y * y),
                c3e * z * (x * x - y * y), -c3a * x * (x * x - 3 * y * y)]
    return torch.stack(out, 0)                                               # [(d+1)^2, n]


# ------------------------------------------------------------------ projection

def project_torch(s, cam):
    """Eq. 2-3 and the SH colour in FP64 torch.  s: dict of tensors (means,
    scales, quats, opacity, sh) and int sh_degree.  Returns u, v, conic
    (A, B, C), colour [3][n], opacity."""
    V = torch.as_tensor(np.asarray(cam.viewmat, np.float64).reshape(3, 4), dtype=F64)
    W = V[:, :3]
    pc = W @ s["means"] + V[:, 3:4]
    px, py, pz = pc[0], pc[1], pc[2]
    w, x, y, z = s["quats"]
    R = torch.stack([torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
                     torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
                     torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)])])
    R = R.permute(2, 0, 1)                                                   # [n, 3, 3]
    M = R * s["scales"].T[:, None, :]
    Sig = M @ M.transpose(1, 2)
    limx = 1.3 * float(np.float32(cam.tan_half_fov_x))
    limy = 1.3 * float(np.float32(cam.tan_half_fov_y))
    rx, ry = px / pz, py / pz
    tx = torch.clamp(rx, -limx, limx) * pz
    ty = torch.clamp(ry, -limy, limy) * pz
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    zero = torch.zeros_like(pz)
    J = torch.stack([torch.stack([fx / pz, zero, -fx * tx / (pz * pz)]),
                     torch.stack([zero, fy / pz, -fy * ty / (pz * pz)])]).permute(2, 0, 1)   # [n, 2, 3]
    Tm = J @ W
    cov = Tm @ Sig @ Tm.transpose(1, 2)
    a = cov[:, 0, 0] + 0.3
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + 0.3
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det])
    u = fx * rx + cx
    v = fy * ry + cy
    campos = torch.as_tensor(np.asarray(cam.campos, np.float64), dtype=F64)[:, None]
    dvec = s["means"] - campos
    dvec = dvec / torch.linalg.norm(dvec, dim=0, keepdim=True)
    Y = sh_basis_cartesian(s["sh_degree"], dvec)                            # [(d+1)^2, n]
    k = Y.shape[0]
    col = torch.einsum("kn,kcn->cn", Y, s["sh"][:k]) + 0.5
    col = torch.clamp(col, min=0.0)
    return types.SimpleNamespace(u=u, v=v, conic=conic, colour=col, opacity=s["opacity"], depth=pz)


# ------------------------------------------------------------------ compositing

def composite_torch(pr, cam, ranges, vals):
    """Eq. 1 + Eq. 4 over the given tile lists (ranges [tiles][2] into the
    depth-ordered Gaussian ids vals).  Decisions in FP64 under no_grad."""
    W, H = int(cam.width), int(cam.height)
    tiles_x = (W + 15) // 16
    bg = torch.as_tensor(np.asarray(cam.bg, np.float64), dtype=F64)
    img = torch.zeros((3, H, W), dtype=F64)
    for tile in range(ranges.shape[0]):
        s0, s1 = int(ranges[tile, 0]), int(ranges[tile, 1])
        ty, tx = divmod(tile, tiles_x)
        xs = torch.arange(tx * 16, min(tx * 16 + 16, W), dtype=F64)
        ys = torch.arange(ty * 16, min(ty * 16 + 16, H), dtype=F64)
        py_, px_ = torch.meshgrid(ys, xs, indexing="ij")
        px_, py_ = px_.reshape(-1, 1), py_.reshape(-1, 1)                    # [P, 1]
        P = px_.shape[0]
        if s1 <= s0:
            col = bg[:, None].expand(3, P)
        else:
            ids = torch.as_tensor(np.asarray(vals[s0:s1], np.int64))
            u, v = pr.u[ids][None], pr.v[ids][None]
            A, B, C = pr.conic[0][ids][None], pr.conic[1][ids][None], pr.conic[2][ids][None]
            dx, dy = u - px_, v - py_
            power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy       # [P, L]
            raw = pr.opacity[ids][None] * torch.exp(power)
            alpha = torch.clamp(raw, max=0.99)
            with torch.no_grad():
                use = (power <= 0) & (alpha >= 1.0 / 255.0)
                a0 = torch.where(use, alpha, torch.zeros_like(alpha))
                trans = torch.cumprod(1.0 - a0, 1)                           # T after each entry
                stopped = trans < 1e-4                                        # the entry that would cross
                # entries from the first crossing on are excluded
                keep = use & (torch.cumsum(stopped.to(torch.int64), 1) == 0)
            a = torch.where(keep, alpha, torch.zeros_like(alpha))
            Tb = torch.cumprod(torch.cat([torch.ones((P, 1), dtype=F64), 1.0 - a[:, :-1]], 1), 1)   # T before
            wgt = a * Tb
            cols = pr.colour[:, ids]                                          # [3, L]
            T_final = Tb[:, -1] * (1.0 - a[:, -1])
            col = (wgt @ cols.T).T + bg[:, None] * T_final[None]
        img[:, ty * 16:ty * 16 + ys.shape[0], tx * 16:tx * 16 + xs.shape[0]] = col.reshape(3, ys.shape[0], xs.shape[0])
    return img


def render_torch(s, cam, ranges, vals):
    return composite_torch(project_torch(s, cam), cam, ranges, vals)


# ------------------------------------------------------------------ gradients

SPLAT_KEYS = ("means", "scales", "quats", "opacity", "sh")


def render_grads(splats, cam, ranges, vals, weight):
    """Gradient of L = sum(weight * image) with respect to the render-ready
    Gaussians (means, scales, quats, opacity, sh), FP64."""
    s = {k: _t(getattr(splats, k), True) for k in SPLAT_KEYS}
    s["sh_degree"] = int(splats.sh_degree)
    img = render_torch(s, cam, ranges, vals)
    loss = (torch.as_tensor(np.asarray(weight, np.float64)) * img).sum()
    # a frame that no Gaussian reaches is the background alone (Eq. 4 over
    # empty lists): the loss is constant and every gradient is zero
    if loss.requires_grad:
        loss.backward()
    return img.detach().numpy(), {k: (s[k].grad.numpy() if s[k].grad is not None else np.zeros(tuple(s[k].shape)))
                                  for k in SPLAT_KEYS}


def _leaf_inputs(g, planes, mlp):
    p = {k: _t(getattr(g, k), True) for k in CANON_KEYS}
    pl = [[_t(x, True) for x in lv] for lv in planes.planes]
    m = {k: (_t(getattr(mlp, k), True) if getattr(mlp, k, None) is not None else None) for k in MLP_KEYS}
    return p, pl, m


def _collect(p, pl, m):
    grads = {k: (p[k].grad.numpy() if p[k].grad is not None else np.zeros(tuple(p[k].shape)))
             for k in CANON_KEYS}
    grads["planes"] = [[x.grad.numpy() for x in lv] for lv in pl]
    for k in MLP_KEYS:
        if m[k] is not None:
            grads[k] = m[k].grad.numpy()
    return grads


def relu_flags(g, planes, mlp, t, rel: float = 1e-5):
    """Gaussians with a hidden unit whose FP64 pre-activation W1 f_h + b1 lies
    within rel x (sum |W1 f_h| + |b1|) of zero: there the ReLU decision of a
    binary32 forward may differ from FP64's, and the gradient with it."""
    p, pl, m = _leaf_inputs(g, planes, mlp)
    with torch.no_grad():
        feats = []
        n = p["means"].shape[1]
        lo = torch.as_tensor(np.asarray(planes.bmin, np.float64), dtype=F64)[:, None]
        hi = torch.as_tensor(np.asarray(planes.bmax, np.float64), dtype=F64)[:, None]
        u = 2.0 * (p["means"] - lo) / (hi - lo) - 1.0
        u = torch.cat([u, torch.full((1, n), 2.0 * t - 1.0, dtype=F64)], 0)
        for lv in pl:
            f = torch.ones((lv[0].shape[2], n), dtype=F64)
            for x, (a, b) in zip(lv, _PLANES):
                grid = torch.stack([u[a], u[b]], -1)[None, None]
                f = f * torch.nn.functional.grid_sample(x.permute(2, 0, 1)[None], grid, mode="bilinear",
                                                        padding_mode="border", align_corners=True)[0, :, 0, :]
            feats.append(f)
        fh = torch.cat(feats, 0).T
        pre = fh @ m["w1"].T + m["b1"]
        mag = fh.abs() @ m["w1"].abs().T + m["b1"].abs()
        return ((pre.abs() <= rel * mag).any(dim=1)).numpy()


def deform_grads(g, planes, mlp, t, gout):
    """Gradient of L = sum_k <gout[k], deform(...)[k]> (k over means, scales,
    quats, opacity, sh) with respect to the canonical Gaussians, every plane
    cell and the decoder weights, FP64."""
    p, pl, m = _leaf_inputs(g, planes, mlp)
    d = deform_torch(p, pl, m, t, planes.bmin, planes.bmax)
    loss = sum((torch.as_tensor(np.asarray(gout[k], np.float64)).reshape(d[k].shape) * d[k]).sum()
               for k in SPLAT_KEYS)
    loss.backward()
    return _collect(p, pl, m)


MLP_KEYS = ("w1", "b1", "wx", "bx", "wr", "br", "ws", "bs", "wc", "bc", "wa", "ba")
CANON_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def deform_render_grads(g, planes, mlp, t, cam, ranges, vals, weight, frozen=None):
    """Gradient of L = sum(weight * image) of the deform-then-render path
    with respect to the canonical Gaussians, every plane cell and the
    decoder weights, FP64.  Returns (image, grads) with grads["planes"] a
    list over scales of six arrays shaped like the planes.  ``frozen``
    (bool [n], optional): Gaussians whose deformed values pass no gradient
    back (they still render), e.g. those relu_flags marks."""
    p, pl, m = _leaf_inputs(g, planes, mlp)
    d = deform_torch(p, pl, m, t, planes.bmin, planes.bmax)
    if frozen is not None:
        keep = torch.as_tensor(~np.asarray(frozen, bool))
        for k in SPLAT_KEYS:
            d[k] = torch.where(keep, d[k], d[k].detach())
    d["sh_degree"] = int(g.sh_degree)
    img = render_torch(d, cam, ranges, vals)
    loss = (torch.as_tensor(np.asarray(weight, np.float64)) * img).sum()
    loss.backward()
    return img.detach().numpy(), _collect(p, pl, m)

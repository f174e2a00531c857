"""Backward kernels on the GPU against the gradient oracle (FP64 autograd of
the paper's forward with the discrete decisions held fixed).

The loss is L = sum(w * image) with w = +-1 per pixel and channel, zero on
the pixels the C oracle flags as near a compositing threshold (there the
binary32 and FP64 decisions may differ, and the gradient with them).

Bars: every gradient entry within GRAD_TOL of the largest entry of its
array (relative to max |oracle|): FP32 terms carry ~1e-7 relative error, and
the back-to-front T / (1 - alpha) recursion adds ~6e-8 per step over lists of
a few hundred entries.  And element by element, |gpu - ref| <= ELEM_ATOL max
|ref| + ELEM_RTOL |ref|, so that the small entries of arrays with a wide
range (border plane cells, rarely hit Gaussians) are checked too: a single
term carries ~1e-6 relative error, and an entry summed from terms of both
signs may cancel down to the absolute part (plane cells summed by FP32
atomics from thousands of terms: observed up to 3.7e-6 of the largest
entry)."""
import numpy as np
import pytest

import oracle
from oracle import grad as og
from paper_2310_08528_amd import g4d, synth
from tests.gpu_util import log
from tests.parity_util import chain_reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GRAD_TOL = 5e-5
ELEM_ATOL = 1e-5
ELEM_RTOL = 1e-3


def _elem_ratio(a, r):
    """Largest |a - r| / (ELEM_ATOL max|r| + ELEM_RTOL |r|) over the array (<= 1 passes)."""
    a = np.asarray(a, np.float64).reshape(np.shape(r))
    den = ELEM_ATOL * max(float(np.abs(r).max()), 1e-30) + ELEM_RTOL * np.abs(r)
    return float((np.abs(a - r) / den).max()) if np.size(r) else 0.0


def _gpu_forward(s32, cam):
    import torch
    S = g4d.DeviceSplats.from_host(s32, DEV)
    ws = g4d.RenderWorkspace(S.n, cam.width, cam.height, 64 * S.n + 4096, DEV)
    img = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=DEV)
    T = torch.empty((cam.height, cam.width), dtype=torch.float32, device=DEV)
    nc = torch.empty((cam.height, cam.width), dtype=torch.int32, device=DEV)
    g4d.render(S, cam, ws, img, T, nc)
    return S, ws, img, T, nc


def _weights(r, seed):
    rng = np.random.default_rng(seed)
    return rng.choice([-1.0, 1.0], size=r.image.shape) * (r.flag == 0)[None]


def _compare(gpu, ref, name):
    errs, elem = {}, {}
    for k in og.SPLAT_KEYS:
        a = np.asarray(gpu[k], np.float64).reshape(ref[k].shape)
        scale = max(float(np.abs(ref[k]).max()), 1e-30)
        errs[k] = float(np.abs(a - ref[k]).max() / scale)
        elem[k] = _elem_ratio(a, ref[k])
    log(f"[render bwd] {name}: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()) +
        " | per element " + " ".join(f"{k}={v:.2f}" for k, v in elem.items()))
    assert max(elem.values()) <= 1.0, elem
    return errs


def _render_bwd_case(s32, cam, name, seed=0):
    import torch
    S, ws, img, T, nc = _gpu_forward(s32, cam)
    r = oracle.render(s32, cam)
    w = _weights(r, seed)
    gimg = torch.as_tensor(w, dtype=torch.float32).to(DEV)
    grad = g4d.DeviceSplatsGrad(S.n, S.sh_degree, DEV)
    g4d.render_backward(S, cam, ws, T, nc, gimg, grad)
    torch.cuda.synchronize()
    gpu = {k: getattr(grad, k).cpu().numpy() for k in og.SPLAT_KEYS}
    _, ref = og.render_grads(s32, cam, r.ranges, r.vals, w)
    return _compare(gpu, ref, name)


@pytest.mark.parametrize("seed,deg", [(0, 0), (1, 1), (2, 2), (3, 3)])
def test_render_backward_tiny(dev, seed, deg):
    sc = synth.tiny_scene(seed, sh_degree=deg)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, 0.3)
    s32 = oracle.to_splats32(d, sc.gaussians.sh, deg)
    errs = _render_bwd_case(s32, sc.cameras[0], f"tiny seed {seed} SH{deg}")
    assert max(errs.values()) <= GRAD_TOL, errs


def test_render_backward_background_and_ragged_tiles(dev):
    """Non-zero background (the T_N bg term) and a frame whose tiles are cut
    by the image border."""
    sc = synth.tiny_scene(12, n=300, width=70, height=50, sh_degree=2)
    cam = synth.look_at_camera((0.6, 0.3, 3.0), (0.0, 0.0, 0.0), 70, 50, 50.0, bg=(0.2, 0.5, 0.9))
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, 0.3)
    s32 = oracle.to_splats32(d, sc.gaussians.sh, 2)
    errs = _render_bwd_case(s32, cam, "bg + ragged 70x50")
    assert max(errs.values()) <= GRAD_TOL, errs


def test_render_backward_small_config_subset(dev):
    """The training configuration's generator at 500 Gaussians, 64x64."""
    sc = synth.config1(plane_dist="uniform", n=500)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 64, 64, 50.0)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, 0.5)
    s32 = oracle.to_splats32(d, sc.gaussians.sh, 0)
    errs = _render_bwd_case(s32, cam, "C1 500 @ 64x64", seed=3)
    assert max(errs.values()) <= GRAD_TOL, errs


def test_render_backward_many_gaussians(dev):
    """20000 Gaussians of the 100k configuration's generator (SH degree 3) at
    96x96: more Gaussians than the kernel takes eight entries per group for,
    so the four-entry form runs (the one the 100k training step uses)."""
    sc = synth.config2(plane_dist="uniform", n=20_000, n_cams=1, n_times=1)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 96, 96, 50.0)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, 0.5)
    s32 = oracle.to_splats32(d, sc.gaussians.sh, 3)
    errs = _render_bwd_case(s32, cam, "C2 generator 20k @ 96x96", seed=5)
    assert max(errs.values()) <= GRAD_TOL, errs


def test_backward_empty_and_fully_culled(dev):
    """No Gaussians: both backward calls succeed and the deformation
    backward still clears every plane and decoder gradient.  Every Gaussian
    culled (behind the camera, inside the near plane, NaN, off-screen): every
    splat gradient is exactly zero, as the oracle's is."""
    import dataclasses
    import torch
    from tests.helpers import axis_camera, splats
    cam = axis_camera(width=40, height=24, cx=19.5, cy=11.5, bg=(0.1, 0.2, 0.3))
    log("[bwd edge] everything culled")
    s = splats([[0, 0, -2.0], [0, 0, 0.1], [np.nan, 0, 3.0], [500.0, 0, 3.0]], [[0.1] * 3] * 4,
               [[1, 0, 0, 0]] * 4, [0.9] * 4, colours=[[1, 1, 1]] * 4)
    S, ws, img, T, nc = _gpu_forward(s, cam)
    r = oracle.render(s, cam)
    assert r.K == 0
    w = _weights(r, 7)
    grad = g4d.DeviceSplatsGrad(S.n, S.sh_degree, DEV)
    for k in og.SPLAT_KEYS:
        getattr(grad, k).fill_(float("nan"))
    g4d.render_backward(S, cam, ws, T, nc, torch.as_tensor(w, dtype=torch.float32).to(DEV), grad)
    torch.cuda.synchronize()
    _, ref = og.render_grads(s, cam, r.ranges, r.vals, w)
    for k in og.SPLAT_KEYS:
        np.testing.assert_array_equal(getattr(grad, k).cpu().numpy().reshape(ref[k].shape), 0.0)
        assert not np.abs(ref[k]).max() > 0.0, k

    log("[bwd edge] empty set")
    sc = synth.tiny_scene(5, n=40, sh_degree=1)
    g = sc.gaussians
    g0 = dataclasses.replace(g, means=g.means[:, :0], log_scales=g.log_scales[:, :0], quats=g.quats[:, :0],
                             opacity_logits=g.opacity_logits[:0], sh=g.sh[..., :0])
    G, P, M = g4d.DeviceGaussians(g0, DEV), g4d.DevicePlanes(sc.planes, DEV), g4d.DeviceMLP(sc.mlp, DEV)
    assert G.n == 0
    S0 = g4d.DeviceSplats(0, 1, G.sh, DEV)
    ws0 = g4d.RenderWorkspace(1, cam.width, cam.height, 4096, DEV)
    g4d.deform(G, P, M, 0.4, S0)
    g4d.render(S0, cam, ws0, img, T, nc)
    gs = g4d.DeviceSplatsGrad(0, 1, DEV)
    g4d.render_backward(S0, cam, ws0, T, nc, torch.zeros_like(img), gs)
    gd = g4d.DeviceDeformGrad(G, P, M, DEV)
    outs = [x for lv in gd.planes for x in lv] + [v for v in gd.w.values() if v is not None]
    for x in outs:
        x.fill_(float("nan"))
    g4d.deform_backward(G, P, M, 0.4, gs, gd)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(T.cpu().numpy(), 1.0)
    for x in outs:
        assert x.numel() > 0 and not torch.any(x != 0).item()


# ---------------------------------------------------------------- deformation

def _deform_compare(gpu, ref, name, tol):
    errs = {}
    for k in og.CANON_KEYS + tuple(k for k in og.MLP_KEYS if k in ref):
        if k in ref and k in gpu and gpu[k] is not None:
            scale = max(float(np.abs(ref[k]).max()), 1e-30)
            errs[k] = float(np.abs(np.asarray(gpu[k], np.float64).reshape(ref[k].shape) - ref[k]).max() / scale)
    elem = {k: _elem_ratio(gpu[k], ref[k]) for k in errs}
    pe, pel = 0.0, 0.0
    for l, lv in enumerate(ref["planes"]):
        for q, r in enumerate(lv):
            scale = max(float(np.abs(r).max()), 1e-30)
            pe = max(pe, float(np.abs(np.asarray(gpu["planes"][l][q], np.float64) - r).max() / scale))
            pel = max(pel, _elem_ratio(gpu["planes"][l][q], r))
    errs["planes"] = pe
    elem["planes"] = pel
    log(f"[deform bwd] {name}: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()) +
        " | per element " + " ".join(f"{k}={v:.2f}" for k, v in elem.items()))
    bad = {k: v for k, v in errs.items() if v > tol}
    assert not bad, bad
    bad = {k: v for k, v in elem.items() if v > 1.0}
    assert not bad, bad


def _cell_edge_flags(means, planes, rel=4.0 * 2.0 ** -24):
    """Means strictly inside the box whose grid coordinate
    g = (x - bmin) (R - 1) / (bmax - bmin), along any axis at any scale, lies
    within rel x (R - 1) cells of an integer (the binary32 evaluation's reach:
    two roundings of g).  A mean on or beyond the border has no slope along
    that axis on either side (the border clamp), so it is not flagged."""
    x = np.asarray(means, np.float64)
    flag = np.zeros(x.shape[1], bool)
    for res in planes.res:
        for k in range(3):
            r = res[k] - 1
            inside = (x[k] > planes.bmin[k]) & (x[k] < planes.bmax[k])
            gk = (x[k] - planes.bmin[k]) * r / (planes.bmax[k] - planes.bmin[k])
            flag |= inside & (np.abs(gk - np.rint(gk)) <= rel * r + 1e-12)
    return flag


def _morton_order(means, bmin, bmax):
    from tests.test_gpu_spatial_order import _morton_order as mo
    return mo(means, bmin, bmax)


def _gpu_deform_backward(sc, t, gout):
    import torch
    G, P, M = (g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV),
               g4d.DeviceMLP(sc.mlp, DEV))
    go = g4d.DeviceSplatsGrad(G.n, G.sh_degree, DEV)
    for k in og.SPLAT_KEYS:
        getattr(go, k).copy_(torch.as_tensor(np.asarray(gout[k], np.float32)).reshape(getattr(go, k).shape))
    d = g4d.DeviceDeformGrad(G, P, M, DEV)
    g4d.deform_backward(G, P, M, t, go, d)
    torch.cuda.synchronize()
    out = {k: getattr(d, k).cpu().numpy() for k in og.CANON_KEYS}
    out.update({k: v.cpu().numpy() for k, v in d.w.items() if v is not None})
    out["planes"] = [[p.cpu().numpy() for p in lv] for lv in d.planes]
    return out


@pytest.mark.parametrize("case", ["tiny_h32", "small_config", "headline_shape", "heads_sh3", "blocks_of_64",
                                  "headline_shape_64", "heads_sh3_64", "headline_100k_morton"])
def test_deform_backward_matches_oracle(dev, case):
    """Up to 4096 Gaussians the kernel takes 16 per block, above it 64 (the
    last three cases).  headline_shape_64 runs the 100k configuration's
    variant as the benchmark does: two encoder passes (32 features, two
    scales) and the time-plane updates scattered straight into the planes
    (their rows at t exceed the block's LDS); heads_sh3_64 the 59-row head
    variant at 64 per block.  headline_100k_morton is the training leg's
    scene at full size (100k Gaussians), stored in the Morton order of its
    means as the benchmark stores it: blocks of spatially close Gaussians,
    so their plane updates go through the LDS windows."""
    if case == "headline_100k_morton":
        sc = synth.config2(plane_dist="uniform", n_cams=1, n_times=1)
        g = sc.gaussians
        o = _morton_order(g.means, sc.planes.bmin, sc.planes.bmax)
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            setattr(g, k, np.ascontiguousarray(getattr(g, k)[..., o]))
    elif case == "blocks_of_64":
        sc = synth.config1(plane_dist="uniform", n=9000)
    elif case == "headline_shape_64":
        sc = synth.config2(plane_dist="uniform", n=6000)
    elif case == "heads_sh3_64":
        sc = synth.tiny_scene(10, n=6000, sh_degree=3, colour_opacity=True)
    elif case == "tiny_h32":
        sc = synth.tiny_scene(8, n=300)
    elif case == "small_config":
        sc = synth.config1(plane_dist="uniform", n=2000)
    elif case == "headline_shape":
        sc = synth.config2(plane_dist="uniform", n=3000)
    else:
        sc = synth.tiny_scene(9, n=500, sh_degree=3, colour_opacity=True)
    g = sc.gaussians
    rng = np.random.default_rng(21)
    gout = {"means": rng.normal(size=(3, g.n)), "scales": rng.normal(size=(3, g.n)),
            "quats": rng.normal(size=(4, g.n)), "opacity": rng.normal(size=g.n),
            "sh": rng.normal(size=np.shape(g.sh))}
    t = 0.37
    # Gaussians with a hidden unit at the ReLU threshold (within binary32
    # rounding of zero) carry no loss: there the two sides' masks may differ
    flag = og.relu_flags(g, sc.planes, sc.mlp, t)
    log(f"[deform bwd] {case}: {int(flag.sum())} of {g.n} Gaussians at a ReLU threshold")
    assert flag.mean() < 0.01
    gout = {k: (v * ~flag).astype(np.float32).astype(np.float64) for k, v in gout.items()}
    gpu = _gpu_deform_backward(sc, t, gout)
    ref = og.deform_grads(g, sc.planes, sc.mlp, t, gout)
    # a mean within binary32 rounding of a plane-cell boundary may fall in
    # either cell on the two sides: the bilinear slopes (its position
    # gradient) jump there, while every plane-cell gradient is continuous
    edge = _cell_edge_flags(g.means, sc.planes)
    log(f"[deform bwd] {case}: {int(edge.sum())} of {g.n} means within rounding of a cell boundary")
    assert edge.mean() < 0.01
    gpu["means"] = np.where(edge[None, :], 0.0, gpu["means"])
    ref["means"] = np.where(edge[None, :], 0.0, ref["means"])
    _deform_compare(gpu, ref, case, 1e-4)


def test_training_step_gradients_match_oracle(dev):
    """The whole chain on the training configuration's 500-Gaussian 64x64
    subset: GPU deform + render, then render backward and deform backward,
    against the FP64 oracle's gradient of the same loss (every canonical
    parameter, every plane cell, every decoder weight)."""
    import torch
    sc = synth.config1(plane_dist="uniform", n=500)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 64, 64, 50.0)
    t = 0.5
    assert not og.relu_flags(sc.gaussians, sc.planes, sc.mlp, t).any()   # no hidden unit at the ReLU threshold
    G, P, M = (g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV),
               g4d.DeviceMLP(sc.mlp, DEV))
    S = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, DEV)
    g4d.deform(G, P, M, t, S)
    ws = g4d.RenderWorkspace(G.n, 64, 64, 64 * G.n + 4096, DEV)
    img = torch.empty((3, 64, 64), device=DEV)
    T = torch.empty((64, 64), device=DEV)
    nc = torch.empty((64, 64), dtype=torch.int32, device=DEV)
    g4d.render(S, cam, ws, img, T, nc)
    torch.cuda.synchronize()
    host = type("H", (), {k: getattr(S, k).cpu().numpy() for k in ("means", "scales", "quats", "opacity")})
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t)
    r, w, n_flag = chain_reference(d, sc.gaussians.sh, 0, host, cam, 5)
    gs = g4d.DeviceSplatsGrad(G.n, G.sh_degree, DEV)
    g4d.render_backward(S, cam, ws, T, nc, torch.as_tensor(w, dtype=torch.float32).to(DEV), gs)
    d = g4d.DeviceDeformGrad(G, P, M, DEV)
    g4d.deform_backward(G, P, M, t, gs, d)
    torch.cuda.synchronize()
    gpu = {k: getattr(d, k).cpu().numpy() for k in og.CANON_KEYS}
    gpu.update({k: v.cpu().numpy() for k, v in d.w.items() if v is not None})
    gpu["planes"] = [[p.cpu().numpy() for p in lv] for lv in d.planes]
    _, ref = og.deform_render_grads(sc.gaussians, sc.planes, sc.mlp, t, cam, r.ranges, r.vals, w)
    _deform_compare(gpu, ref, "training step C1 500 @ 64x64", 2e-4)


def test_training_step_gradients_full_size(dev):
    """The training configuration at its full size (2000 Gaussians, 800x800),
    in the launch configuration the benchmark times: every gradient against
    the FP64 oracle.  Gaussians at a ReLU threshold pass no gradient back on
    either side; flagged pixels carry no loss."""
    import time
    import torch
    sc = synth.config1(plane_dist="uniform")
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 800, 800, 50.0)
    t = 0.5
    frozen = og.relu_flags(sc.gaussians, sc.planes, sc.mlp, t)
    G, P, M = (g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV),
               g4d.DeviceMLP(sc.mlp, DEV))
    S = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, DEV)
    g4d.deform(G, P, M, t, S)
    ws = g4d.RenderWorkspace(G.n, 800, 800, 256 * G.n + 4096, DEV)
    img = torch.empty((3, 800, 800), device=DEV)
    T = torch.empty((800, 800), device=DEV)
    nc = torch.empty((800, 800), dtype=torch.int32, device=DEV)
    g4d.render(S, cam, ws, img, T, nc)
    torch.cuda.synchronize()
    host = type("H", (), {k: getattr(S, k).cpu().numpy() for k in ("means", "scales", "quats", "opacity")})
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t)
    r, w, n_flag = chain_reference(d, sc.gaussians.sh, 0, host, cam, 6)
    gs = g4d.DeviceSplatsGrad(G.n, G.sh_degree, DEV)
    g4d.render_backward(S, cam, ws, T, nc, torch.as_tensor(w, dtype=torch.float32).to(DEV), gs)
    fz = torch.as_tensor(frozen).to(DEV)
    for k in og.SPLAT_KEYS:
        getattr(gs, k)[..., fz] = 0.0
    d = g4d.DeviceDeformGrad(G, P, M, DEV)
    g4d.deform_backward(G, P, M, t, gs, d)
    torch.cuda.synchronize()
    gpu = {k: getattr(d, k).cpu().numpy() for k in og.CANON_KEYS}
    gpu.update({k: v.cpu().numpy() for k, v in d.w.items() if v is not None})
    gpu["planes"] = [[p.cpu().numpy() for p in lv] for lv in d.planes]
    t0 = time.time()
    _, ref = og.deform_render_grads(sc.gaussians, sc.planes, sc.mlp, t, cam, r.ranges, r.vals, w, frozen)
    log(f"[training full size] oracle gradient in {time.time() - t0:.1f} s; {int(frozen.sum())} Gaussians at a "
        f"ReLU threshold, {n_flag} flagged pixels")
    _deform_compare(gpu, ref, "training step C1 2000 @ 800x800", 2e-4)

"""Backward kernels on the GPU against the gradient oracle (FP64 autograd of
the paper's forward with the discrete decisions held fixed).

The loss is L = sum(w * image) with w = +-1 per pixel and channel, zero on
the pixels the C oracle flags as near a compositing threshold (there the
binary32 and FP64 decisions may differ, and the gradient with them).

Bar: every gradient entry within GRAD_TOL of the largest entry of its array
(relative to max |oracle|), derived in the design doc from the FP32 arithmetic of
the backward walk."""
import numpy as np
import pytest

import oracle
from oracle import grad as og
from paper_2310_08528_amd import g4d, synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GRAD_TOL = 5e-5


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
    errs = {}
    for k in og.SPLAT_KEYS:
        a = np.asarray(gpu[k], np.float64).reshape(ref[k].shape)
        scale = max(float(np.abs(ref[k]).max()), 1e-30)
        errs[k] = float(np.abs(a - ref[k]).max() / scale)
    log(f"[render bwd] {name}: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
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

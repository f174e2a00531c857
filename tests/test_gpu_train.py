"""The training direction end to end: the autograd binding's gradients
against the FP64 oracle, the L1 loss kernel against its definition, and a
short optimisation that fits a target rendered from perturbed parameters
(the training configuration's set-up, at reduced size)."""
import numpy as np
import pytest

import oracle
from oracle import grad as og
from paper_2310_08528_amd import autograd as ga
from paper_2310_08528_amd import g4d, synth
from tests.gpu_util import gpu_deform, log
from tests.parity_util import chain_reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_l1_loss_kernel_matches_its_definition(dev):
    import torch
    rng = np.random.default_rng(0)
    a = rng.uniform(size=(3, 37, 53)).astype(np.float32)
    b = rng.uniform(size=(3, 37, 53)).astype(np.float32)
    b[0, 0, :5] = a[0, 0, :5]                      # equal values: zero gradient
    ta, tb = torch.as_tensor(a).to(DEV), torch.as_tensor(b).to(DEV)
    loss = torch.empty((), device=DEV)
    grad = torch.empty_like(ta)
    g4d.l1_loss(ta, tb, loss, grad)
    torch.cuda.synchronize()
    d = a.astype(np.float64) - b
    assert abs(float(loss) - np.abs(d).mean()) <= 1e-6 * np.abs(d).mean()
    np.testing.assert_array_equal(grad.cpu().numpy(), (np.sign(d) / d.size).astype(np.float32))


def test_autograd_gradients_match_oracle(dev):
    import torch
    sc = synth.config1(plane_dist="uniform", n=500)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 64, 64, 50.0)
    t = 0.5
    scene = ga.Scene4D(sc.gaussians, sc.planes, sc.mlp, DEV)
    ws = g4d.RenderWorkspace(scene.n, 64, 64, 64 * scene.n + 4096, DEV)
    img = ga.render_image(scene, cam, t, ws)
    # the oracle's own structure; pixels whose decisions differ on the GPU's deformed set carry no loss
    host, _ = gpu_deform(sc, t)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t)
    r, w, _ = chain_reference(d, sc.gaussians.sh, 0, host, cam, 7)
    loss = (img * torch.as_tensor(w, dtype=torch.float32).to(DEV)).sum()
    loss.backward()
    torch.cuda.synchronize()
    _, ref = og.deform_render_grads(sc.gaussians, sc.planes, sc.mlp, t, cam, r.ranges, r.vals, w)
    worst = 0.0
    for k in og.CANON_KEYS:
        got = scene.canon[k].grad.cpu().numpy().astype(np.float64)
        worst = max(worst, np.abs(got - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-30))
    for l, lv in enumerate(scene.planes):
        for q, p in enumerate(lv):
            rq = ref["planes"][l][q]
            worst = max(worst, np.abs(p.grad.cpu().numpy() - rq).max() / max(np.abs(rq).max(), 1e-30))
    for k, v in scene.mlp.items():
        if v is not None:
            worst = max(worst, np.abs(v.grad.cpu().numpy() - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-30))
    log(f"[autograd] worst relative gradient error {worst:.2e}")
    assert worst <= 2e-4


def test_fitting_a_perturbed_target_lowers_the_loss(dev):
    """Render a target from the scene, perturb the canonical means, opacity
    and colour, and take Adam steps on the L1 loss: the loss must fall by
    more than half."""
    import torch
    sc = synth.config1(plane_dist="uniform", n=1000)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 96, 96, 50.0)
    t = 0.5
    scene = ga.Scene4D(sc.gaussians, sc.planes, sc.mlp, DEV)
    ws = g4d.RenderWorkspace(scene.n, 96, 96, 128 * scene.n + 4096, DEV)
    with torch.no_grad():
        target = ga.render_image(scene, cam, t, ws).clone()
        rng = np.random.default_rng(3)
        scene.canon["means"] += torch.as_tensor(rng.normal(0, 0.03, size=(3, scene.n)), dtype=torch.float32,
                                                device=DEV)
        scene.canon["opacity_logits"] += torch.as_tensor(rng.normal(0, 0.5, size=scene.n), dtype=torch.float32,
                                                         device=DEV)
        scene.canon["sh"] += torch.as_tensor(rng.normal(0, 0.3, size=tuple(scene.canon["sh"].shape)),
                                             dtype=torch.float32, device=DEV)
    opt = torch.optim.Adam([scene.canon["means"], scene.canon["opacity_logits"], scene.canon["sh"]], lr=5e-3)
    losses = []
    for it in range(60):
        opt.zero_grad()
        loss = ga.l1_loss(ga.render_image(scene, cam, t, ws), target)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    log(f"[fit] L1 {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]


def test_tv_kernel_matches_oracle(dev):
    import torch
    from oracle import train as ot
    sc = synth.config2(plane_dist="uniform", n=500)
    G, P, M = (g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV),
               g4d.DeviceMLP(sc.mlp, DEV))
    d = g4d.DeviceDeformGrad(G, P, M, DEV)
    rng = np.random.default_rng(2)
    base = [[rng.normal(size=tuple(p.shape)).astype(np.float32) for p in lv] for lv in d.planes]
    for lv, bl in zip(d.planes, base):
        for p, b in zip(lv, bl):
            p.copy_(torch.as_tensor(b))
    loss = torch.empty((), device=DEV)
    g4d.tv_loss(P, 0.25, loss, d)
    torch.cuda.synchronize()
    v, g = ot.tv_loss(sc.planes.planes, 0.25)
    log(f"[tv] {float(loss):.6f} vs {v:.6f}")
    assert abs(float(loss) - v) <= 1e-5 * abs(v)
    for l, lv in enumerate(d.planes):
        for q, p in enumerate(lv):
            ref = base[l][q] + g[l][q]      # the kernel adds to what is there
            np.testing.assert_allclose(p.cpu().numpy(), ref, rtol=0, atol=1e-6 * np.abs(ref).max())


def test_tv_unaligned_planes_equal_the_aligned_result(dev):
    """Planes and gradients that are not 16-byte aligned take the kernel's
    one-value-per-thread form; its gradients equal the four-channel form's
    bit for bit (the same expressions per value) and the loss agrees up to
    the order of the block sums."""
    import torch
    sc = synth.config2(plane_dist="uniform", n=500)
    G, P, M = (g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV),
               g4d.DeviceMLP(sc.mlp, DEV))
    rng = np.random.default_rng(5)
    base = [[rng.normal(size=tuple(t.shape)).astype(np.float32) for t in lv] for lv in P.tensors]

    def shifted(t):
        # a copy 4 bytes past a 16-byte boundary
        buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
        v = buf[1:].view(t.shape)
        v.copy_(t)
        return v

    def run(unaligned):
        d = g4d.DeviceDeformGrad(G, P, M, DEV)
        for lv, bl in zip(d.planes, base):
            for q, b in enumerate(bl):
                lv[q].copy_(torch.as_tensor(b))
        keep = P.tensors
        if unaligned:
            P.tensors = [[shifted(t) for t in lv] for lv in keep]
            d.planes = [[shifted(t) for t in lv] for lv in d.planes]
        loss = torch.empty((), device=DEV)
        g4d.tv_loss(P, 0.25, loss, d)
        torch.cuda.synchronize()
        P.tensors = keep
        return float(loss), [[t.cpu().numpy() for t in lv] for lv in d.planes]

    la, ga = run(False)
    lu, gu = run(True)
    log(f"[tv] aligned {la:.7f} unaligned {lu:.7f}")
    assert abs(la - lu) <= 1e-6 * abs(la)
    for lva, lvu in zip(ga, gu):
        for a, u in zip(lva, lvu):
            np.testing.assert_array_equal(a, u)


def test_adam_kernel_matches_oracle(dev):
    import torch
    from oracle import train as ot
    rng = np.random.default_rng(3)
    sizes = [1, 33, 5000, 70001]
    ps = [rng.normal(size=s).astype(np.float32) for s in sizes]
    dp = [torch.as_tensor(p).to(DEV) for p in ps]
    dm = [torch.zeros_like(p) for p in dp]
    dv = [torch.zeros_like(p) for p in dp]
    ref = [(p.astype(np.float64), np.zeros(s), np.zeros(s)) for p, s in zip(ps, sizes)]
    lrs = [1e-3, 2e-2, 1.6e-3, 1.6e-4]
    for step in range(1, 4):
        gs = [rng.normal(size=s).astype(np.float32) for s in sizes]
        dg = [torch.as_tensor(g).to(DEV) for g in gs]
        g4d.adam_step(list(zip(dp, dg, dm, dv, lrs)), step)
        ref = [ot.adam(p, g, m, v, lr, step) for (p, m, v), g, lr in zip(ref, gs, lrs)]
    torch.cuda.synchronize()
    for x, (p, _, _) in zip(dp, ref):
        np.testing.assert_allclose(x.cpu().numpy(), p, rtol=0, atol=1e-6 * max(1.0, np.abs(p).max()))


def test_training_iteration_with_tv_and_adam_kernels(dev):
    """Forward, L1 + TV, backward and the Adam kernel on every trainable
    tensor (learning rates of the appendix: 1.6e-3 for the planes, 1.6e-4 for
    the decoder): the image loss falls."""
    import torch
    sc = synth.config1(plane_dist="uniform", n=1000)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 96, 96, 50.0)
    t = 0.5
    scene = ga.Scene4D(sc.gaussians, sc.planes, sc.mlp, DEV)
    ws = g4d.RenderWorkspace(scene.n, 96, 96, 128 * scene.n + 4096, DEV)
    with torch.no_grad():
        target = ga.render_image(scene, cam, t, ws).clone()
        rng = np.random.default_rng(4)
        scene.canon["sh"] += torch.as_tensor(rng.normal(0, 0.3, size=tuple(scene.canon["sh"].shape)),
                                             dtype=torch.float32, device=DEV)
        for lv in scene.planes:
            for p in lv:
                p.mul_(torch.as_tensor(rng.uniform(0.9, 1.1, size=tuple(p.shape)), dtype=torch.float32,
                                       device=DEV))
    params = scene.parameters()
    lrs = [1.6e-3] * 5 + [1.6e-3] * sum(len(lv) for lv in scene.planes) + \
          [1.6e-4] * sum(1 for v in scene.mlp.values() if v is not None)
    moments = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    P = g4d.DevicePlanes.__new__(g4d.DevicePlanes)
    P.n_scales, P.feat, P.res, P.bmin, P.bmax, P.tensors = (scene.n_scales, scene.feat, scene.res, scene.bmin,
                                                            scene.bmax, scene.planes)
    tvl = torch.empty((), device=DEV)
    losses = []
    for step in range(1, 41):
        for p in params:
            p.grad = None
        loss = ga.l1_loss(ga.render_image(scene, cam, t, ws), target)
        loss.backward()
        grad = type("D", (), {})()
        grad.struct = lambda: _plane_grad_struct(scene)
        g4d.tv_loss(P, 0.01, tvl, grad)
        with torch.no_grad():
            g4d.adam_step([(p, p.grad, m, v, lr) for p, (m, v), lr in zip(params, moments, lrs)], step)
        losses.append(loss.item())
    log(f"[iteration] L1 {losses[0]:.4f} -> {losses[-1]:.4f}, TV {float(tvl):.3e}")
    assert losses[-1] < 0.7 * losses[0]


def _plane_grad_struct(scene):
    d = g4d.DeformGrad()
    for l, lv in enumerate(scene.planes):
        for q, p in enumerate(lv):
            d.plane[l][q] = p.grad.data_ptr()
    return d


def test_autograd_with_colour_and_opacity_heads(dev):
    """The chain with the appendix's heads: the render's SH and opacity
    gradients reach the colour and opacity heads through the deformation."""
    import torch
    sc = synth.tiny_scene(34, n=400, width=64, height=64, sh_degree=1, colour_opacity=True)
    cam, t = sc.cameras[0], 0.3
    assert not og.relu_flags(sc.gaussians, sc.planes, sc.mlp, t).any()   # no hidden unit at the ReLU threshold
    scene = ga.Scene4D(sc.gaussians, sc.planes, sc.mlp, DEV)
    ws = g4d.RenderWorkspace(scene.n, 64, 64, 64 * scene.n + 4096, DEV)
    img = ga.render_image(scene, cam, t, ws)
    host, _ = gpu_deform(sc, t)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t)
    r, w, _ = chain_reference(d, d.sh, 1, host, cam, 8)
    (img * torch.as_tensor(w, dtype=torch.float32).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    _, ref = og.deform_render_grads(sc.gaussians, sc.planes, sc.mlp, t, cam, r.ranges, r.vals, w)
    worst = {}
    for k in og.CANON_KEYS:
        got = scene.canon[k].grad.cpu().numpy().astype(np.float64)
        worst[k] = np.abs(got - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-30)
    for k in ("wc", "bc", "wa", "ba", "w1"):
        got = scene.mlp[k].grad.cpu().numpy().astype(np.float64)
        worst[k] = np.abs(got - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-30)
    log("[autograd heads] " + " ".join(f"{k}={v:.1e}" for k, v in worst.items()))
    assert max(worst.values()) <= 2e-4, worst


def test_render_image_reports_capacity_overflow(dev):
    sc = synth.config1(plane_dist="uniform", n=500)
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 64, 64, 50.0)
    scene = ga.Scene4D(sc.gaussians, sc.planes, sc.mlp, DEV)
    ws = g4d.RenderWorkspace(scene.n, 64, 64, 100, DEV)      # far too few instances
    with pytest.raises(g4d.G4DError) as e:
        ga.render_image(scene, cam, 0.5, ws)
    assert e.value.status == g4d.ECAPACITY

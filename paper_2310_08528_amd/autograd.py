"""torch.autograd binding of the deform-then-render path (training direction).

``Scene4D`` holds a scene's trainable tensors on the device (canonical
Gaussians, the HexPlane cells, the decoder weights) and ``render_image``
returns the frame at (camera, t) as a differentiable tensor: its forward is
g4d_deform + g4d_render, its backward g4d_render_backward +
g4d_deform_backward.  Marshalling only; every step runs in libg4d.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional

import numpy as np

from . import g4d

_MLP_KEYS = ("w1", "b1", "wx", "bx", "wr", "br", "ws", "bs", "wc", "bc", "wa", "ba")
_CANON_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


class Scene4D:
    """Trainable 4D scene on one device (FP32, contiguous).  Built from the
    host arrays of a synthetic scene (gaussians, planes, mlp)."""

    def __init__(self, gaussians, planes, mlp, device, requires_grad: bool = True):
        import torch
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device).requires_grad_(
            requires_grad)
        self.device = device
        self.n, self.sh_degree = int(gaussians.n), int(gaussians.sh_degree)
        self.canon = {k: f(getattr(gaussians, k)) for k in _CANON_KEYS}
        self.n_scales, self.feat = int(planes.n_scales), int(planes.feat)
        self.res = [tuple(int(x) for x in r) for r in planes.res]
        self.bmin = [float(x) for x in planes.bmin]
        self.bmax = [float(x) for x in planes.bmax]
        self.planes = [[f(p) for p in lv] for lv in planes.planes]
        self.mlp = {k: (f(getattr(mlp, k)) if getattr(mlp, k, None) is not None else None) for k in _MLP_KEYS}
        self.in_dim, self.hidden = int(mlp.in_dim), int(mlp.hidden)

    def parameters(self) -> List:
        out = [self.canon[k] for k in _CANON_KEYS]
        out += [p for lv in self.planes for p in lv]
        out += [v for v in self.mlp.values() if v is not None]
        return out

    # -- C ABI views of the current tensors
    def gaussians_struct(self) -> g4d.Gaussians:
        c = self.canon
        return g4d.Gaussians(self.n, self.sh_degree, c["means"].data_ptr(), c["log_scales"].data_ptr(),
                             c["quats"].data_ptr(), c["opacity_logits"].data_ptr(), c["sh"].data_ptr())

    def planes_struct(self) -> g4d.Planes:
        s = g4d.Planes()
        s.n_scales, s.feat = self.n_scales, self.feat
        for k in range(3):
            s.bmin[k], s.bmax[k] = self.bmin[k], self.bmax[k]
        for l in range(self.n_scales):
            for k in range(4):
                s.res[l][k] = self.res[l][k]
            for p in range(6):
                s.plane[l][p] = self.planes[l][p].data_ptr()
        return s

    def mlp_struct(self) -> g4d.MLP:
        m = g4d.MLP()
        m.in_dim, m.hidden, m.precision = self.in_dim, self.hidden, g4d.MLP_F32
        for k, v in self.mlp.items():
            setattr(m, k, v.data_ptr() if v is not None else None)
        return m


class _Frame:
    """Per-frame device state kept from the forward for the backward."""

    def __init__(self, scene: Scene4D, cam, ws: g4d.RenderWorkspace):
        import torch
        dev = scene.device
        n, d = scene.n, scene.sh_degree
        e = lambda *shape: torch.empty(shape, dtype=torch.float32, device=dev)
        self.means, self.scales, self.quats, self.opacity = e(3, n), e(3, n), e(4, n), e(n)
        self.sh = e((d + 1) ** 2, 3, n) if scene.mlp["wc"] is not None else None
        self.image = e(3, cam.height, cam.width)
        self.final_T = e(cam.height, cam.width)
        self.n_contrib = torch.empty((cam.height, cam.width), dtype=torch.int32, device=dev)
        self.ws = ws

    def splats_struct(self, scene: Scene4D) -> g4d.Splats:
        sh = self.sh if self.sh is not None else scene.canon["sh"]
        return g4d.Splats(scene.n, scene.sh_degree, self.means.data_ptr(), self.scales.data_ptr(),
                          self.quats.data_ptr(), self.opacity.data_ptr(), sh.data_ptr())


def _function():
    import torch

    class DeformRender(torch.autograd.Function):
        @staticmethod
        def forward(ctx, scene: Scene4D, cam, t: float, ws, *params):
            lib = g4d.load()
            fr = _Frame(scene, cam, ws)
            gs, ps, ms, ss = scene.gaussians_struct(), scene.planes_struct(), scene.mlp_struct(), fr.splats_struct(scene)
            cs = cam if isinstance(cam, g4d.Camera) else g4d.camera_struct(cam)
            stream = torch.cuda.current_stream().cuda_stream
            g4d.check(lib.g4d_deform(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(ms), float(t),
                                     ctypes.byref(ss), stream), "g4d_deform")
            g4d.check(lib.g4d_render(ctypes.byref(ss), ctypes.byref(cs), ctypes.byref(ws.ws),
                                     fr.image.data_ptr(), fr.final_T.data_ptr(), fr.n_contrib.data_ptr(), stream),
                      "g4d_render")
            ctx.scene, ctx.cam, ctx.t, ctx.frame = scene, cs, float(t), fr
            return fr.image.clone()

        @staticmethod
        def backward(ctx, grad_image):
            lib = g4d.load()
            scene, fr = ctx.scene, ctx.frame
            stream = torch.cuda.current_stream().cuda_stream
            gi = grad_image.contiguous()
            sg = g4d.DeviceSplatsGrad(scene.n, scene.sh_degree, scene.device)
            ss = fr.splats_struct(scene)
            g4d.check(lib.g4d_render_backward(ctypes.byref(ss), ctypes.byref(ctx.cam), ctypes.byref(fr.ws.ws),
                                              fr.final_T.data_ptr(), fr.n_contrib.data_ptr(), gi.data_ptr(),
                                              ctypes.byref(sg.struct()), stream), "g4d_render_backward")
            grads = {k: torch.empty_like(v) for k, v in scene.canon.items()}
            pgrads = [[torch.empty_like(p) for p in lv] for lv in scene.planes]
            mgrads = {k: (torch.empty_like(v) if v is not None else None) for k, v in scene.mlp.items()}
            dg = g4d.DeformGrad()
            for k in _CANON_KEYS:
                setattr(dg, k, grads[k].data_ptr())
            for l, lv in enumerate(pgrads):
                for p, x in enumerate(lv):
                    dg.plane[l][p] = x.data_ptr()
            for k, v in mgrads.items():
                setattr(dg, k, v.data_ptr() if v is not None else None)
            gs, ps, ms = scene.gaussians_struct(), scene.planes_struct(), scene.mlp_struct()
            g4d.check(lib.g4d_deform_backward(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(ms), ctx.t,
                                              ctypes.byref(sg.struct()), ctypes.byref(dg), stream),
                      "g4d_deform_backward")
            out = [grads[k] for k in _CANON_KEYS]
            out += [x for lv in pgrads for x in lv]
            out += [v for v in mgrads.values() if v is not None]
            return (None, None, None, None, *out)

    return DeformRender


_FN = None


def render_image(scene: Scene4D, cam, t: float, ws: g4d.RenderWorkspace, check: bool = True):
    """The frame of ``scene`` at time t through ``cam`` ([3][H][W], FP32),
    differentiable with respect to scene.parameters().  The workspace holds
    the frame's sorted lists until the backward: do not render with it in
    between.  With ``check`` (one stream synchronisation) a frame whose tile
    instances exceeded the workspace capacity raises G4DError(ECAPACITY)
    instead of returning an image and gradients of truncated lists."""
    global _FN
    if _FN is None:
        _FN = _function()
    img = _FN.apply(scene, cam, float(t), ws, *scene.parameters())
    if check:
        st = g4d.read_status(ws)
        if st.overflow:
            raise g4d.G4DError(g4d.ECAPACITY, f"render_image: {st.instances} instances, capacity "
                                              f"{ws.capacity}")
        if st.sort_error:
            raise g4d.G4DError(g4d.EDEVICE, "render_image: sort")
    return img


def l1_loss(image, target):
    """mean |image - target| with the hand-written kernel (value and
    gradient in one pass); differentiable with respect to image."""
    import torch

    class L1(torch.autograd.Function):
        @staticmethod
        def forward(ctx, img, tgt):
            loss = torch.empty((), dtype=torch.float32, device=img.device)
            grad = torch.empty_like(img)
            g4d.l1_loss(img.contiguous(), tgt.contiguous(), loss, grad)
            ctx.save_for_backward(grad)
            return loss

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return grad * g, None

    return L1.apply(image, target)

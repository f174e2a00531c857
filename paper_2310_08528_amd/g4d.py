"""Thin ctypes binding of libg4d (declared in include/g4d.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the deform and render path runs in the
library's HIP kernels.  There is no fallback: if libg4d.so is missing or
cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libg4d.so")

c_i32, c_i64, c_f32, c_f64, c_sz, c_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                         ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p)

MAX_SCALES = 4
TILE = 16
MAX_BATCH_JOBS = 8

OK, EINVAL, EUNSUPPORTED, ECAPACITY, EHIP, EBUSY, ENOMEM, ENOTFOUND, EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7, -8
MLP_F32, MLP_BF16 = 0, 1
EXPORT_SORTED_KEYS, EXPORT_SORTED_GIDS, EXPORT_RECT, EXPORT_DEPTH_BITS, EXPORT_RANGES, \
    EXPORT_SPLAT2D, EXPORT_DEPTH_ORDER = range(7)


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_i32), ("sh_degree", c_i32), ("means", c_p), ("log_scales", c_p),
                ("quats", c_p), ("opacity_logits", c_p), ("sh", c_p)]


class Planes(ctypes.Structure):
    _fields_ = [("n_scales", c_i32), ("feat", c_i32), ("bmin", c_f32 * 3), ("bmax", c_f32 * 3),
                ("res", (c_i32 * 4) * MAX_SCALES), ("plane", (c_p * 6) * MAX_SCALES)]


class MLP(ctypes.Structure):
    _fields_ = [("in_dim", c_i32), ("hidden", c_i32), ("precision", c_i32),
                ("w1", c_p), ("b1", c_p), ("wx", c_p), ("bx", c_p), ("wr", c_p), ("br", c_p),
                ("ws", c_p), ("bs", c_p), ("wc", c_p), ("bc", c_p), ("wa", c_p), ("ba", c_p)]


class Splats(ctypes.Structure):
    _fields_ = [("n", c_i32), ("sh_degree", c_i32), ("means", c_p), ("scales", c_p), ("quats", c_p),
                ("opacity", c_p), ("sh", c_p)]


class SplatsGrad(ctypes.Structure):
    _fields_ = [("means", c_p), ("scales", c_p), ("quats", c_p), ("opacity", c_p), ("sh", c_p)]


class DeformGrad(ctypes.Structure):
    _fields_ = [("means", c_p), ("log_scales", c_p), ("quats", c_p), ("opacity_logits", c_p), ("sh", c_p),
                ("plane", (c_p * 6) * 4),
                ("w1", c_p), ("b1", c_p), ("wx", c_p), ("bx", c_p), ("wr", c_p), ("br", c_p), ("ws", c_p),
                ("bs", c_p), ("wc", c_p), ("bc", c_p), ("wa", c_p), ("ba", c_p)]


class AdamTensor(ctypes.Structure):
    _fields_ = [("param", c_p), ("grad", c_p), ("m", c_p), ("v", c_p), ("count", c_i64), ("lr", c_f32)]


class Camera(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("viewmat", c_f32 * 12), ("fx", c_f32),
                ("fy", c_f32), ("cx", c_f32), ("cy", c_f32), ("tan_half_fov_x", c_f32),
                ("tan_half_fov_y", c_f32), ("near_plane", c_f32), ("campos", c_f32 * 3),
                ("bg", c_f32 * 3)]


class Workspace(ctypes.Structure):
    _fields_ = [("ptr", c_p), ("bytes", c_sz), ("n_max", c_i32), ("width_max", c_i32),
                ("height_max", c_i32), ("instance_capacity", c_i64)]


class DeviceStatus(ctypes.Structure):
    _fields_ = [("instances", c_i64), ("overflow", c_i32), ("sort_error", c_i32), ("visible", c_i32),
                ("tiles", c_i32), ("blend_evals", c_i64), ("blend_composited", c_i64)]


class DeformJob(ctypes.Structure):
    _fields_ = [("G", ctypes.POINTER(Gaussians)), ("P", ctypes.POINTER(Planes)),
                ("M", ctypes.POINTER(MLP)), ("t", c_f32), ("out", ctypes.POINTER(Splats))]


class Placement(ctypes.Structure):
    _fields_ = [("rotation", c_f32 * 4), ("scale", c_f32), ("translation", c_f32 * 3)]


class ComposeItem(ctypes.Structure):
    _fields_ = [("G", ctypes.POINTER(Gaussians)), ("P", ctypes.POINTER(Planes)),
                ("M", ctypes.POINTER(MLP)), ("t", c_f32), ("place", Placement)]


MAX_COMPOSE_ITEMS = 64


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", c_sz), ("max_slots", c_i32), ("use_graphs", c_i32),
                ("batch_deform", c_i32), ("max_width", c_i32), ("max_height", c_i32),
                ("instance_factor", c_f64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("rejected", c_i64), ("p50_ms", c_f64),
                ("p99_ms", c_f64), ("mean_ms", c_f64), ("max_ms", c_f64), ("wall_s", c_f64),
                ("frames_per_s", c_f64), ("batched_launches", c_i64), ("graph_replays", c_i64),
                ("eager_renders", c_i64), ("overflow_retries", c_i64), ("peak_bytes", c_sz)]


class SimConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", c_sz), ("max_slots", c_i32), ("batch_deform", c_i32), ("n_requests", c_i32),
                ("arrival_s", c_p), ("service_s", c_p), ("bytes", c_p), ("class_id", c_p), ("shape_class", c_p),
                ("overlap", c_f64)]


class SimResult(ctypes.Structure):
    _fields_ = [("p50_ms", c_f64), ("p99_ms", c_f64), ("mean_ms", c_f64), ("max_ms", c_f64),
                ("makespan_s", c_f64), ("peak_bytes", c_sz), ("max_in_flight", c_i32), ("rejected", c_i32),
                ("batched_launches", c_i64), ("buffer_reuses", c_i64), ("latency_ms", c_p), ("admit_order", c_p)]


# symbol -> (restype, argtypes); the full set declared in include/g4d.h
SIGNATURES = {
    "g4d_deform": (c_i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Planes), ctypes.POINTER(MLP), c_f32,
                           ctypes.POINTER(Splats), c_p]),
    "g4d_deform_batched": (c_i32, [ctypes.POINTER(DeformJob), c_i32, c_p]),
    "g4d_deform_compose": (c_i32, [ctypes.POINTER(ComposeItem), c_i32, ctypes.POINTER(Splats), c_p]),
    "g4d_deform_features": (c_i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Planes), c_f32, c_p, c_p]),
    "g4d_spatial_order": (c_i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(c_f32), ctypes.POINTER(c_f32),
                                  ctypes.POINTER(Workspace), c_p, c_p]),
    "g4d_render_workspace_bytes": (c_sz, [c_i32, c_i32, c_i32, c_i64]),
    "g4d_render": (c_i32, [ctypes.POINTER(Splats), ctypes.POINTER(Camera), ctypes.POINTER(Workspace), c_p, c_p,
                           c_p, c_p]),
    "g4d_deform_backward": (c_i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Planes), ctypes.POINTER(MLP), c_f32,
                                    ctypes.POINTER(SplatsGrad), ctypes.POINTER(DeformGrad), c_p]),
    "g4d_render_backward": (c_i32, [ctypes.POINTER(Splats), ctypes.POINTER(Camera), ctypes.POINTER(Workspace),
                                    c_p, c_p, c_p, ctypes.POINTER(SplatsGrad), c_p]),
    "g4d_l1_loss": (c_i32, [c_p, c_p, c_i64, c_p, c_p, c_p]),
    "g4d_tv_loss": (c_i32, [ctypes.POINTER(Planes), c_f32, c_p, ctypes.POINTER(DeformGrad), c_p]),
    "g4d_adam_step": (c_i32, [ctypes.POINTER(AdamTensor), c_i32, c_f32, c_f32, c_f32, c_i32, c_p]),
    "g4d_render_noalloc": (c_i32, [ctypes.POINTER(Splats), ctypes.POINTER(Camera), c_p, c_p, c_p,
                                   ctypes.POINTER(DeviceStatus), c_p]),
    "g4d_read_status": (c_i32, [ctypes.POINTER(Workspace), ctypes.POINTER(DeviceStatus), c_p]),
    "g4d_render_export": (c_i32, [ctypes.POINTER(Workspace), c_i32, c_i32, c_i64, c_p, c_sz, c_p]),
    "g4d_set_stage_events": (c_i32, [ctypes.POINTER(c_p), c_i32]),
    "g4d_status_string": (ctypes.c_char_p, [c_i32]),
    "g4d_last_hip_error": (c_i32, []),
    "g4d_version": (ctypes.c_char_p, []),
    "g4d_server_create": (c_i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(c_p)]),
    "g4d_server_add_scene": (c_i32, [c_p, ctypes.POINTER(Gaussians), ctypes.POINTER(Planes), ctypes.POINTER(MLP),
                                     ctypes.POINTER(c_i32)]),
    "g4d_server_submit": (c_i32, [c_p, c_i32, ctypes.POINTER(Camera), c_f32, c_p, ctypes.POINTER(ctypes.c_uint64)]),
    "g4d_server_wait": (c_i32, [c_p, ctypes.c_uint64, ctypes.POINTER(c_f64)]),
    "g4d_server_drain": (c_i32, [c_p]),
    "g4d_server_stats_get": (c_i32, [c_p, ctypes.POINTER(ServerStats)]),
    "g4d_server_reset_stats": (c_i32, [c_p]),
    "g4d_server_destroy": (c_i32, [c_p]),
    "g4d_server_simulate": (c_i32, [ctypes.POINTER(SimConfig), ctypes.POINTER(SimResult)]),
}

_lib = None


class G4DError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load().g4d_status_string(status).decode()
        if status == EHIP:
            msg += f" (hipError {load().g4d_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{status}]" if what else f"{msg} [{status}]")


def load():
    """Load libg4d.so (built by paper_2310_08528_amd.build).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_08528_amd.build`")
    # torch first: its bundled HIP runtime carries the same soname as the
    # system one, so libg4d then binds to the runtime torch already uses
    # (one runtime per process, shared streams and device pointers).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str = "") -> None:
    if status != OK:
        raise G4DError(status, what)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ------------------------------------------------------- device-side objects

class DeviceGaussians:
    """Canonical Gaussians in device tensors (SoA float32)."""

    def __init__(self, g, device):
        import torch
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        self.n, self.sh_degree = int(g.n), int(g.sh_degree)
        self.means, self.log_scales, self.quats = f(g.means), f(g.log_scales), f(g.quats)
        self.opacity_logits, self.sh = f(g.opacity_logits), f(g.sh)

    def struct(self) -> Gaussians:
        return Gaussians(self.n, self.sh_degree, _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats),
                         _ptr(self.opacity_logits), _ptr(self.sh))

    def nbytes(self) -> int:
        return sum(t.numel() * 4 for t in (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh))


class DevicePlanes:
    def __init__(self, planes, device):
        import torch
        self.n_scales, self.feat = planes.n_scales, planes.feat
        self.res = [tuple(int(x) for x in r) for r in planes.res]
        self.bmin = [float(x) for x in planes.bmin]
        self.bmax = [float(x) for x in planes.bmax]
        self.tensors = [[torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).to(device) for p in lv]
                        for lv in planes.planes]

    def struct(self) -> Planes:
        s = Planes()
        s.n_scales, s.feat = self.n_scales, self.feat
        for k in range(3):
            s.bmin[k], s.bmax[k] = self.bmin[k], self.bmax[k]
        for l in range(self.n_scales):
            for k in range(4):
                s.res[l][k] = self.res[l][k]
            for p in range(6):
                s.plane[l][p] = _ptr(self.tensors[l][p])
        return s

    def nbytes(self) -> int:
        return sum(t.numel() * 4 for lv in self.tensors for t in lv)


class DeviceMLP:
    def __init__(self, mlp, device, precision: int = MLP_F32):
        import torch
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        self.in_dim, self.hidden, self.precision = mlp.in_dim, mlp.hidden, precision
        self.w = {k: f(getattr(mlp, k)) for k in ("w1", "b1", "wx", "bx", "wr", "br", "ws", "bs")}
        # optional colour / opacity heads (absent: null pointers)
        for k in ("wc", "bc", "wa", "ba"):
            a = getattr(mlp, k, None)
            self.w[k] = None if a is None else f(a)

    @property
    def has_colour(self) -> bool:
        return self.w["wc"] is not None

    def struct(self) -> MLP:
        w = self.w
        return MLP(self.in_dim, self.hidden, self.precision, _ptr(w["w1"]), _ptr(w["b1"]), _ptr(w["wx"]),
                   _ptr(w["bx"]), _ptr(w["wr"]), _ptr(w["br"]), _ptr(w["ws"]), _ptr(w["bs"]),
                   _ptr(w["wc"]), _ptr(w["bc"]), _ptr(w["wa"]), _ptr(w["ba"]))


class DeviceSplats:
    """Render-ready Gaussians (deform output / render input) in device tensors.

    With a decoder that has a colour head, the deform writes the SH
    coefficients: pass sh=None to give the splats a buffer of their own."""

    def __init__(self, n, sh_degree, sh, device, means=None, scales=None, quats=None, opacity=None):
        import torch
        mk = lambda shape, t: (torch.empty(shape, dtype=torch.float32, device=device) if t is None
                               else torch.as_tensor(np.ascontiguousarray(t, dtype=np.float32)).to(device)
                               if not isinstance(t, torch.Tensor) else t.contiguous())
        self.n, self.sh_degree = int(n), int(sh_degree)
        self.means, self.scales = mk((3, n), means), mk((3, n), scales)
        self.quats, self.opacity = mk((4, n), quats), mk((n,), opacity)
        if sh is None:
            self.sh = torch.empty((3 * (self.sh_degree + 1) ** 2, n), dtype=torch.float32, device=device)
        else:
            self.sh = sh if isinstance(sh, torch.Tensor) else torch.as_tensor(
                np.ascontiguousarray(sh, dtype=np.float32)).to(device)

    @classmethod
    def from_host(cls, s, device):
        return cls(s.n, s.sh_degree, s.sh, device, s.means, s.scales, s.quats, s.opacity)

    def struct(self) -> Splats:
        return Splats(self.n, self.sh_degree, _ptr(self.means), _ptr(self.scales), _ptr(self.quats),
                      _ptr(self.opacity), _ptr(self.sh))


def camera_struct(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    v = np.asarray(cam.viewmat, dtype=np.float32).reshape(-1)
    for i in range(12):
        c.viewmat[i] = float(v[i])
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.tan_half_fov_x, c.tan_half_fov_y, c.near_plane = cam.tan_half_fov_x, cam.tan_half_fov_y, cam.near
    for i in range(3):
        c.campos[i] = float(cam.campos[i])
        c.bg[i] = float(cam.bg[i])
    return c


def workspace_bytes(n: int, width: int, height: int, capacity: int) -> int:
    return int(load().g4d_render_workspace_bytes(n, width, height, capacity))


class RenderWorkspace:
    """Caller-owned render scratch (a torch uint8 tensor on the device)."""

    def __init__(self, n_max: int, width_max: int, height_max: int, capacity: int, device):
        import torch
        nbytes = workspace_bytes(n_max, width_max, height_max, capacity)
        if nbytes == 0:
            raise G4DError(EINVAL, "workspace size")
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ws = Workspace(aligned, nbytes, n_max, width_max, height_max, capacity)
        self.n_max, self.width_max, self.height_max, self.capacity = n_max, width_max, height_max, capacity

    def fits(self, n, width, height) -> bool:
        return n <= self.n_max and width <= self.width_max and height <= self.height_max


# --------------------------------------------------------------- the calls

def deform(G: DeviceGaussians, P: DevicePlanes, M: DeviceMLP, t: float, out: DeviceSplats, stream=None):
    gs, ps, ms, os_ = G.struct(), P.struct(), M.struct(), out.struct()
    check(load().g4d_deform(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(ms), float(t), ctypes.byref(os_),
                            _stream(stream)), "g4d_deform")


def deform_batched(jobs, stream=None):
    """jobs: list of (DeviceGaussians, DevicePlanes, DeviceMLP, t, DeviceSplats)."""
    keep = []
    arr = (DeformJob * len(jobs))()
    for i, (G, P, M, t, out) in enumerate(jobs):
        gs, ps, ms, os_ = G.struct(), P.struct(), M.struct(), out.struct()
        keep += [gs, ps, ms, os_]
        arr[i] = DeformJob(ctypes.pointer(gs), ctypes.pointer(ps), ctypes.pointer(ms), float(t), ctypes.pointer(os_))
    check(load().g4d_deform_batched(arr, len(jobs), _stream(stream)), "g4d_deform_batched")


def placement(rotation=(1.0, 0.0, 0.0, 0.0), scale=1.0, translation=(0.0, 0.0, 0.0)) -> Placement:
    """A scene's placement in a composition: quaternion (w, x, y, z), uniform
    scale, translation."""
    p = Placement()
    for k in range(4):
        p.rotation[k] = float(rotation[k])
    p.scale = float(scale)
    for k in range(3):
        p.translation[k] = float(translation[k])
    return p


def deform_compose(items, out: DeviceSplats, stream=None):
    """items: list of (DeviceGaussians, DevicePlanes, DeviceMLP, t, placement
    or None).  Writes every item's deformed, placed set into its index range
    of ``out`` (out.n = sum of the items' n; out.sh a buffer of its own)."""
    keep = []
    arr = (ComposeItem * len(items))()
    for i, (G, P, M, t, pl) in enumerate(items):
        gs, ps, ms = G.struct(), P.struct(), M.struct()
        keep += [gs, ps, ms]
        arr[i] = ComposeItem(ctypes.pointer(gs), ctypes.pointer(ps), ctypes.pointer(ms), float(t),
                             pl if pl is not None else placement())
    os_ = out.struct()
    check(load().g4d_deform_compose(arr, len(items), ctypes.byref(os_), _stream(stream)), "g4d_deform_compose")


def spatial_order(G: DeviceGaussians, bmin, bmax, ws: "RenderWorkspace", stream=None):
    """The Morton order of G's canonical means over the box [bmin, bmax] (an
    int32 device tensor [n]: the index of the i-th Gaussian of the order)."""
    import torch
    order = torch.empty(max(G.n, 1), dtype=torch.int32, device=G.means.device)
    gs = G.struct()
    lo = (c_f32 * 3)(*[float(v) for v in bmin])
    hi = (c_f32 * 3)(*[float(v) for v in bmax])
    check(load().g4d_spatial_order(ctypes.byref(gs), lo, hi, ctypes.byref(ws.ws), _ptr(order), _stream(stream)),
          "g4d_spatial_order")
    return order[:G.n]


def store_in_order(G: DeviceGaussians, order):
    """Permute every per-Gaussian array of G in place into `order` (a
    one-time data-layout step; the tensors keep their storage)."""
    idx = order.long()
    for t in (G.means, G.log_scales, G.quats, G.opacity_logits, G.sh):
        t.copy_(t[..., idx])


def deform_features(G: DeviceGaussians, P: DevicePlanes, t: float, features, stream=None):
    gs, ps = G.struct(), P.struct()
    check(load().g4d_deform_features(ctypes.byref(gs), ctypes.byref(ps), float(t), _ptr(features),
                                     _stream(stream)), "g4d_deform_features")


def render(S: DeviceSplats, cam, ws: RenderWorkspace, image, final_T=None, n_contrib=None, stream=None):
    ss = S.struct()
    cs = cam if isinstance(cam, Camera) else camera_struct(cam)
    check(load().g4d_render(ctypes.byref(ss), ctypes.byref(cs), ctypes.byref(ws.ws), _ptr(image), _ptr(final_T),
                            _ptr(n_contrib), _stream(stream)), "g4d_render")


def render_noalloc(S: DeviceSplats, cam, image, final_T=None, n_contrib=None, status=True, stream=None):
    """g4d_render with the library's fixed device array as its workspace (no
    allocation).  status=True waits for the stream and returns the frame's
    DeviceStatus (raising on an overflow); status=False only enqueues."""
    ss = S.struct()
    cs = cam if isinstance(cam, Camera) else camera_struct(cam)
    st = DeviceStatus() if status else None
    check(load().g4d_render_noalloc(ctypes.byref(ss), ctypes.byref(cs), _ptr(image), _ptr(final_T),
                                    _ptr(n_contrib), ctypes.byref(st) if st is not None else None,
                                    _stream(stream)), "g4d_render_noalloc")
    return st


class DeviceSplatsGrad:
    """Gradients with respect to render-ready Gaussians, device tensors."""

    def __init__(self, n, sh_degree, device):
        import torch
        e = lambda *shape: torch.empty(shape, dtype=torch.float32, device=device)
        self.n, self.sh_degree = int(n), int(sh_degree)
        self.means, self.scales, self.quats = e(3, n), e(3, n), e(4, n)
        self.opacity, self.sh = e(n), e((sh_degree + 1) ** 2, 3, n)

    def struct(self) -> SplatsGrad:
        return SplatsGrad(_ptr(self.means), _ptr(self.scales), _ptr(self.quats), _ptr(self.opacity), _ptr(self.sh))


def render_backward(S: DeviceSplats, cam, ws: RenderWorkspace, final_T, n_contrib, grad_image,
                    grad: DeviceSplatsGrad, stream=None):
    """dL/d(render-ready Gaussians) through the last render on ``ws``."""
    ss, gs = S.struct(), grad.struct()
    cs = cam if isinstance(cam, Camera) else camera_struct(cam)
    check(load().g4d_render_backward(ctypes.byref(ss), ctypes.byref(cs), ctypes.byref(ws.ws), _ptr(final_T),
                                     _ptr(n_contrib), _ptr(grad_image), ctypes.byref(gs), _stream(stream)),
          "g4d_render_backward")


class DeviceDeformGrad:
    """Gradients of the deformation's inputs (canonical Gaussians, plane
    cells, decoder weights), device tensors shaped like the inputs."""

    def __init__(self, G: DeviceGaussians, P: DevicePlanes, M: DeviceMLP, device):
        import torch
        e = lambda t: torch.empty_like(t) if t is not None else None
        self.means, self.log_scales, self.quats = e(G.means), e(G.log_scales), e(G.quats)
        self.opacity_logits, self.sh = e(G.opacity_logits), e(G.sh)
        self.planes = [[e(p) for p in lv] for lv in P.tensors]
        self.w = {k: e(v) for k, v in M.w.items()}

    def struct(self) -> DeformGrad:
        d = DeformGrad()
        d.means, d.log_scales, d.quats = _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats)
        d.opacity_logits, d.sh = _ptr(self.opacity_logits), _ptr(self.sh)
        for l, lv in enumerate(self.planes):
            for p, t in enumerate(lv):
                d.plane[l][p] = _ptr(t)
        for k, v in self.w.items():
            setattr(d, k, _ptr(v))
        return d


def deform_backward(G: DeviceGaussians, P: DevicePlanes, M: DeviceMLP, t: float, grad_out: DeviceSplatsGrad,
                    grad: DeviceDeformGrad, stream=None):
    """dL/d(canonical Gaussians, plane cells, decoder weights) from
    dL/d(render-ready set)."""
    gs, ps, ms, go, gd = G.struct(), P.struct(), M.struct(), grad_out.struct(), grad.struct()
    check(load().g4d_deform_backward(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(ms), float(t),
                                     ctypes.byref(go), ctypes.byref(gd), _stream(stream)), "g4d_deform_backward")


def l1_loss(image, target, loss=None, grad=None, stream=None):
    """mean |image - target| into the device scalar ``loss`` and its gradient
    sign(image - target) / count into ``grad`` (either may be None)."""
    check(load().g4d_l1_loss(_ptr(image), _ptr(target), int(image.numel()), _ptr(loss), _ptr(grad),
                             _stream(stream)), "g4d_l1_loss")


def tv_loss(P: DevicePlanes, weight: float, loss=None, grad: Optional["DeviceDeformGrad"] = None, stream=None):
    """Grid total variation of the planes into ``loss``; adds its gradient to
    grad.planes."""
    ps = P.struct()
    gd = grad.struct() if grad is not None else None
    check(load().g4d_tv_loss(ctypes.byref(ps), float(weight), _ptr(loss),
                             ctypes.byref(gd) if gd is not None else None, _stream(stream)), "g4d_tv_loss")


def adam_step(tensors, step: int, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """tensors: list of (param, grad, m, v, lr) device tensors (FP32,
    contiguous, same sizes)."""
    arr = (AdamTensor * len(tensors))()
    for i, (p, g, m, v, lr) in enumerate(tensors):
        arr[i] = AdamTensor(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(p.numel()), float(lr))
    check(load().g4d_adam_step(arr, len(tensors), float(beta1), float(beta2), float(eps), int(step),
                               _stream(stream)), "g4d_adam_step")


def read_status(ws: RenderWorkspace, stream=None) -> DeviceStatus:
    st = DeviceStatus()
    check(load().g4d_read_status(ctypes.byref(ws.ws), ctypes.byref(st), _stream(stream)), "g4d_read_status")
    return st


def export(ws: RenderWorkspace, kind: int, n: int, k: int, dst, stream=None):
    check(load().g4d_render_export(ctypes.byref(ws.ws), int(kind), int(n), int(k), _ptr(dst),
                                   dst.numel() * dst.element_size(), _stream(stream)), "g4d_render_export")


def set_stage_events(events):
    """events: list of 9 raw hipEvent_t handles (int or None), or None to stop."""
    if events is None:
        check(load().g4d_set_stage_events(None, 0), "g4d_set_stage_events")
        return
    arr = (c_p * len(events))(*[e or None for e in events])
    check(load().g4d_set_stage_events(arr, len(events)), "g4d_set_stage_events")


def version() -> str:
    return load().g4d_version().decode()


# ------------------------------------------------------------------ serving

class Server:
    """Continuous-batching request loop (g4d_server_*).  Scenes are copied
    into server-owned device memory; images go to caller device tensors."""

    def __init__(self, hbm_budget: int, max_slots: int = 8, use_graphs: bool = True, batch_deform: bool = True,
                 max_width: int = 1352, max_height: int = 1014, instance_factor: float = 64.0):
        import torch  # noqa: F401  (one HIP runtime per process)
        self.lib = load()
        cfg = ServerConfig(int(hbm_budget), int(max_slots), int(bool(use_graphs)), int(bool(batch_deform)),
                           int(max_width), int(max_height), float(instance_factor))
        h = c_p()
        check(self.lib.g4d_server_create(ctypes.byref(cfg), ctypes.byref(h)), "g4d_server_create")
        self.h = h

    def add_scene(self, G: DeviceGaussians, P: DevicePlanes, M: DeviceMLP) -> int:
        gs, ps, ms = G.struct(), P.struct(), M.struct()
        sid = c_i32()
        check(self.lib.g4d_server_add_scene(self.h, ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(ms),
                                            ctypes.byref(sid)), "g4d_server_add_scene")
        return sid.value

    def submit(self, scene: int, cam, t: float, out) -> int:
        cs = cam if isinstance(cam, Camera) else camera_struct(cam)
        tk = ctypes.c_uint64()
        check(self.lib.g4d_server_submit(self.h, int(scene), ctypes.byref(cs), float(t), _ptr(out),
                                         ctypes.byref(tk)), "g4d_server_submit")
        return tk.value

    def wait(self, ticket: int) -> float:
        ms = c_f64()
        check(self.lib.g4d_server_wait(self.h, ctypes.c_uint64(ticket), ctypes.byref(ms)), "g4d_server_wait")
        return ms.value

    def drain(self):
        check(self.lib.g4d_server_drain(self.h), "g4d_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        check(self.lib.g4d_server_stats_get(self.h, ctypes.byref(st)), "g4d_server_stats_get")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def reset_stats(self):
        check(self.lib.g4d_server_reset_stats(self.h), "g4d_server_reset_stats")

    def close(self):
        if getattr(self, "h", None):
            check(self.lib.g4d_server_destroy(self.h), "g4d_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(arrival_s, service_s, nbytes, class_id, shape_class, hbm_budget, max_slots, batch_deform=True,
             overlap=0.5):
    """Run the serving scheduler on a simulated device (no GPU)."""
    n = len(arrival_s)
    a = np.ascontiguousarray(arrival_s, dtype=np.float64)
    sv = np.ascontiguousarray(service_s, dtype=np.float64)
    by = np.ascontiguousarray(nbytes, dtype=np.uint64)
    ci = np.ascontiguousarray(class_id, dtype=np.int32)
    sc = np.ascontiguousarray(shape_class, dtype=np.int32)
    lat = np.full(n, -2.0)
    order = np.full(n, -1, dtype=np.int32)
    cfg = SimConfig(int(hbm_budget), int(max_slots), int(bool(batch_deform)), n,
                    a.ctypes.data, sv.ctypes.data, by.ctypes.data, ci.ctypes.data, sc.ctypes.data, float(overlap))
    res = SimResult()
    res.latency_ms = lat.ctypes.data
    res.admit_order = order.ctypes.data
    check(load().g4d_server_simulate(ctypes.byref(cfg), ctypes.byref(res)), "g4d_server_simulate")
    out = {k: getattr(res, k) for k, _ in SimResult._fields_ if k not in ("latency_ms", "admit_order")}
    out["latency_ms"] = lat
    out["admit_order"] = order
    return out

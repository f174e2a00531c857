"""Seeded synthetic inputs for the deform-then-splat render.

This module produces *data only*: canonical Gaussians, HexPlane feature
planes, deformation-MLP weights, pinhole cameras, timestamps and request
arrival traces.  It holds none of the method's arithmetic (no interpolation,
no MLP evaluation, no projection, no compositing), so both the HIP path and
the CPU oracle can consume the same inputs without sharing any method code.

Every workload is drawn from ``numpy.random.default_rng`` streams spawned from
``SeedSequence(1000 + config_id)`` in a fixed order, one child stream per
field, so that each field is reproducible on its own.

Scene shapes follow the paper's workloads: D-NeRF-like object scenes at
800x800 with up to ~100k Gaussians (Sec. 5.1, Fig. on FPS vs. number of
Gaussians), Neu3D-like real scenes at 1352x1014 (Tab. 3, App. A.1), and the
HexPlane field of Sec. 4.2 (six planes per scale, ``h`` features, spatial
resolutions upsampled per scale, Eq. 7).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

# Order of the six planes of one scale (Sec. 4.2, Eq. 7): (a, b) axis pairs,
# with axis indices 0=x, 1=y, 2=z, 3=t.  A plane is stored channels-last as
# [n_b][n_a][F] float32.
PLANE_AXES = ((0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3))
PLANE_NAMES = ("xy", "xz", "yz", "xt", "yt", "zt")

_STREAMS = ("means", "log_scales", "quats", "opacity", "sh", "planes", "mlp",
            "cameras", "timestamps", "arrivals", "extra")


@dataclasses.dataclass
class Gaussians:
    """Canonical 3D Gaussians, structure-of-arrays, float32 (Sec. 3.1).

    means [3][n]; log_scales [3][n]; quats [4][n] in (w, x, y, z) order;
    opacity_logits [n]; sh [(d+1)^2][3][n] real-SH coefficients per channel.
    """
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])


@dataclasses.dataclass
class Planes:
    """Multi-resolution HexPlane feature planes (Sec. 4.2, Eq. 7).

    planes[l][p] is float32 [n_b][n_a][feat] for plane p in PLANE_AXES order.
    res[l] = (Rx, Ry, Rz, Rt).  bmin/bmax: axis-aligned bounds that map the
    canonical means onto [-1, 1] for the plane lookups.
    """
    feat: int
    res: List[Sequence[int]]
    planes: List[List[np.ndarray]]
    bmin: np.ndarray
    bmax: np.ndarray

    @property
    def n_scales(self) -> int:
        return len(self.planes)

    @property
    def in_dim(self) -> int:
        return self.feat * self.n_scales

    def nbytes(self) -> int:
        return sum(p.nbytes for lv in self.planes for p in lv)


@dataclasses.dataclass
class MLP:
    """Deformation decoder weights (Sec. 4.2): one hidden layer and three heads.

    w1 [hidden][in_dim], b1 [hidden]; wx [3][hidden], bx [3];
    wr [4][hidden], br [4]; ws [3][hidden], bs [3].  float32, row-major.
    Optional heads of the appendix's colour and opacity deformation:
    wc [3 (d+1)^2][hidden], bc [3 (d+1)^2] (one row per SH coefficient, in
    the colour array's order) and wa [1][hidden], ba [1]; None when absent.
    """
    w1: np.ndarray
    b1: np.ndarray
    wx: np.ndarray
    bx: np.ndarray
    wr: np.ndarray
    br: np.ndarray
    ws: np.ndarray
    bs: np.ndarray
    wc: Optional[np.ndarray] = None
    bc: Optional[np.ndarray] = None
    wa: Optional[np.ndarray] = None
    ba: Optional[np.ndarray] = None

    @property
    def in_dim(self) -> int:
        return int(self.w1.shape[1])

    @property
    def hidden(self) -> int:
        return int(self.w1.shape[0])


@dataclasses.dataclass
class Camera:
    """Pinhole view M = [R, T] (Sec. 4.1) with OpenCV axes (x right, y down,
    z forward).  viewmat is the row-major 3x4 world-to-camera matrix.
    Pixel (px, py) is sampled at image coordinates (px, py)."""
    width: int
    height: int
    viewmat: np.ndarray          # float32 [3][4]
    fx: float
    fy: float
    cx: float
    cy: float
    campos: np.ndarray           # float32 [3], camera centre in world space
    tan_half_fov_x: float
    tan_half_fov_y: float
    near: float = 0.2
    bg: Sequence[float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Scene:
    gaussians: Gaussians
    planes: Planes
    mlp: MLP
    cameras: List[Camera]
    timestamps: np.ndarray
    name: str = ""


def _streams(config_id: int) -> Dict[str, np.random.Generator]:
    ss = np.random.SeedSequence(1000 + int(config_id))
    kids = ss.spawn(len(_STREAMS))
    return {k: np.random.default_rng(s) for k, s in zip(_STREAMS, kids)}


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# ----------------------------------------------------------------- Gaussians

def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh_coeffs(rng, n, degree, kind):
    k = (degree + 1) ** 2
    if kind == "rgb0":
        # Degree-0 colour drawn uniformly: the DC coefficient is uniform on
        # [-sqrt(pi), sqrt(pi)], which spans colours [0, 1] after the usual
        # DC normalisation and +0.5 offset.
        assert degree == 0
        lim = math.sqrt(math.pi)
        return rng.uniform(-lim, lim, size=(1, 3, n))
    return rng.normal(0.0, 0.2, size=(k, 3, n))


def make_gaussians(rng: Dict[str, np.random.Generator], n: int, means: np.ndarray,
                   sh_degree: int, sh_kind: str) -> Gaussians:
    return Gaussians(
        means=_f32(means),
        log_scales=_f32(rng["log_scales"].normal(-3.0, 0.5, size=(3, n))),
        quats=_f32(_unit_quats(rng["quats"], n)),
        opacity_logits=_f32(rng["opacity"].normal(0.0, 1.0, size=n)),
        sh=_f32(_sh_coeffs(rng["sh"], n, sh_degree, sh_kind)),
        sh_degree=sh_degree,
    )


def means_cube(rng, n, half=1.0):
    return rng.uniform(-half, half, size=(3, n))


def means_shell(rng, n, radius=1.0, fill=0.10, noise=0.02):
    """Noisy sphere shell plus uniform fill of the ball (object-scale scene)."""
    n_fill = int(round(fill * n))
    n_shell = n - n_fill
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = np.empty(n)
    r[:n_shell] = radius + rng.normal(0.0, noise, size=n_shell)
    r[n_shell:] = radius * rng.uniform(0.0, 1.0, size=n_fill) ** (1.0 / 3.0)
    return d * r


def means_box_cluster(rng, n, frac_box=0.70):
    """Wide box [-5,5]x[-2,2]x[-5,5] (y up) plus a dense cluster at the origin."""
    n_box = int(round(frac_box * n))
    out = np.empty((3, n))
    out[0, :n_box] = rng.uniform(-5.0, 5.0, size=n_box)
    out[1, :n_box] = rng.uniform(-2.0, 2.0, size=n_box)
    out[2, :n_box] = rng.uniform(-5.0, 5.0, size=n_box)
    out[:, n_box:] = rng.normal(0.0, 0.5, size=(3, n - n_box))
    return out


# -------------------------------------------------------------------- planes

def make_planes(rng: np.random.Generator, means: np.ndarray, feat: int,
                spatial: Sequence[int], temporal: int, dist: str = "normal",
                spatial_xyz: Optional[Sequence[Sequence[int]]] = None) -> Planes:
    """Planes for each scale l with spatial resolution spatial[l] on x, y, z
    and an un-upsampled temporal resolution.  dist='normal' draws N(0, 0.1);
    dist='uniform' draws U(0.5, 1.5) so that the per-plane product stays O(1)
    and varies per Gaussian (used by parity tests); dist='zero' gives zeros;
    dist='one' gives ones."""
    res, planes = [], []
    for li, s in enumerate(spatial):
        r = tuple(spatial_xyz[li]) if spatial_xyz is not None else (s, s, s)
        r = (int(r[0]), int(r[1]), int(r[2]), int(temporal))
        res.append(r)
        level = []
        for (a, b) in PLANE_AXES:
            shape = (r[b], r[a], feat)
            if dist == "normal":
                v = rng.normal(0.0, 0.1, size=shape)
            elif dist == "uniform":
                v = rng.uniform(0.5, 1.5, size=shape)
            elif dist == "zero":
                v = np.zeros(shape)
            elif dist == "one":
                v = np.ones(shape)
            else:
                raise ValueError(dist)
            level.append(_f32(v))
        planes.append(level)
    m = np.asarray(means, dtype=np.float64)
    bmin = m.min(axis=1)
    bmax = m.max(axis=1)
    # keep a non-degenerate box on every axis
    span = np.maximum(bmax - bmin, 1e-6)
    bmax = bmin + span
    return Planes(feat=feat, res=res, planes=planes, bmin=_f32(bmin), bmax=_f32(bmax))


def make_mlp(rng: np.random.Generator, in_dim: int, hidden: int, zero_bias: bool = False,
             zero: bool = False, colour_rows: int = 0, opacity: bool = False) -> MLP:
    """PyTorch-default uniform init.  The colour (colour_rows > 0) and
    opacity heads are drawn after the base weights, which therefore do not
    depend on whether they are present."""
    def lin(fan_out, fan_in):
        k = 1.0 / math.sqrt(fan_in)
        w = rng.uniform(-k, k, size=(fan_out, fan_in))
        b = rng.uniform(-k, k, size=fan_out)
        if zero:
            w = np.zeros_like(w)
        if zero or zero_bias:
            b = np.zeros_like(b)
        return _f32(w), _f32(b)
    w1, b1 = lin(hidden, in_dim)
    wx, bx = lin(3, hidden)
    wr, br = lin(4, hidden)
    ws, bs = lin(3, hidden)
    m = MLP(w1=w1, b1=b1, wx=wx, bx=bx, wr=wr, br=br, ws=ws, bs=bs)
    if colour_rows:
        m.wc, m.bc = lin(colour_rows, hidden)
    if opacity:
        m.wa, m.ba = lin(1, hidden)
    return m


def sh_rows(sh_degree: int) -> int:
    """SH coefficients per Gaussian: 3 colour channels x (d+1)^2 bands."""
    return 3 * (sh_degree + 1) ** 2


# ------------------------------------------------------------------- cameras

def look_at_camera(pos, target, width, height, fov_x_deg=50.0, up=(0.0, 1.0, 0.0),
                   near=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    pos = np.asarray(pos, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    z = target - pos
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ pos
    V = np.concatenate([R, t[:, None]], axis=1)
    tan_x = math.tan(math.radians(fov_x_deg) / 2.0)
    fx = (width / 2.0) / tan_x
    fy = fx
    tan_y = (height / 2.0) / fy
    return Camera(width=int(width), height=int(height), viewmat=_f32(V), fx=float(np.float32(fx)),
                  fy=float(np.float32(fy)), cx=float(np.float32((width - 1) / 2.0)),
                  cy=float(np.float32((height - 1) / 2.0)), campos=_f32(pos),
                  tan_half_fov_x=float(np.float32(tan_x)), tan_half_fov_y=float(np.float32(tan_y)),
                  near=float(np.float32(near)), bg=tuple(float(np.float32(b)) for b in bg))


def ring_cameras(n_cams, radius, width, height, height_y=0.0, fov_x_deg=50.0):
    cams = []
    for k in range(n_cams):
        th = 2.0 * math.pi * k / n_cams
        pos = (radius * math.sin(th), height_y, radius * math.cos(th))
        cams.append(look_at_camera(pos, (0.0, 0.0, 0.0), width, height, fov_x_deg))
    return cams


def pinhole_camera(width, height, fx, fy, cx, cy, viewmat=None, campos=None,
                   tan_half_fov_x=None, tan_half_fov_y=None, near=0.2, bg=(0, 0, 0)) -> Camera:
    """Camera with explicit intrinsics (identity pose unless given)."""
    V = np.zeros((3, 4)) if viewmat is None else np.asarray(viewmat, dtype=np.float64)
    if viewmat is None:
        V[:, :3] = np.eye(3)
    if campos is None:
        R = V[:, :3]
        campos = -R.T @ V[:, 3]
    tx = (width / 2.0) / fx if tan_half_fov_x is None else tan_half_fov_x
    ty = (height / 2.0) / fy if tan_half_fov_y is None else tan_half_fov_y
    return Camera(width=int(width), height=int(height), viewmat=_f32(V), fx=float(np.float32(fx)),
                  fy=float(np.float32(fy)), cx=float(np.float32(cx)), cy=float(np.float32(cy)),
                  campos=_f32(campos), tan_half_fov_x=float(np.float32(tx)),
                  tan_half_fov_y=float(np.float32(ty)), near=float(np.float32(near)),
                  bg=tuple(float(np.float32(b)) for b in bg))


# ------------------------------------------------------------------- configs

CONFIG_NOTES = {
    1: "2k Gaussians in [-1,1]^3, SH0, planes 32/t8 F16, MLP 16-64-10, 128x128, t=0.5",
    2: "100k Gaussians on a noisy shell, SH3, planes 64+128/t25 F32, MLP 64-64-10, 800x800, "
       "20 ring cameras x 20 timestamps",
    4: "300k Gaussians, box + cluster, SH3, planes 64/128/256 t150 F32, MLP 96-128-10, 1352x1014",
}


def config1(plane_dist: str = "normal", n: int = 2000, zero_field: bool = False) -> Scene:
    rng = _streams(1)
    means = means_cube(rng["means"], n)
    g = make_gaussians(rng, n, means, 0, "rgb0")
    pl = make_planes(rng["planes"], g.means, 16, [32], 8, "zero" if zero_field else plane_dist)
    mlp = make_mlp(rng["mlp"], pl.in_dim, 64, zero_bias=zero_field)
    cams = [look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 128, 128, 50.0)]
    return Scene(g, pl, mlp, cams, np.array([0.5]), "C1")


def config2(plane_dist: str = "normal", n: int = 100_000, width: int = 800, height: int = 800,
            n_cams: int = 20, n_times: int = 20, colour_opacity: bool = False) -> Scene:
    """colour_opacity adds the appendix's colour and opacity heads."""
    rng = _streams(2)
    means = means_shell(rng["means"], n)
    g = make_gaussians(rng, n, means, 3, "normal")
    pl = make_planes(rng["planes"], g.means, 32, [64, 128], 25, plane_dist)
    mlp = make_mlp(rng["mlp"], pl.in_dim, 64, colour_rows=sh_rows(3) if colour_opacity else 0,
                   opacity=colour_opacity)
    cams = ring_cameras(n_cams, 4.0, width, height)
    ts = np.linspace(0.0, 1.0, n_times)
    return Scene(g, pl, mlp, cams, ts, "C2")


def config4(plane_dist: str = "normal", n: int = 300_000, width: int = 1352, height: int = 1014,
            n_cams: int = 20, n_times: int = 300) -> Scene:
    rng = _streams(4)
    means = means_box_cluster(rng["means"], n)
    g = make_gaussians(rng, n, means, 3, "normal")
    pl = make_planes(rng["planes"], g.means, 32, [64, 128, 256], 150, plane_dist)
    mlp = make_mlp(rng["mlp"], pl.in_dim, 128)
    cams = ring_cameras(n_cams, 8.0, width, height)
    ts = np.linspace(0.0, 1.0, n_times)
    return Scene(g, pl, mlp, cams, ts, "C4")


def tiny_scene(seed: int, n: int = 48, width: int = 48, height: int = 40, sh_degree: int = 1,
               plane_dist: str = "uniform", log_scale_mean: float = -2.2,
               colour_opacity: bool = False) -> Scene:
    """A few dozen Gaussians in front of one camera: small enough for
    per-pixel brute force over every Gaussian."""
    rng = _streams(100 + seed)
    means = means_cube(rng["means"], n, 0.8)
    g = make_gaussians(rng, n, means, sh_degree, "normal")
    g.log_scales = _f32(rng["extra"].normal(log_scale_mean, 0.4, size=(3, n)))
    pl = make_planes(rng["planes"], g.means, 16, [8], 4, plane_dist)
    mlp = make_mlp(rng["mlp"], pl.in_dim, 32, colour_rows=sh_rows(sh_degree) if colour_opacity else 0,
                   opacity=colour_opacity)
    cam = look_at_camera((0.6, 0.3, 3.0), (0.0, 0.0, 0.0), width, height, 50.0)
    return Scene(g, pl, mlp, [cam], np.array([0.3]), f"tiny{seed}")


def serving_scenes(scale: float = 1.0):
    """Three resident scenes for the serving mix: 50k and 150k Gaussians from
    the 2k-config generator family and 300k from the large-scene generator.
    `scale` shrinks every scene for quick tests."""
    out = []
    for cid, n, gen in ((51, 50_000, "cube"), (52, 150_000, "cube"), (53, 300_000, "box")):
        n = max(16, int(n * scale))
        rng = _streams(cid)
        if gen == "cube":
            means = means_cube(rng["means"], n)
            g = make_gaussians(rng, n, means, 0, "rgb0")
            pl = make_planes(rng["planes"], g.means, 16, [32], 8)
            mlp = make_mlp(rng["mlp"], pl.in_dim, 64)
            radius = 4.0
        else:
            means = means_box_cluster(rng["means"], n)
            g = make_gaussians(rng, n, means, 3, "normal")
            pl = make_planes(rng["planes"], g.means, 32, [64, 128, 256], 150)
            mlp = make_mlp(rng["mlp"], pl.in_dim, 128)
            radius = 8.0
        out.append((g, pl, mlp, radius))
    return out


def composition(n_each: int = 50_000, width: int = 800, height: int = 800, n_cams: int = 20,
                n_times: int = 20):
    """Two trained-scene stand-ins placed side by side in one space (the
    composition workload): a 100k-configuration-family shell (SH3, planes
    64+128 x t25 F32, MLP 64) and a small-configuration-family cube (SH0,
    planes 32 x t8 F16, MLP 64) whose decoder also has the colour and opacity
    heads, each with n_each Gaussians.  Returns (items, cameras, timestamps)
    with items = [(gaussians, planes, mlp, (rotation wxyz, scale,
    translation))]; the two decoders run as two deform launches."""
    out = []
    rng = _streams(70)
    means = means_shell(rng["means"], n_each)
    g = make_gaussians(rng, n_each, means, 3, "normal")
    pl = make_planes(rng["planes"], g.means, 32, [64, 128], 25)
    mlp = make_mlp(rng["mlp"], pl.in_dim, 64)
    th = math.radians(30.0)
    out.append((g, pl, mlp, ((math.cos(th / 2), 0.0, math.sin(th / 2), 0.0), 0.8, (-1.1, 0.0, 0.0))))
    rng = _streams(71)
    means = means_cube(rng["means"], n_each)
    g = make_gaussians(rng, n_each, means, 0, "rgb0")
    pl = make_planes(rng["planes"], g.means, 16, [32], 8)
    mlp = make_mlp(rng["mlp"], pl.in_dim, 64, colour_rows=sh_rows(0), opacity=True)
    out.append((g, pl, mlp, ((1.0, 0.0, 0.0, 0.0), 0.7, (1.1, 0.0, 0.0))))
    cams = ring_cameras(n_cams, 4.5, width, height)
    return out, cams, np.linspace(0.0, 1.0, n_times)


def poisson_arrivals(rate_hz: float, duration_s: float, n_scenes: int, n_cams: int,
                     resolutions: Sequence[Sequence[int]], seed: int = 5):
    """Poisson request trace: (arrival_s, scene, camera, t, (W, H))."""
    rng = _streams(seed)["arrivals"]
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append((t, int(rng.integers(n_scenes)), int(rng.integers(n_cams)),
                    float(rng.uniform(0.0, 1.0)), tuple(resolutions[int(rng.integers(len(resolutions)))])))
    return out

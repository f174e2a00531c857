"""CPU oracle for the 4D-GS deform-then-splat render.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product path.

The arithmetic lives in ``g4d_oracle.c`` (plain C, FP64 continuous values,
binary32 replica of the discrete tile/key structure); this module builds it
with gcc, loads it with ctypes and wraps it with numpy.  See the C file's
header for the precision policy and the paper passages each step follows
(Sec. 3.1 Eq. 1-4; Sec. 4.1; Sec. 4.2 Eq. 7-8).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import types
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "g4d_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
TILE = 16

_lib = None


def build_lib(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (host code only)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build_lib(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.orc_bilinear.argtypes = [P, i32, i32, i32, f64, f64, P]
    lib.orc_deform.argtypes = [i32, P, P, P, P, i32, i32, P, P, P, P, i32, i32,
                               P, P, P, P, P, P, P, P, f64, i32, P, P, P, P, P, P,
                               i32, P, P, P, P, P, P]
    lib.orc_to_bf16.argtypes = [i64, P, P]
    lib.orc_sh_basis.argtypes = [i32, i32, f64, f64, f64]
    lib.orc_sh_basis.restype = f64
    lib.orc_project.argtypes = [i32, i32, P, P, P, P, P, P, P, i32, i32, P, P, P, P, P]
    lib.orc_count_instances.argtypes = [i32, P]
    lib.orc_count_instances.restype = i64
    lib.orc_emit_instances.argtypes = [i32, P, P, i32, P, P]
    lib.orc_sort_instances.argtypes = [i64, P, P]
    lib.orc_tile_ranges.argtypes = [i64, P, i32, P]
    lib.orc_blend.argtypes = [i32, i32, P, P, P, P, P, P, f64, P, P, P, P, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def set_threads(n: int) -> None:
    """Limit OpenMP threads of the oracle (affects later calls)."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


# --------------------------------------------------------------- primitives

def bilinear(plane: np.ndarray, ua: float, ub: float) -> np.ndarray:
    """One align-corners, border-clamped bilinear query of a [nb][na][F]
    plane at (ua, ub) in [-1, 1] (Sec. 4.2, Eq. 7 'interp')."""
    plane = _c(plane, np.float32)
    nb, na, F = plane.shape
    out = np.zeros(F, dtype=np.float64)
    _load().orc_bilinear(_p(plane), na, nb, F, float(ua), float(ub), _p(out))
    return out


def to_bf16(x) -> np.ndarray:
    """The BF16-emulation mode's rounding: x rounded to binary32, then to
    bfloat16 (nearest, ties to even), returned as float64."""
    x = _c(x, np.float64)
    out = np.zeros_like(x)
    _load().orc_to_bf16(int(x.size), _p(x), _p(out))
    return out


def sh_basis(l: int, m: int, d) -> float:
    """Real SH basis function Y_l^m at unit direction d (closed form)."""
    return float(_load().orc_sh_basis(l, m, float(d[0]), float(d[1]), float(d[2])))


# ------------------------------------------------------------------ deform

def deform(g, planes, mlp, t: float, bf16_emulate: bool = False, want_features: bool = False):
    """FP64 deformation (Sec. 4.2, Eq. 7-8) of canonical Gaussians ``g``.

    Returns a namespace with FP64 means [3][n], scales [3][n] (linear),
    quats [4][n] (unit), opacity [n] (sigmoid), and optionally f_h [n][in]
    and the raw deltas [n][10] (dx 3, dr 4, ds 3).  With the appendix's
    colour head (mlp.wc) ``sh`` is the FP64 C + dC [3 (d+1)^2][n], else
    None; with the opacity head (mlp.wa) the opacity is sigmoid(logit +
    dalpha)."""
    lib = _load()
    n = g.n
    L, F = planes.n_scales, planes.feat
    assert F * L <= 256 and mlp.hidden <= 512 and mlp.in_dim == F * L
    means, ls, qs, ol = (_c(x, np.float32) for x in (g.means, g.log_scales, g.quats, g.opacity_logits))
    res = _c(np.array(planes.res, dtype=np.int32).reshape(-1), np.int32)
    plist = [_c(p, np.float32) for lv in planes.planes for p in lv]
    parr = (ctypes.c_void_p * len(plist))(*[p.ctypes.data for p in plist])
    bmin, bmax = _c(planes.bmin, np.float32), _c(planes.bmax, np.float32)
    ws = [_c(x, np.float32) for x in (mlp.w1, mlp.b1, mlp.wx, mlp.bx, mlp.wr, mlp.br, mlp.ws, mlp.bs)]
    om = np.zeros((3, n)); osc = np.zeros((3, n)); oq = np.zeros((4, n)); oo = np.zeros(n)
    fh = np.zeros((n, mlp.in_dim)) if want_features else None
    dl = np.zeros((n, 10)) if want_features else None
    wc, wa = getattr(mlp, "wc", None), getattr(mlp, "wa", None)
    n_sh = 3 * (g.sh_degree + 1) ** 2 if wc is not None else 0
    if wc is not None:
        assert np.asarray(wc).shape == (n_sh, mlp.hidden)
    wc, bc = (_c(wc, np.float32), _c(mlp.bc, np.float32)) if wc is not None else (None, None)
    wa, ba = (_c(wa, np.float32), _c(mlp.ba, np.float32)) if wa is not None else (None, None)
    sh_in = _c(g.sh, np.float32).reshape(-1) if n_sh else None
    osh = np.zeros((n_sh, n)) if n_sh else None
    heads = [n_sh] + [_p(x) if x is not None else None for x in (wc, bc, wa, ba, sh_in, osh)]
    lib.orc_deform(n, _p(means), _p(ls), _p(qs), _p(ol), L, F, _p(bmin), _p(bmax), _p(res),
                   ctypes.cast(parr, ctypes.c_void_p), mlp.in_dim, mlp.hidden,
                   *[_p(w) for w in ws], float(t), int(bool(bf16_emulate)),
                   _p(om), _p(osc), _p(oq), _p(oo),
                   _p(fh) if fh is not None else None, _p(dl) if dl is not None else None, *heads)
    return types.SimpleNamespace(means=om, scales=osc, quats=oq, opacity=oo, features=fh, delta=dl,
                                 sh=None if osh is None else osh.reshape(np.shape(g.sh)))


def _quat_matrix(q):
    """Rotation matrix of the unit quaternion q = (w, x, y, z)."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _quat_mul(a, b):
    """Hamilton product a (x) b of quaternions (w, x, y, z); b may be [4][n]."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def place(d, rotation, scale, translation):
    """The rigid edit of a deformed set (Sec. 5.4 composition, appendix
    "Editing with 4D Gaussians": the rotation must reach the Gaussians'
    quaternions and the scaling their scales): mean'' = s R mean' + T,
    quat'' = rotation (x) quat', scales'' = s scales'.  FP64."""
    q = np.asarray(rotation, dtype=np.float64)
    q = q / np.linalg.norm(q)
    R = _quat_matrix(q)
    T = np.asarray(translation, dtype=np.float64)[:, None]
    return types.SimpleNamespace(means=scale * (R @ d.means) + T, scales=scale * d.scales,
                                 quats=_quat_mul(q, d.quats), opacity=d.opacity.copy(), sh=d.sh)


def compose(items, sh_degree_out: int):
    """Multi-scene composition (Sec. 5.4): G' = {G'_1, ..., G'_n}.  items:
    list of (gaussians, planes, mlp, t, (rotation, scale, translation) or
    None).  Each item is deformed (FP64), placed, and concatenated in order;
    SH coefficients are padded with zero rows up to sh_degree_out.  Returns
    FP64 means/scales/quats/opacity and the SH [(D+1)^2][3][N]."""
    parts, shs = [], []
    for g, planes, mlp, t, pl in items:
        d = deform(g, planes, mlp, t)
        if pl is not None:
            d = place(d, *pl)
        parts.append(d)
        sh = np.asarray(g.sh if d.sh is None else d.sh, dtype=np.float64)
        rows = np.zeros(((sh_degree_out + 1) ** 2, 3, g.n))
        rows[:sh.shape[0]] = sh
        shs.append(rows)
    cat = lambda k: np.concatenate([getattr(p, k) for p in parts], axis=-1)
    return types.SimpleNamespace(means=cat("means"), scales=cat("scales"), quats=cat("quats"),
                                 opacity=cat("opacity"), sh=np.concatenate(shs, axis=-1),
                                 sh_degree=int(sh_degree_out))


def to_splats32(d, sh: np.ndarray, sh_degree: int):
    """Round an FP64 deformation result to the binary32 render input."""
    return types.SimpleNamespace(
        means=_c(d.means, np.float32), scales=_c(d.scales, np.float32),
        quats=_c(d.quats, np.float32), opacity=_c(d.opacity, np.float32),
        sh=_c(sh, np.float32), sh_degree=int(sh_degree), n=int(d.means.shape[1]))


def _cam_arrays(cam):
    view = _c(np.asarray(cam.viewmat).reshape(-1), np.float32)
    intr = _c([cam.fx, cam.fy, cam.cx, cam.cy, cam.tan_half_fov_x, cam.tan_half_fov_y, cam.near],
              np.float32)
    campos = _c(cam.campos, np.float32)
    return view, intr, campos


# ---------------------------------------------------------------- render

def project(s, cam):
    """Per-Gaussian projection (Sec. 3.1, Eq. 2-3): binary32 key path and
    FP64 continuous values.  ``s`` has means, scales, quats, sh, sh_degree."""
    lib = _load()
    n = int(s.means.shape[1])
    means, scales, quats, sh = (_c(x, np.float32) for x in (s.means, s.scales, s.quats, s.sh))
    view, intr, campos = _cam_arrays(cam)
    rect = np.zeros((n, 4), dtype=np.int32)
    depth = np.zeros(n, dtype=np.uint32)
    radius = np.zeros(n, dtype=np.int32)
    f32v = np.zeros((n, 8), dtype=np.float32)
    f64v = np.zeros((n, 8), dtype=np.float64)
    lib.orc_project(n, int(s.sh_degree), _p(means), _p(scales), _p(quats), _p(sh), _p(view),
                    _p(intr), _p(campos), int(cam.width), int(cam.height), _p(rect), _p(depth),
                    _p(radius), _p(f32v), _p(f64v))
    return types.SimpleNamespace(rect=rect, depth_bits=depth, radius=radius, f32=f32v, f64=f64v)


def tiles_xy(width: int, height: int):
    return (width + TILE - 1) // TILE, (height + TILE - 1) // TILE


def instances(rect: np.ndarray, depth_bits: np.ndarray, tiles_x: int):
    """Emit (key, gid) tile instances and order them by key, ties by gid."""
    lib = _load()
    rect = _c(rect, np.int32)
    depth_bits = _c(depth_bits, np.uint32)
    n = rect.shape[0]
    k = int(lib.orc_count_instances(n, _p(rect)))
    keys = np.zeros(max(k, 1), dtype=np.uint64)
    vals = np.zeros(max(k, 1), dtype=np.uint32)
    lib.orc_emit_instances(n, _p(rect), _p(depth_bits), int(tiles_x), _p(keys), _p(vals))
    emitted = (keys[:k].copy(), vals[:k].copy())
    lib.orc_sort_instances(k, _p(keys), _p(vals))
    return types.SimpleNamespace(K=k, keys=keys[:k], vals=vals[:k], emitted_keys=emitted[0],
                                 emitted_vals=emitted[1])


def tile_ranges(keys: np.ndarray, n_tiles: int) -> np.ndarray:
    lib = _load()
    keys = _c(keys, np.uint64)
    out = np.zeros((n_tiles, 2), dtype=np.int64)
    lib.orc_tile_ranges(int(keys.shape[0]), _p(keys), int(n_tiles), _p(out))
    return out


def blend(cam, ranges, vals, opacity, proj, margin: float = 1e-5):
    lib = _load()
    W, H = int(cam.width), int(cam.height)
    img = np.zeros((3, H, W)); T = np.zeros((H, W))
    nc = np.zeros((H, W), dtype=np.int32); fl = np.zeros((H, W), dtype=np.int32)
    ev = np.zeros((H, W), dtype=np.int32)
    used = np.zeros((H, W, 2), dtype=np.int64)
    ranges = _c(ranges, np.int64)
    vals = _c(vals, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, dtype=np.uint32)
    opacity = _c(opacity, np.float32)
    bg = _c(cam.bg, np.float32)
    lib.orc_blend(W, H, _p(ranges), _p(vals), _p(opacity), _p(_c(proj.f32, np.float32)),
                  _p(_c(proj.f64, np.float64)), _p(bg), float(margin), _p(img), _p(T), _p(nc), _p(fl), _p(ev), _p(used))
    return img, T, nc, fl, ev, used


def render(s, cam, margin: float = 1e-5):
    """Full oracle render of binary32 render-ready Gaussians ``s`` (means,
    scales, quats, opacity, sh, sh_degree) through camera ``cam``."""
    proj = project(s, cam)
    tx, ty = tiles_xy(cam.width, cam.height)
    inst = instances(proj.rect, proj.depth_bits, tx)
    rng = tile_ranges(inst.keys, tx * ty)
    img, T, nc, fl, ev, used = blend(cam, rng, inst.vals, s.opacity, proj, margin)
    return types.SimpleNamespace(image=img, final_T=T, n_contrib=nc, flag=fl, evals=ev, used=used, proj=proj,
                                 K=inst.K, keys=inst.keys, vals=inst.vals, ranges=rng,
                                 tiles_x=tx, tiles_y=ty)


def deform_render(g, planes, mlp, t, cam, margin: float = 1e-5):
    d = deform(g, planes, mlp, t)
    s = to_splats32(d, g.sh if d.sh is None else d.sh, g.sh_degree)
    return s, render(s, cam, margin)

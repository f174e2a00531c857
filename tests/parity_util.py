"""Host-side comparison logic shared by the GPU parity tests (no GPU calls).

Two comparisons whose bars need more than an element-wise difference:

* admissible_bf16_check: the BF16-input decoder (Sec. 4.2 decoder with
  bfloat16 operands, FP32 accumulation) against the oracle's BF16-emulation
  mode, gated on the maximum error over every Gaussian.  Rounding an FP32
  intermediate (f_h, h) to bfloat16 is discontinuous: where the value lies
  closer to a rounding boundary than FP32 arithmetic can resolve, either
  neighbour is a correct result.  Those entries are enumerated; a Gaussian
  passes when the GPU's outputs match the emulation, within the bar, under
  one admissible choice of roundings.

* e2e_compare: GPU deform then GPU render against the oracle's FP64 deform
  then oracle render (Eq. 7-8 into Eq. 1-4), element-wise on every pixel
  whose discrete decisions agree.  A pixel is excluded when the oracle flags
  one of its own compositing decisions as near a threshold, or when the
  sequence of Gaussians it composites differs between the oracle's
  deformed set and the GPU's (a tile rectangle, radius or depth order moved
  by the FP32-vs-FP64 deformation, or a skip/stop decision that moved with
  it).
"""
from __future__ import annotations

import itertools
import types

import numpy as np
import torch

import oracle

U32 = 2.0 ** -24     # unit roundoff of binary32


def bf16(x) -> np.ndarray:
    """float32 -> bfloat16 (torch: nearest, ties to even) -> float64."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).to(
        torch.float64).numpy()


def bf16_boundary_distance(x32: np.ndarray):
    """Distance of binary32 values to the nearest bfloat16 rounding boundary
    (the midpoint of the two bfloat16 neighbours), and those neighbours."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32)
    lo_bits = u & np.uint32(0xffff0000)
    mid = (lo_bits | np.uint32(0x8000)).view(np.float32).astype(np.float64)
    lo = lo_bits.view(np.float32).astype(np.float64)
    hi = (lo_bits + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    return np.abs(x32.astype(np.float64) - mid), lo, hi


def _outputs(g, gi, delta, n_sh):
    """Eq. 8 and the activations in FP64 for Gaussian(s) gi from the decoder
    rows delta [..., 10 + n_sh + wa]: (means, quats, scales) and, with the
    appendix heads, the colour C + dC and the opacity sigmoid(logit + da)."""
    mu = g.means[:, gi].astype(np.float64).T
    ls = g.log_scales[:, gi].astype(np.float64).T
    q = g.quats[:, gi].astype(np.float64).T
    parts = [mu + delta[..., 0:3]]
    qq = q + delta[..., 3:7]
    parts.append(qq / np.linalg.norm(qq, axis=-1, keepdims=True))
    parts.append(np.exp(ls + delta[..., 7:10]))
    o = 10
    if n_sh:
        parts.append(np.asarray(g.sh, np.float64).reshape(n_sh, -1)[:, gi].T + delta[..., o:o + n_sh])
        o += n_sh
    if delta.shape[-1] > o:
        logit = g.opacity_logits[gi].astype(np.float64)
        parts.append((1.0 / (1.0 + np.exp(-(logit + delta[..., o]))))[..., None])
    return np.concatenate(parts, axis=-1)


def _gather(d, n_sh, has_a):
    parts = [d.means.T, d.quats.T, d.scales.T]
    if n_sh:
        parts.append(np.asarray(d.sh, np.float64).reshape(n_sh, -1).T)
    if has_a:
        parts.append(np.asarray(d.opacity, np.float64)[:, None])
    return np.concatenate(parts, axis=1).astype(np.float64)


def admissible_bf16_check(sc, t, gpu, eps_f: float, tol: float = 1e-5, max_flips: int = 6):
    """Check the GPU's BF16-decoder outputs (gpu.means/quats/scales and,
    with the appendix heads, gpu.sh/opacity; host float32, component-major)
    against the BF16 emulation.

    eps_f bounds the relative error of the GPU's FP32 f_h against the FP64
    f_h (the caller checks it on the exported features); an f_h entry closer
    than that to a bfloat16 boundary may round either way.  An h entry may
    round either way when it is within the FP32 accumulation bound
    (K + 2) u (sum |W1 f| + |b1|) of a boundary; a hidden unit whose
    pre-activation is within that bound of zero adds at most the bound times
    its head weights (added to the bar).  Flip sets (entries rounded to
    their other neighbour) are tried in order of size up to max_flips.
    Returns counts and the worst error under the best admissible rounding."""
    g, m = sc.gaussians, sc.mlp
    wc, wa = getattr(m, "wc", None), getattr(m, "wa", None)
    n_sh = 3 * (g.sh_degree + 1) ** 2 if wc is not None else 0
    d64 = oracle.deform(g, sc.planes, m, t, want_features=True)
    emu = oracle.deform(g, sc.planes, m, t, bf16_emulate=True)
    f = d64.features
    n, K = f.shape
    W1 = bf16(m.w1)
    b1 = m.b1.astype(np.float64)
    rows = [m.wx, m.wr, m.ws] + ([wc] if n_sh else []) + ([wa] if wa is not None else [])
    bias = [m.bx, m.br, m.bs] + ([m.bc] if n_sh else []) + ([m.ba] if wa is not None else [])
    W2 = bf16(np.concatenate(rows, 0))
    b2 = np.concatenate(bias, 0).astype(np.float64)
    f32 = f.astype(np.float32)
    fb = bf16(f32)
    # base path (every entry rounded as the emulation rounds it) equals the oracle's emulation
    h = np.maximum(fb @ W1.T + b1, 0.0)
    hb = bf16(h.astype(np.float32))
    base = _outputs(g, np.arange(n), hb @ W2.T + b2, n_sh)
    emu_out = _gather(emu, n_sh, wa is not None)
    assert np.abs(base - emu_out).max() <= 1e-12 * (1 + np.abs(emu_out).max())
    got = _gather(gpu, n_sh, wa is not None)
    err = np.abs(got - emu_out) / (1.0 + np.abs(emu_out))
    worst = err.max(axis=1)
    passed = worst <= tol
    df, flo, fhi = bf16_boundary_distance(f32)
    near_f = df <= eps_f * np.abs(f)
    alt_f = np.where(fb == flo, fhi, flo)               # the other neighbour of each f_h entry
    gam = (K + 2) * U32
    absW1, absW2 = np.abs(W1), np.abs(W2)
    stats = types.SimpleNamespace(n=n, base_pass=int(passed.sum()), alt_pass=0, fail=0,
                                  near_f_gaussians=int(near_f.any(axis=1).sum()), worst=0.0,
                                  worst_base=float(worst.max()) if n else 0.0, failed=[], max_flips=0)
    best_all = np.where(passed, worst, 0.0)
    q_all = g.quats.astype(np.float64)
    for gi in np.flatnonzero(~passed):
        fi = np.flatnonzero(near_f[gi])
        best, found = np.inf, False
        cache = {}

        def h_state(fs):
            # h of this f_h choice: its bfloat16 values, the entries within FP32 reach of a
            # boundary (with their other neighbour) and the ReLU slack on every decoder row
            if fs not in cache:
                fv = fb[gi].copy()
                fv[list(fs)] = alt_f[gi, list(fs)]
                pre = W1 @ fv + b1
                band = gam * (absW1 @ np.abs(fv) + np.abs(b1))
                hv = np.maximum(pre, 0.0)
                h32 = hv.astype(np.float32)
                dh, hlo, hhi = bf16_boundary_distance(h32)
                hb0 = bf16(h32)
                near_h = np.flatnonzero((dh <= band) & (hv > 0))
                alt_h = np.where(hb0 == hlo, hhi, hlo)
                amb = np.abs(pre) <= band
                cache[fs] = (hb0, near_h, alt_h, absW2[:, amb] @ band[amb])
            return cache[fs]

        # flip sets in order of their total size: the first admissible match ends the search
        for total in range(0, max_flips + 1):
            for wf in range(0, min(total, len(fi)) + 1):
                for fs in itertools.combinations(fi.tolist(), wf):
                    hb0, near_h, alt_h, slack_d = h_state(tuple(fs))
                    wh = total - wf
                    if wh > len(near_h):
                        continue
                    subsets = list(itertools.combinations(range(len(near_h)), wh))
                    H = np.repeat(hb0[None], len(subsets), 0)
                    for r, sub in enumerate(subsets):
                        idx = near_h[list(sub)]
                        H[r, idx] = alt_h[idx]
                    dl = H @ W2.T + b2                                  # [C, rows]
                    out = _outputs(g, gi, dl, n_sh)
                    # row slack in output space: means and colour 1:1, quats by 2 / |q + dr|,
                    # scales by the scale, opacity by 1/4 (the sigmoid's slope)
                    qn = np.linalg.norm(q_all[:, gi][None] + dl[:, 3:7], axis=1, keepdims=True)
                    sl = np.concatenate([np.broadcast_to(slack_d[0:3], (len(H), 3)), 2 * slack_d[3:7] / qn,
                                         slack_d[7:10] * out[:, 7:10],
                                         np.broadcast_to(slack_d[10:10 + n_sh], (len(H), n_sh)),
                                         np.broadcast_to(0.25 * slack_d[10 + n_sh:], (len(H), dl.shape[1] - 10 - n_sh))],
                                        axis=1)
                    e = np.max((np.abs(got[gi][None] - out) - sl) / (1.0 + np.abs(out)), axis=1)
                    best = min(best, float(e.min()))
                    if e.min() <= tol:
                        found = True
                        break
                if found:
                    break
            if found:
                stats.max_flips = max(stats.max_flips, total)
                break
        if found:
            stats.alt_pass += 1
        else:
            stats.fail += 1
            stats.failed.append((int(gi), best))
        best_all[gi] = best
    stats.worst = float(np.max(best_all)) if n else 0.0
    return stats


def tile_list_differences(r_a, r_b) -> int:
    """Number of tiles whose sorted instance lists differ between two oracle
    renders of the same frame."""
    n = 0
    for t in range(r_a.ranges.shape[0]):
        a = r_a.vals[r_a.ranges[t, 0]:r_a.ranges[t, 1]]
        b = r_b.vals[r_b.ranges[t, 0]:r_b.ranges[t, 1]]
        n += not np.array_equal(a, b)
    return n


def e2e_compare(gpu_image, orc_own, orc_on_gpu_set):
    """Per-pixel end-to-end comparison.  orc_own: the oracle's render of its
    own FP64 deformation (the expected image).  orc_on_gpu_set: the oracle's
    render of the GPU's deformed set, used only to find the pixels whose
    discrete decisions differ between the two deformations."""
    flag = (orc_own.flag != 0) | (orc_on_gpu_set.flag != 0) | (orc_own.used != orc_on_gpu_set.used).any(-1)
    ok = ~flag
    d = np.abs(gpu_image - orc_own.image)[:, ok]
    return types.SimpleNamespace(max_img=float(d.max()) if d.size else 0.0, flagged=int(flag.sum()),
                                 pixels=int(flag.size), tiles_differ=tile_list_differences(orc_own, orc_on_gpu_set),
                                 decision_flagged=int((orc_own.used != orc_on_gpu_set.used).any(-1).sum()))


def psnr(a, b) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def chain_reference(d, sh, sh_degree, host, cam, seed):
    """For a loss L = sum(w * image) through GPU deform + render: the
    oracle's render of its own deformed set d (FP64, rounded to binary32),
    whose tile lists the gradient oracle follows, and weights w = +-1 that
    are zero on every pixel flagged by the oracle or whose composited
    sequence differs between d and the GPU's deformed set `host` (there
    the two sides take different discrete decisions)."""
    own = oracle.render(oracle.to_splats32(d, sh, sh_degree), cam)
    on_gpu = oracle.render(oracle.to_splats32(host, sh if getattr(host, "sh", None) is None else host.sh,
                                              sh_degree), cam)
    flag = (own.flag != 0) | (on_gpu.flag != 0) | (own.used != on_gpu.used).any(-1)
    w = np.random.default_rng(seed).choice([-1.0, 1.0], size=own.image.shape) * (~flag)[None]
    return own, w, int(flag.sum())

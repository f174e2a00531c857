"""The appendix's colour and opacity deformation heads on the GPU: the HIP
deform (one 16-row head tile, or four when the colour head at SH degree >= 1
brings the head rows past 16) against the FP64 oracle, the rendered frame,
batching, the serving loop and the argument checks.

Bars as for the base method: deformation outputs (including the SH
coefficients C + dC) within def_tol of the oracle, keys bit-exact and the
image within 1e-4 of the oracle on the GPU's deformed set."""
import numpy as np
import pytest

import oracle
from paper_2310_08528_amd import g4d, synth
from tests.gpu_util import gpu_deform, gpu_render, log
from tests.parity_util import admissible_bf16_check
from tests.test_gpu_parity import _check_e2e, _check_render, def_tol, features_eps

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _errors(host, d):
    errs = {}
    for k in ("means", "scales", "quats", "opacity", "sh"):
        ref = np.asarray(getattr(d, k), dtype=np.float64)
        got = np.asarray(getattr(host, k), dtype=np.float64).reshape(ref.shape)
        errs[k] = float((np.abs(got - ref) / (1.0 + np.abs(ref))).max())
    return errs


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_deform_colour_opacity_heads_tiny(dev, deg):
    sc = synth.tiny_scene(20 + deg, n=300, sh_degree=deg, colour_opacity=True)
    rows = synth.sh_rows(deg) + 11
    log(f"[colour heads] SH degree {deg}: {rows} head rows, {'1 tile' if rows <= 16 else '4 tiles'}")
    host, _ = gpu_deform(sc, 0.3)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, 0.3)
    errs = _errors(host, d)
    log("   max rel err " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= def_tol(sc.planes), errs
    # the heads did move colour and opacity
    assert np.abs(host.sh - sc.gaussians.sh).max() > 1e-3


@pytest.mark.parametrize("t", [0.0, 0.37])
def test_deform_colour_opacity_heads_full_size(dev, t):
    """100k Gaussians, SH degree 3 (48 colour rows + 1 opacity row), in the
    headline configuration's field and decoder shape."""
    sc = synth.config2(plane_dist="uniform", colour_opacity=True)
    host, _ = gpu_deform(sc, t)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t)
    errs = _errors(host, d)
    log(f"[colour heads C2 100k t={t}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= def_tol(sc.planes), errs


def test_colour_heads_three_scales_hidden64(dev):
    """The large configuration's three-scale field (f_h 96) with a 64-wide
    decoder and SH degree 3 colour + opacity heads, on a ragged 5003
    Gaussians: the four-tile kernel shape whose W1 is held as per-wave
    register fragments (an LDS copy would limit the blocks per CU)."""
    import dataclasses
    sc = synth.config4(plane_dist="uniform", n=5003)
    mlp = synth.make_mlp(np.random.default_rng(9), sc.planes.in_dim, 64, colour_rows=synth.sh_rows(3),
                         opacity=True)
    sc = dataclasses.replace(sc, mlp=mlp)
    host, _ = gpu_deform(sc, 0.41)
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, 0.41)
    errs = _errors(host, d)
    log("[colour heads, 3 scales, hidden 64] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= def_tol(sc.planes), errs


def test_zero_heads_leave_the_base_outputs_bitwise_unchanged(dev):
    """All-zero colour and opacity heads: the four-tile kernel gives the same
    means, scales, quats and opacity as the one-tile kernel without heads,
    and returns the canonical SH coefficients."""
    import dataclasses
    sc = synth.tiny_scene(31, n=1000, sh_degree=3)
    rows, hid = synth.sh_rows(3), sc.mlp.hidden
    z = lambda *s: np.zeros(s, dtype=np.float32)
    m0 = dataclasses.replace(sc.mlp, wc=z(rows, hid), bc=z(rows), wa=z(1, hid), ba=z(1))
    base, _ = gpu_deform(sc, 0.55)
    heads, _ = gpu_deform(sc, 0.55, mlp=m0)
    for k in ("means", "scales", "quats", "opacity"):
        assert np.array_equal(getattr(base, k), getattr(heads, k)), k
    assert np.array_equal(heads.sh, sc.gaussians.sh)


def test_bf16_decoder_with_one_head_tile(dev):
    """SH degree 0 colour + opacity heads fit the one-tile kernel, which the
    BF16 decoder supports too: every output (colour and opacity included)
    against the oracle's BF16 emulation at 1e-5 under an admissible rounding
    of the entries within FP32 reach of a bfloat16 boundary."""
    import torch
    sc = synth.tiny_scene(24, n=2000, sh_degree=0, colour_opacity=True)
    t = 0.6
    host16, _ = gpu_deform(sc, t, precision=g4d.MLP_BF16)
    d64 = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t, want_features=True)
    e64 = _errors(host16, d64)
    log(f"[colour heads bf16] vs fp64 {e64}")
    for k in e64:
        assert e64[k] <= 0.05, (k, e64[k])
    G, P = g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV)
    f = torch.empty((G.n, sc.planes.in_dim), dtype=torch.float32, device=DEV)
    g4d.deform_features(G, P, t, f)
    torch.cuda.synchronize()
    eps = features_eps(sc.planes)
    ef = float((np.abs(f.cpu().numpy() - d64.features) / np.abs(d64.features)).max())
    assert ef <= eps, (ef, eps)
    st = admissible_bf16_check(sc, t, host16, eps_f=eps)
    log(f"   vs emulation: {st.base_pass} as emulated, {st.alt_pass} under another admissible rounding "
        f"(at most {st.max_flips} entries), {st.fail} failing; worst {st.worst:.2e}")
    assert st.fail == 0, st.failed[:10]


def test_bf16_decoder_with_four_head_tiles_is_unsupported(dev):
    sc = synth.tiny_scene(25, n=64, sh_degree=2, colour_opacity=True)
    with pytest.raises(g4d.G4DError) as e:
        gpu_deform(sc, 0.5, precision=g4d.MLP_BF16)
    assert e.value.status == g4d.EUNSUPPORTED


def test_colour_head_output_must_not_alias_the_input(dev):
    import torch
    sc = synth.tiny_scene(26, n=64, sh_degree=1, colour_opacity=True)
    G = g4d.DeviceGaussians(sc.gaussians, DEV)
    P, M = g4d.DevicePlanes(sc.planes, DEV), g4d.DeviceMLP(sc.mlp, DEV)
    out = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, DEV)     # SH pointer = the input's
    with pytest.raises(g4d.G4DError) as e:
        g4d.deform(G, P, M, 0.5, out)
    assert e.value.status == g4d.EINVAL
    torch.cuda.synchronize()


def test_frame_with_deformed_colour_and_opacity(dev):
    """Both heads: the render of the oracle's deformed set (colour and
    opacity moved) with keys bit-exact and the image within tolerance, then
    GPU deform + render against the oracle's deform + render, element-wise
    on every pixel whose discrete decisions agree."""
    sc = synth.tiny_scene(27, n=3000, width=160, height=120, sh_degree=3, colour_opacity=True,
                          log_scale_mean=-3.0)
    cam, t = sc.cameras[0], 0.42
    d = oracle.deform(sc.gaussians, sc.planes, sc.mlp, t)
    s = oracle.to_splats32(d, d.sh, 3)
    _check_render(s, cam, "colour + opacity heads frame", capacity=1 << 20)
    _check_e2e(sc, t, cam, "colour + opacity heads", capacity=1 << 20)


def test_batched_colour_jobs_equal_single_calls(dev):
    import torch
    scs = [synth.tiny_scene(40 + i, n=n, sh_degree=2, colour_opacity=True) for i, n in enumerate((500, 77, 1300))]
    objs = [(g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV), g4d.DeviceMLP(sc.mlp, DEV))
            for sc in scs]
    ts = [0.2, 0.5, 0.8]
    singles, batched = [], []
    for (G, P, M), t in zip(objs, ts):
        o = g4d.DeviceSplats(G.n, G.sh_degree, None, DEV)
        g4d.deform(G, P, M, t, o)
        singles.append(o)
        batched.append(g4d.DeviceSplats(G.n, G.sh_degree, None, DEV))
    g4d.deform_batched([(G, P, M, t, o) for (G, P, M), t, o in zip(objs, ts, batched)])
    torch.cuda.synchronize()
    for a, b in zip(singles, batched):
        for k in ("means", "scales", "quats", "opacity", "sh"):
            assert torch.equal(getattr(a, k), getattr(b, k)), k
    # a job without heads runs a different kernel: one launch cannot hold both
    plain = synth.tiny_scene(40, n=500, sh_degree=2)
    Gp, Pp, Mp = objs[0][0], objs[0][1], g4d.DeviceMLP(plain.mlp, DEV)
    with pytest.raises(g4d.G4DError) as e:
        g4d.deform_batched([(objs[0][0], objs[0][1], objs[0][2], 0.1, batched[0]),
                            (Gp, Pp, Mp, 0.1, g4d.DeviceSplats(Gp.n, 2, Gp.sh, DEV))])
    assert e.value.status == g4d.EINVAL


def test_served_colour_scene_equals_direct_path(dev):
    """A scene whose decoder has colour and opacity heads, served beside a
    scene without them: each image equals the direct deform + render."""
    import torch
    with_heads = synth.tiny_scene(50, n=4000, sh_degree=3, colour_opacity=True)
    without = synth.tiny_scene(51, n=3000, sh_degree=1)
    srv = g4d.Server(1 << 30, max_slots=4, max_width=128, max_height=128)
    dev_objs = []
    for sc in (with_heads, without):
        G, P, M = (g4d.DeviceGaussians(sc.gaussians, DEV), g4d.DevicePlanes(sc.planes, DEV),
                   g4d.DeviceMLP(sc.mlp, DEV))
        srv.add_scene(G, P, M)
        dev_objs.append((G, P, M))
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(12):
        s = i % 2
        cams = synth.ring_cameras(8, 3.0, 96, 80)
        reqs.append((s, cams[int(rng.integers(8))], float(rng.uniform(0, 1))))
    outs = [torch.full((3, c.height, c.width), -1.0, device=DEV) for _, c, _ in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(s, c, t, o) for (s, c, t), o in zip(reqs, outs)]
    for tk in tickets:
        srv.wait(tk)
    torch.cuda.synchronize()
    srv.close()
    for (s, c, t), o in zip(reqs, outs):
        G, P, M = dev_objs[s]
        S = g4d.DeviceSplats(G.n, G.sh_degree, None if M.has_colour else G.sh, DEV)
        ws = g4d.RenderWorkspace(G.n, c.width, c.height, 64 * G.n + 4096, DEV)
        img = torch.empty((3, c.height, c.width), device=DEV)
        g4d.deform(G, P, M, t, S)
        g4d.render(S, c, ws, img)
        torch.cuda.synchronize()
        assert torch.equal(o, img), (s, t)

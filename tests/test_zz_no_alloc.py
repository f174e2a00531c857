"""g4d_render_noalloc (the render with the library's fixed device array as
its workspace) against g4d_render with a caller workspace, through the C ABI:
two calls in a row, the second on a smaller input (fewer Gaussians, a smaller
and ragged image), so the second runs on an array the first left dirty.  The
two entry points run the same kernels, so image, final transmittance,
n_contrib and the instance count must agree bit for bit."""
import ctypes

import numpy as np
import pytest

from paper_2310_08528_amd import g4d, synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _frame(sc, cam, t, dev):
    import torch
    G = g4d.DeviceGaussians(sc.gaussians, dev)
    P = g4d.DevicePlanes(sc.planes, dev)
    M = g4d.DeviceMLP(sc.mlp, dev)
    S = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, dev)
    g4d.deform(G, P, M, t, S)
    torch.cuda.synchronize()
    return (G, P, M), S


def _outputs(cam, dev):
    import torch
    H, W = cam.height, cam.width
    return (torch.full((3, H, W), -1.0, dtype=torch.float32, device=dev),
            torch.full((H, W), -1.0, dtype=torch.float32, device=dev),
            torch.full((H, W), -1, dtype=torch.int32, device=dev))


def _check_same(sc, cam, t, dev, name):
    import torch
    log(f"[no-alloc] {name}: n={sc.gaussians.n} {cam.width}x{cam.height} t={t}")
    keep, S = _frame(sc, cam, t, dev)
    n = S.n
    ws = g4d.RenderWorkspace(max(n, 1), cam.width, cam.height, 64 * n + 4096, dev)
    ref = _outputs(cam, dev)
    g4d.render(S, cam, ws, *ref)
    torch.cuda.synchronize()
    st_ref = g4d.read_status(ws)
    got = _outputs(cam, dev)
    st = g4d.render_noalloc(S, cam, *got)
    assert st.overflow == 0 and st.sort_error == 0 and st_ref.overflow == 0
    assert st.instances == st_ref.instances and st.visible == st_ref.visible and st.tiles == st_ref.tiles
    for a, b, what in zip(got, ref, ("image", "final_T", "n_contrib")):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(a, b), (name, what, float(np.abs(a.astype(np.float64) - b).max()))
    # the asynchronous form (no status) gives the same frame
    again = _outputs(cam, dev)
    g4d.render_noalloc(S, cam, *again, status=False)
    torch.cuda.synchronize()
    for a, b in zip(again, ref):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), name
    log(f"[no-alloc] {name}: K={st.instances} identical")


def test_noalloc_render_equals_workspace_render_on_two_calls(dev):
    # first call: 100k Gaussians at 800x800 (the benchmark frame)
    sc = synth.config2(n_cams=20, n_times=20)
    _check_same(sc, sc.cameras[3], 0.37, dev, "100k 800x800")
    # second call, smaller: 2000 Gaussians, a ragged 100x75 image
    sc1 = synth.config1(plane_dist="uniform")
    cam = synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 100, 75, 50.0)
    _check_same(sc1, cam, 0.5, dev, "2000 100x75")


def test_noalloc_refuses_sizes_beyond_the_array(dev):
    import torch
    lib = g4d.load()
    cam = g4d.camera_struct(synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 4096, 4096, 50.0))
    # 3 million Gaussians need more than the array for their per-Gaussian records alone
    spl = g4d.Splats(3_000_000, 0, None, None, None, None, None)
    img = torch.empty(1, dtype=torch.float32, device=dev)
    st = g4d.DeviceStatus()
    assert lib.g4d_render_noalloc(ctypes.byref(spl), ctypes.byref(cam), ctypes.c_void_p(img.data_ptr()), None,
                                  None, ctypes.byref(st), None) == g4d.ENOMEM
    assert lib.g4d_render_noalloc(None, ctypes.byref(cam), ctypes.c_void_p(img.data_ptr()), None, None, None,
                                  None) == g4d.EINVAL

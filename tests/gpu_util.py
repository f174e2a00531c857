"""GPU-side helpers for the parity tests: run the HIP path through the C ABI
and bring its outputs and intermediates back to the host."""
import sys
import types

import numpy as np

from paper_2310_08528_amd import g4d


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_render(splats_host, cam, capacity=None, device="cuda:0", ws=None, want_intermediates=True):
    """Render binary32 render-ready Gaussians (host arrays) on the GPU."""
    import torch
    n = int(splats_host.means.shape[1])
    S = g4d.DeviceSplats.from_host(splats_host, device)
    if capacity is None:
        capacity = max(1024, min((1 << 30) - 1, 64 * n + 4096))
    if ws is None:
        ws = g4d.RenderWorkspace(max(n, 1), cam.width, cam.height, capacity, device)
    H, W = cam.height, cam.width
    img = torch.full((3, H, W), -1.0, dtype=torch.float32, device=device)
    T = torch.full((H, W), -1.0, dtype=torch.float32, device=device)
    nc = torch.full((H, W), -1, dtype=torch.int32, device=device)
    g4d.render(S, cam, ws, img, T, nc)
    torch.cuda.synchronize()
    st = g4d.read_status(ws)
    out = types.SimpleNamespace(image=img.cpu().numpy(), final_T=T.cpu().numpy(), n_contrib=nc.cpu().numpy(),
                                K=int(st.instances), overflow=int(st.overflow), sort_error=int(st.sort_error),
                                visible=int(st.visible), tiles=int(st.tiles), blend_evals=int(st.blend_evals),
                                ws=ws)
    if want_intermediates:
        K = min(out.K, ws.capacity)
        keys = torch.empty(max(K, 1), dtype=torch.int64, device=device)
        gids = torch.empty(max(K, 1), dtype=torch.int32, device=device)
        rect = torch.empty((max(n, 1), 4), dtype=torch.int32, device=device)
        depth = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        order = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        spl = torch.empty((max(n, 1), 12), dtype=torch.float32, device=device)
        tiles = out.tiles
        ranges = torch.empty((max(tiles, 1), 2), dtype=torch.int32, device=device)
        g4d.export(ws, g4d.EXPORT_SORTED_KEYS, n, K, keys)
        g4d.export(ws, g4d.EXPORT_SORTED_GIDS, n, K, gids)
        g4d.export(ws, g4d.EXPORT_RECT, n, 0, rect)
        g4d.export(ws, g4d.EXPORT_DEPTH_BITS, n, 0, depth)
        g4d.export(ws, g4d.EXPORT_DEPTH_ORDER, n, 0, order)
        g4d.export(ws, g4d.EXPORT_SPLAT2D, n, 0, spl)
        g4d.export(ws, g4d.EXPORT_RANGES, n, tiles, ranges)
        torch.cuda.synchronize()
        out.keys = keys.cpu().numpy().view(np.uint64)[:K]
        out.gids = gids.cpu().numpy().view(np.uint32)[:K]
        out.rect = rect.cpu().numpy()[:n]
        out.depth_bits = depth.cpu().numpy().view(np.uint32)[:n]
        out.order = order.cpu().numpy().view(np.uint32)[:n]
        out.splat2d = spl.cpu().numpy()[:n]
        out.ranges = ranges.cpu().numpy().view(np.uint32)[:tiles].astype(np.int64)
    return out


def gpu_deform(scene, t, device="cuda:0", precision=g4d.MLP_F32, planes=None, mlp=None):
    """Deform a synthetic scene's Gaussians on the GPU; returns host float32
    arrays (render-ready) and the device objects."""
    import torch
    G = g4d.DeviceGaussians(scene.gaussians, device)
    P = g4d.DevicePlanes(planes or scene.planes, device)
    M = g4d.DeviceMLP(mlp or scene.mlp, device, precision)
    # with a colour head the deform writes the SH coefficients into a buffer of their own
    out = g4d.DeviceSplats(G.n, G.sh_degree, None if M.has_colour else G.sh, device)
    g4d.deform(G, P, M, t, out)
    torch.cuda.synchronize()
    sh = out.sh.cpu().numpy().reshape(np.shape(scene.gaussians.sh)) if M.has_colour else scene.gaussians.sh
    host = types.SimpleNamespace(means=out.means.cpu().numpy(), scales=out.scales.cpu().numpy(),
                                 quats=out.quats.cpu().numpy(), opacity=out.opacity.cpu().numpy(),
                                 sh=sh, sh_degree=scene.gaussians.sh_degree, n=G.n)
    return host, (G, P, M, out)


def compare_images(gpu, orc, tol=1e-4):
    """Element-wise image/T comparison on pixels the oracle did not flag."""
    ok = orc.flag == 0
    d_img = np.abs(gpu.image - orc.image)[:, ok]
    d_T = np.abs(gpu.final_T - orc.final_T)[ok]
    return types.SimpleNamespace(max_img=float(d_img.max()) if d_img.size else 0.0,
                                 max_T=float(d_T.max()) if d_T.size else 0.0,
                                 flagged=int((~ok).sum()), pixels=int(ok.size),
                                 nc_mismatch=int((gpu.n_contrib != orc.n_contrib)[ok].sum()),
                                 ok=bool((d_img.size == 0 or d_img.max() <= tol) and
                                         (d_T.size == 0 or d_T.max() <= tol)))

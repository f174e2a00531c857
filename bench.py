"""Benchmark of the deform-then-splat render on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

A step is one frame of the whole hot path: the HexPlane deformation of all
Gaussians at timestamp t (g4d_deform) followed by the tile render through
one camera (g4d_render), inputs resident in HBM, image left on the device.
The reported rate runs the frames with --in-flight (default 4) frames in
flight: frame k goes to slot k % m, each slot with its own stream, splat
buffer, workspace and image (as serving slots do); the one-frame-at-a-time
rate and the rates at 1, 2, 3, 4, 6 and 8 frames in flight are reported
beside it.  The scene is stored once, before timing, in the Morton order of
its means (--layout morton; --layout index keeps the generated order).
Workload: 100k Gaussians on a noisy sphere shell (SH degree 3), planes at
spatial 64/128 and temporal 25 with 32 features, MLP 64-64-10, 800x800,
frames cycling through 20 ring cameras x 20 timestamps.

Prints one JSON line with frames/s, the roofline of the dominant kernel
(timed live with HIP events around it on the render stream) and the CPU
oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "deform+splat frames/s @800², 100k Gaussians; served p50/p99 ms vs plain"

# MI355X peaks: published HBM and FP32 vector (157.3 TFLOP/s counts packed
# fused multiply-adds); the VALU issue rate for wave64 instructions from the
# unit counts: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4
# cycles at 2.4 GHz.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4

# Algorithmic work of the blend per evaluated (pixel, Gaussian) pair, as the
# measurement contract counts it: about 24 binary32 operations (offset 2,
# quadratic form 7, exponent scale and exp 3, clamp 1, the two skip tests 2,
# T (1 - alpha) 2, stop test 1, weight 1, colour accumulation 6 - 1 for the
# transmittance update folded into the weight).  An evaluated pair is every
# list entry a pixel visits up to and including its stop (counted on the
# device, equal to the oracle's count).
BLEND_OPS_PER_EVAL = 24
STAGES = ["clear", "preprocess", "depth_sort", "offsets", "emit", "tile_sort", "ranges_and_order", "blend"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime torch has loaded."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipStreamWaitEvent.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint]

    def create(self):
        e = ctypes.c_void_p()
        assert self.lib.hipEventCreate(ctypes.byref(e)) == 0
        return e.value

    def record(self, e, stream):
        assert self.lib.hipEventRecord(e, stream) == 0

    def wait(self, stream, e):
        assert self.lib.hipStreamWaitEvent(stream, e, 0) == 0

    def elapsed(self, a, b) -> float:
        ms = ctypes.c_float()
        assert self.lib.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return ms.value

    def destroy(self, e):
        self.lib.hipEventDestroy(e)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, int(os.environ.get("OMP_NUM_THREADS", n))))


def cpu_baseline(sc, frames, n_frames: int, single_frames: int = 1):
    """The CPU oracle (FP64 deform + render) on the first n_frames frames on
    all host cores, then on the first single_frames frames on one thread."""
    import oracle
    cores = host_cores()
    oracle.set_threads(cores)
    oracle.build_lib(force=False)
    t0 = time.perf_counter()
    for (ci, t) in frames[:n_frames]:
        oracle.deform_render(sc.gaussians, sc.planes, sc.mlp, t, sc.cameras[ci])
    dt = time.perf_counter() - t0
    out = {"value": n_frames / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_frames} full frames (deform + render, 100k Gaussians, 800x800) of the same "
                     f"frame sequence; {dt:.1f} s on {cores} threads of {cpu_model()}"}
    if single_frames > 0:
        # the same oracle on one thread (its scaling over the host cores)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        for (ci, t) in frames[:single_frames]:
            oracle.deform_render(sc.gaussians, sc.planes, sc.mlp, t, sc.cameras[ci])
        d1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        out["single_thread"] = {"value": single_frames / d1, "unit": "frames/s", "cores": 1,
                                "sample": f"the first {single_frames} of those frames; {d1:.1f} s"}
    return out


def serving_bench(seconds: float, rate: float, budget_gb: float, slots: int, warm_s: float = 2.0,
                  sat_requests: int = 2000, tight_budget_gb: float = 2.0, tight_s: float = 10.0,
                  layout: str = "morton"):
    """Poisson requests over three resident scenes (50k and 150k Gaussians
    from the cube generator, 300k from the box-and-cluster generator), each
    picking a scene, one of 20 ring cameras, t ~ U[0, 1] and a frame size
    from {400x400, 800x800, 1352x1014}.  Served with continuous batching,
    then the same trace through the plain path (one request at a time, no
    batching, no graphs).  Each path then takes the first `sat_requests`
    requests of the trace back to back (closed loop) for its peak rate.
    With layout="morton" each scene is stored in the Morton order of its
    means before it is added (the same one-time step as the frame benchmark's)."""
    import torch
    from paper_2310_08528_amd import g4d, synth
    dev = "cuda:0"
    res = [(400, 400), (800, 800), (1352, 1014)]
    scenes = synth.serving_scenes(1.0)
    cams = [[[g4d.camera_struct(c) for c in synth.ring_cameras(20, radius, w, h)] for (w, h) in res]
            for (_, _, _, radius) in scenes]
    outs = {r: [torch.empty((3, r[1], r[0]), device=dev) for _ in range(48)] for r in res}
    trace = synth.poisson_arrivals(rate, warm_s + seconds, len(scenes), 20, res, seed=5)
    dev_scenes = [(g4d.DeviceGaussians(g, dev), g4d.DevicePlanes(p, dev), g4d.DeviceMLP(m, dev))
                  for (g, p, m, _) in scenes]
    if layout == "morton":
        for (G_, _, _), (_, p, _, _) in zip(dev_scenes, scenes):
            ws_ = g4d.RenderWorkspace(G_.n, 16, 16, 4096, dev)
            g4d.store_in_order(G_, g4d.spatial_order(G_, p.bmin, p.bmax, ws_))
            del ws_
        torch.cuda.synchronize()

    def run(slots_, graphs, batch, budget=budget_gb, dur=seconds):
        srv = g4d.Server(int(budget * (1 << 30)), max_slots=slots_, use_graphs=graphs, batch_deform=batch,
                         max_width=1352, max_height=1014)
        ids = [srv.add_scene(*d) for d in dev_scenes]
        log(f"serving ({slots_} slots, graphs={graphs}, batch={batch}): warming {len(ids) * len(res)} classes")
        # warm every (scene, frame size) class once: sizes its capacity, captures its graph
        for si in ids:
            for ri, r in enumerate(res):
                srv.wait(srv.submit(si, cams[si][ri][0], 0.5, outs[r][0]))
        srv.reset_stats()
        log("serving: trace")
        t0 = time.perf_counter()
        k = 0
        next_log = 5.0
        for (ta, si, ci, t, r) in trace:
            if ta >= warm_s + dur:
                break
            delay = t0 + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            if ta >= warm_s and k == 0:
                srv.reset_stats()
            k += ta >= warm_s
            srv.submit(si, cams[si][res.index(tuple(r))][ci], t, outs[tuple(r)][k % 48])
            if ta >= next_log:
                log(f"serving: t={ta:.0f} s, {k} requests")
                next_log += 5.0
        srv.drain()
        st = srv.stats()
        # closed loop: the measured part of the trace submitted back to back
        # (arrival times ignored), completions per second at saturation
        srv.reset_stats()
        sat = [(si, ci, t, r) for (ta, si, ci, t, r) in trace if warm_s <= ta < warm_s + dur][:sat_requests]
        t0 = time.perf_counter()
        for j, (si, ci, t, r) in enumerate(sat):
            srv.submit(si, cams[si][res.index(tuple(r))][ci], t, outs[tuple(r)][j % 48])
        srv.drain()
        st["saturation_frames_per_s"] = len(sat) / (time.perf_counter() - t0)
        srv.close()
        return st

    log("serving: scenes ready")
    served = run(slots, True, True)
    log(f"served: {served}")
    plain = run(1, False, False)
    log(f"plain: {plain}")
    # the same trace's first `tight_s` seconds with a tight request-memory
    # budget, so that admissions wait for memory
    tight = None
    if tight_budget_gb:
        tight = run(slots, True, True, budget=tight_budget_gb, dur=tight_s)
        log(f"served, {tight_budget_gb:g} GB budget: {tight}")
    keep = ("p50_ms", "p99_ms", "mean_ms", "max_ms", "frames_per_s", "completed", "rejected",
            "batched_launches", "graph_replays", "eager_renders", "overflow_retries", "saturation_frames_per_s")
    out = {"workload": f"Poisson {rate:.0f}/s for {seconds:.0f} s (+{warm_s:.0f} s warm-up), 3 resident scenes "
                       "(50k, 150k, 300k), frames 400x400 / 800x800 / 1352x1014",
           "served": {k: served[k] for k in keep}, "plain": {k: plain[k] for k in keep},
           "slots": slots, "hbm_budget_gb": budget_gb, "layout": layout,
           "peak_request_bytes": int(served["peak_bytes"])}
    if tight is not None:
        out["served_tight_budget"] = {"hbm_budget_gb": tight_budget_gb, "seconds": tight_s,
                                      "peak_request_bytes": int(tight["peak_bytes"]),
                                      **{k: tight[k] for k in keep}}
    return out


def time_scene(sc, precision, steps, warmup, n_frames=None, layout="morton"):
    """frames/s and per-stage ms of deform + render over a scene's frame
    sequence (camera k mod cameras, timestamp k mod timestamps), one frame at
    a time; with layout="morton" the scene is first stored in the Morton
    order of its means."""
    import torch
    from paper_2310_08528_amd import g4d
    dev = "cuda:0"
    ev = HipEvents()
    nc, nt = len(sc.cameras), len(sc.timestamps)
    nf = n_frames or max(nc, nt)
    frames = [(k % nc, float(sc.timestamps[k % nt])) for k in range(nf)]
    G = g4d.DeviceGaussians(sc.gaussians, dev)
    P = g4d.DevicePlanes(sc.planes, dev)
    M = g4d.DeviceMLP(sc.mlp, dev, precision)
    S = g4d.DeviceSplats(G.n, G.sh_degree, None if M.has_colour else G.sh, dev)
    cams = [g4d.camera_struct(c) for c in sc.cameras]
    W, H = sc.cameras[0].width, sc.cameras[0].height
    img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    capacity = 64 * G.n + 4096
    ws = g4d.RenderWorkspace(G.n, W, H, capacity, dev)
    if layout == "morton":
        g4d.store_in_order(G, g4d.spatial_order(G, sc.planes.bmin, sc.planes.bmax, ws))
    kmax = 0
    for (ci, t) in frames:
        g4d.deform(G, P, M, t, S)
        g4d.render(S, cams[ci], ws, img)
        st = g4d.read_status(ws)
        kmax = max(kmax, int(st.instances))
        if st.overflow:
            del ws
            capacity = int(kmax * 1.25) + 4096
            ws = g4d.RenderWorkspace(G.n, W, H, capacity, dev)
    for k in range(warmup):
        ci, t = frames[k % nf]
        g4d.deform(G, P, M, t, S)
        g4d.render(S, cams[ci], ws, img)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ci, t = frames[k % nf]
        g4d.deform(G, P, M, t, S)
        g4d.render(S, cams[ci], ws, img)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = g4d.read_status(ws)
    assert st.overflow == 0 and st.sort_error == 0
    sp = torch.cuda.current_stream().cuda_stream
    n_prof = min(steps, 50)
    stage_ev = [[ev.create() for _ in range(9)] for _ in range(n_prof)]
    dfm_ev = [(ev.create(), ev.create()) for _ in range(n_prof)]
    for k in range(n_prof):
        ci, t = frames[k % nf]
        ev.record(dfm_ev[k][0], sp)
        g4d.deform(G, P, M, t, S)
        ev.record(dfm_ev[k][1], sp)
        g4d.set_stage_events(stage_ev[k])
        g4d.render(S, cams[ci], ws, img)
        g4d.set_stage_events(None)
    torch.cuda.synchronize()
    stages = {"deform": float(np.mean([ev.elapsed(a, b) for a, b in dfm_ev]))}
    for i, name in enumerate(STAGES):
        stages[name] = float(np.mean([ev.elapsed(e[i], e[i + 1]) for e in stage_ev]))
    return {"gaussians": G.n, "width": W, "height": H, "frames": nf, "steps": steps,
            "frames_per_s": round(steps / wall, 2), "ms_per_frame": round(1e3 * wall / steps, 4),
            "stages_ms": {k: round(v, 4) for k, v in stages.items()}, "instances_max": kmax}


def time_composition(steps, warmup, n_each=50_000, layout="morton"):
    """frames/s of the composition workload: two scenes (two deform kernel
    variants, so two launches) placed into one set by g4d_deform_compose,
    then one render at 800x800; with layout="morton" each scene is first
    stored in the Morton order of its means."""
    import torch
    from paper_2310_08528_amd import g4d, synth
    dev = "cuda:0"
    ev = HipEvents()
    items, cams_h, ts = synth.composition(n_each=n_each)
    dev_items = [(g4d.DeviceGaussians(g, dev), g4d.DevicePlanes(pl, dev), g4d.DeviceMLP(m, dev), g4d.placement(*p))
                 for g, pl, m, p in items]
    n = sum(it[0].n for it in dev_items)
    if layout == "morton":
        for (G_, _, _, _), (_, pl, _, _) in zip(dev_items, items):
            ws_ = g4d.RenderWorkspace(G_.n, 16, 16, 4096, dev)
            g4d.store_in_order(G_, g4d.spatial_order(G_, pl.bmin, pl.bmax, ws_))
            del ws_
    S = g4d.DeviceSplats(n, 3, None, dev)
    cams = [g4d.camera_struct(c) for c in cams_h]
    W, H = cams_h[0].width, cams_h[0].height
    img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    nf = max(len(cams), len(ts))
    frames = [(k % len(cams), float(ts[k % len(ts)])) for k in range(nf)]

    def frame(k):
        ci, t = frames[k % nf]
        g4d.deform_compose([(G, P, M, t, pl) for G, P, M, pl in dev_items], S)
        g4d.render(S, cams[ci], ws, img)
    ws = g4d.RenderWorkspace(n, W, H, 64 * n + 4096, dev)
    kmax = 0
    for k in range(nf):
        frame(k)
        st = g4d.read_status(ws)
        kmax = max(kmax, int(st.instances))
    if kmax > 64 * n + 4096:
        ws = g4d.RenderWorkspace(n, W, H, int(kmax * 1.25) + 4096, dev)
    for k in range(warmup):
        frame(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        frame(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = g4d.read_status(ws)
    assert st.overflow == 0 and st.sort_error == 0
    sp = torch.cuda.current_stream().cuda_stream
    marks = [(ev.create(), ev.create(), ev.create()) for _ in range(min(steps, 50))]
    for k, (a, b, c) in enumerate(marks):
        ci, t = frames[k % nf]
        ev.record(a, sp)
        g4d.deform_compose([(G, P, M, t, pl) for G, P, M, pl in dev_items], S)
        ev.record(b, sp)
        g4d.render(S, cams[ci], ws, img)
        ev.record(c, sp)
    torch.cuda.synchronize()
    return {"workload": f"2 scenes x {n_each} Gaussians (shell SH3 F32 64+128/t25 MLP 64; cube SH0 F16 32/t8 "
                        f"MLP 64 with colour + opacity heads), placed, {W}x{H}",
            "gaussians": n, "steps": steps, "frames_per_s": round(steps / wall, 2),
            "ms_per_frame": round(1e3 * wall / steps, 4),
            "compose_ms": round(float(np.mean([ev.elapsed(a, b) for a, b, _ in marks])), 4),
            "render_ms": round(float(np.mean([ev.elapsed(b, c) for _, b, c in marks])), 4),
            "instances_max": kmax}


TRAIN_WORKLOADS = {
    "small": "training iteration, 2000 Gaussians (SH0, planes 32 x t8 F16, MLP 16-64-10), 800x800, "
             "L1 + grid TV; gradients of every canonical parameter, plane cell and decoder weight; "
             "Adam update of all of them",
    "100k": "training iteration, 100k Gaussians (shell, SH3, planes 64/128 x t25 F32, MLP 64-64-10), 800x800, "
            "L1 + grid TV; gradients of every canonical parameter, plane cell and decoder weight; "
            "Adam update of all of them",
}


def time_training_step(steps, warmup, which="small", layout="index"):
    """One training iteration at 800x800: deform + render, the L1 loss and
    its gradient against a target frame, render backward and deform backward
    (gradients of every canonical parameter, plane cell and decoder weight),
    the grid TV term, and the Adam update of every trainable tensor.  "small"
    is the small configuration's scene (2000 Gaussians, SH0, planes 32 x t8
    F16, MLP 16-64-10), "100k" the headline scene (stored in Morton order
    with layout="morton")."""
    import torch
    from paper_2310_08528_amd import g4d, synth
    dev = "cuda:0"
    ev = HipEvents()
    if which == "small":
        sc = synth.config1()
        cam = g4d.camera_struct(synth.look_at_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 800, 800, 50.0))
        cap_per = 256
    else:
        sc = synth.config2(n_cams=1, n_times=20)
        cam = g4d.camera_struct(sc.cameras[0])
        cap_per = 64
    G, P, M = g4d.DeviceGaussians(sc.gaussians, dev), g4d.DevicePlanes(sc.planes, dev), g4d.DeviceMLP(sc.mlp, dev)
    S = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, dev)
    ws = g4d.RenderWorkspace(G.n, 800, 800, cap_per * G.n + 4096, dev)
    if layout == "morton":
        g4d.store_in_order(G, g4d.spatial_order(G, sc.planes.bmin, sc.planes.bmax, ws))
        torch.cuda.synchronize()
    img = torch.empty((3, 800, 800), device=dev)
    T = torch.empty((800, 800), device=dev)
    nc = torch.empty((800, 800), dtype=torch.int32, device=dev)
    g4d.deform(G, P, M, 0.0, S)
    g4d.render(S, cam, ws, img, T, nc)
    target = img.clone()
    loss = torch.empty((), device=dev)
    gimg = torch.empty_like(img)
    gs = g4d.DeviceSplatsGrad(G.n, G.sh_degree, dev)
    gd = g4d.DeviceDeformGrad(G, P, M, dev)
    ts = [0.05 + 0.9 * k / 19 for k in range(20)]
    sp = torch.cuda.current_stream().cuda_stream
    tvl = torch.empty((), device=dev)
    params = [G.means, G.log_scales, G.quats, G.opacity_logits, G.sh] + [p for lv in P.tensors for p in lv] + \
             [v for v in M.w.values() if v is not None]
    grads = [gd.means, gd.log_scales, gd.quats, gd.opacity_logits, gd.sh] + [p for lv in gd.planes for p in lv] + \
            [v for v in gd.w.values() if v is not None]
    lrs = [1.6e-3] * (len(params) - sum(1 for v in M.w.values() if v is not None)) + \
          [1.6e-4] * sum(1 for v in M.w.values() if v is not None)
    moments = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    adam = list(zip(params, grads, [m for m, _ in moments], [v for _, v in moments], lrs))
    n_step = [0]

    def step(k, marks=None):
        t = ts[k % len(ts)]
        if marks: ev.record(marks[0], sp)
        g4d.deform(G, P, M, t, S)
        g4d.render(S, cam, ws, img, T, nc)
        if marks: ev.record(marks[1], sp)
        g4d.l1_loss(img, target, loss, gimg)
        if marks: ev.record(marks[2], sp)
        g4d.render_backward(S, cam, ws, T, nc, gimg, gs)
        if marks: ev.record(marks[3], sp)
        g4d.deform_backward(G, P, M, t, gs, gd)
        if marks: ev.record(marks[4], sp)
        g4d.tv_loss(P, 1.0, tvl, gd)
        n_step[0] += 1
        g4d.adam_step(adam, n_step[0])
        if marks: ev.record(marks[5], sp)
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    assert g4d.read_status(ws).overflow == 0
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    marks = [[ev.create() for _ in range(6)] for _ in range(min(steps, 50))]
    for k, m in enumerate(marks):
        step(k, m)
    torch.cuda.synchronize()
    # medians: an event interval also holds any host delay before the next launch
    st = lambda i: round(float(np.median([ev.elapsed(m[i], m[i + 1]) for m in marks])), 4)
    evals = int(g4d.read_status(ws).blend_evals)
    rb_ms = float(np.median([ev.elapsed(m[2], m[3]) for m in marks]))
    return {"workload": TRAIN_WORKLOADS[which], "layout": layout,
            "steps": steps, "steps_per_s": round(steps / wall, 2), "ms_per_step": round(1e3 * wall / steps, 4),
            "stages_ms": {"forward": st(0), "loss": st(1), "render_backward": st(2), "deform_backward": st(3),
                          "tv_and_adam": st(4)},
            # the backward walk re-evaluates the forward's (pixel, Gaussian) pairs; its
            # VALU issue use is in the counter summary of the training iteration
            "render_backward": {"evaluated_pairs": evals, "ms": round(rb_ms, 4),
                                "ns_per_pair": round(rb_ms * 1e6 / max(evals, 1), 4)}}


def extra_measurements(steps, warmup, layout="morton"):
    """The large configuration (300k Gaussians, planes 64/128/256 x t150,
    MLP 96-128-10, 1352x1014) with the FP32 and the BF16-input MFMA MLP, the
    100k workload with the colour and opacity heads, the composition
    workload, and the 100k workload's generator swept over N at 800x800."""
    from paper_2310_08528_amd import g4d, synth
    out = {}
    log("extra: large configuration")
    sc4 = synth.config4()
    out["large"] = {"workload": "300k Gaussians (box + cluster, SH3), HexPlane 64/128/256 x t150 F32, "
                                "MLP 96-128-10, 1352x1014, 20 ring cameras x 300 timestamps",
                    "layout": layout,
                    "fp32_mlp": time_scene(sc4, g4d.MLP_F32, steps, warmup, n_frames=300, layout=layout),
                    "bf16_mlp": time_scene(sc4, g4d.MLP_BF16, steps, warmup, n_frames=300, layout=layout)}
    del sc4
    log("extra: colour and opacity heads")
    out["colour_opacity_heads"] = {
        "workload": "100k Gaussians, SH3, the 100k configuration's field; decoder with the colour "
                    "(48 rows) and opacity heads, 800x800",
        "fp32_mlp": time_scene(synth.config2(colour_opacity=True), g4d.MLP_F32, steps, warmup, layout=layout)}
    log("extra: composition")
    out["composition"] = time_composition(steps, warmup, layout=layout)
    out["sweep_n"] = {}
    for n in (10_000, 30_000, 100_000, 300_000):
        log(f"extra: N = {n}")
        out["sweep_n"][str(n)] = time_scene(synth.config2(n=n), g4d.MLP_F32, steps, warmup, layout=layout)
    return out


def _profile_json(name):
    md = open(os.path.join(ROOT, "profiles", name)).read()
    return json.loads(md.split("```json", 1)[1].split("```", 1)[0])


def _blend_source_hash():
    src = open(os.path.join(ROOT, "paper_2310_08528_amd", "csrc", "raster.hip")).read()
    a = src.index("// ---------------------------------------------------------------- k_blend")
    b = src.index("// ---------------------------------------------------------------- k_export")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def blend_counters():
    """Counter figures of one blend launch (HBM bytes, VALU and transcendental
    instructions, active cycles) from the committed counter summary, or None
    when the blend kernel's source has changed since they were taken."""
    try:
        data = _profile_json("k_blend_counters_100k_800x800.md")
        if _blend_source_hash() != data.get("kernel_source_sha256"):
            return None
        return data
    except (OSError, ValueError, IndexError, KeyError):
        return None


def rasterizer_traffic():
    """HBM bytes of every rasterizer kernel of one frame, from the committed
    counter summary, or None when the rasterizer source has changed."""
    try:
        data = _profile_json("k_blend_counters_100k_800x800.md")
        src = open(os.path.join(ROOT, "paper_2310_08528_amd", "csrc", "raster.hip")).read()
    except (OSError, ValueError, IndexError):
        return None
    if hashlib.sha256(src.encode()).hexdigest() != data.get("raster_source_sha256"):
        return None
    return int(data["rasterizer_bytes_per_frame"])


def main():
    import faulthandler
    # a hang names where it is stuck: every thread's stack to stderr after
    # four minutes without the run ending (the default run takes about two)
    faulthandler.dump_traceback_later(240, repeat=True, file=sys.stderr)
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=20)
    ap.add_argument("--cpu-single-frames", type=int, default=1)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--layout", choices=("morton", "index"), default="morton",
                    help="store the scene's Gaussians in the Morton order of their canonical means (a one-time "
                         "permutation before anything is timed) or as generated")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--in-flight", type=int, default=4,
                    help="frames in flight for the reported throughput (1 = one frame at a time)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the large configuration (FP32 and BF16 MLP) and a sweep over N")
    ap.add_argument("--profile-frames", type=int, default=0,
                    help="only run this many frames (deform + render, one at a time, after the copy "
                         "calibration if asked) and exit: the workload the committed profiles are taken on")
    ap.add_argument("--training", action="store_true",
                    help="only time the training iteration (2000 Gaussians, 800x800) and print its record")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the render would shard by requests or by image tiles)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_08528_amd import g4d, synth
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ev = HipEvents()
    if args.training:
        print(json.dumps({"training_step": time_training_step(args.steps, args.warmup),
                          "training_step_100k": time_training_step(min(args.steps, 50), min(args.warmup, 5),
                                                                   "100k", args.layout)}), flush=True)
        return

    sc = synth.config2(n=args.n)
    frames = [(k % len(sc.cameras), float(sc.timestamps[(k // len(sc.cameras)) % len(sc.timestamps)]))
              for k in range(len(sc.cameras) * len(sc.timestamps))]
    G = g4d.DeviceGaussians(sc.gaussians, dev)
    P = g4d.DevicePlanes(sc.planes, dev)
    M = g4d.DeviceMLP(sc.mlp, dev)
    S = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, dev)
    cams = [g4d.camera_struct(c) for c in sc.cameras]
    W, H = sc.cameras[0].width, sc.cameras[0].height
    img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    # size the instance capacity over every frame of the sequence (grow on overflow)
    capacity = 64 * G.n + 4096
    ws = g4d.RenderWorkspace(G.n, W, H, capacity, dev)
    if args.profile_frames:
        if args.layout == "morton":
            g4d.store_in_order(G, g4d.spatial_order(G, sc.planes.bmin, sc.planes.bmax, ws))
        if args.copy_calibration:
            src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(5):
                dst.copy_(src)
            del src, dst
        torch.cuda.synchronize()
        for k in range(args.profile_frames):
            ci, t = frames[k % len(frames)]
            g4d.deform(G, P, M, t, S)
            g4d.render(S, cams[ci], ws, img)
        torch.cuda.synchronize()
        st = g4d.read_status(ws)
        assert st.overflow == 0 and st.sort_error == 0
        print(json.dumps({"profile_frames": args.profile_frames, "layout": args.layout}), flush=True)
        return
    kmax = 0
    for (ci, t) in frames:
        g4d.deform(G, P, M, t, S)
        g4d.render(S, cams[ci], ws, img)
        st = g4d.read_status(ws)
        assert st.sort_error == 0
        kmax = max(kmax, int(st.instances))
        if st.overflow:
            del ws
            capacity = int(kmax * 1.25) + 4096
            ws = g4d.RenderWorkspace(G.n, W, H, capacity, dev)
    if capacity > int(kmax * 1.3) + 8192:
        del ws
        capacity = int(kmax * 1.05) + 4096
        ws = g4d.RenderWorkspace(G.n, W, H, capacity, dev)
    log(f"instances: max {kmax} over {len(frames)} frames, capacity {capacity}, "
        f"workspace {ws.ws.bytes / 2**20:.1f} MiB")
    if args.layout == "morton":
        # one-time scene preparation (as when a scene is loaded): the canonical
        # arrays stored in the Morton order of their means
        g4d.store_in_order(G, g4d.spatial_order(G, sc.planes.bmin, sc.planes.bmax, ws))
        torch.cuda.synchronize()

    # structs marshalled once; the loop only passes pointers
    lib = g4d.load()
    gs, ps, ms_, ss = G.struct(), P.struct(), M.struct(), S.struct()
    bG, bP, bM, bS, bW = (ctypes.byref(x) for x in (gs, ps, ms_, ss, ws.ws))
    bC = [ctypes.byref(c) for c in cams]
    ip = img.data_ptr()

    def step(k, stage_events=None):
        ci, t = frames[k % len(frames)]
        r1 = lib.g4d_deform(bG, bP, bM, ctypes.c_float(t), bS, sp)
        if stage_events is not None:
            lib.g4d_set_stage_events(stage_events, 9)
        r2 = lib.g4d_render(bS, bC[ci], bW, ip, None, None, sp)
        if stage_events is not None:
            lib.g4d_set_stage_events(None, 0)
        if r1 or r2:
            raise g4d.G4DError(r1 or r2, "bench step")

    log("warm-up")
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 x 256 MiB device-to-device copies")
        del src, dst

    # ---- timed region: K frames; HIP events around the blend kernel only
    log("timed region")
    K = args.steps
    blend_ev = [(ev.create(), ev.create()) for _ in range(K)]
    blend_arr = [(ctypes.c_void_p * 9)(*([None] * 7 + [a, b])) for a, b in blend_ev]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step(args.warmup + k, blend_arr[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fps = K / wall
    blend_ms = float(np.mean([ev.elapsed(a, b) for a, b in blend_ev]))
    st = g4d.read_status(ws)
    assert st.overflow == 0 and st.sort_error == 0

    log(f"timed: {fps:.1f} frames/s; frames in flight")
    # ---- the same K frames with several in flight: frame k runs (deform,
    # then render) on slot k % m, each slot with its own stream, splat
    # buffer, workspace and image, as m serving slots would
    m_max = max(8, args.in_flight)
    slot_S, slot_W, slot_I, slot_ws, keep = [bS], [bW], [ip], [ws], []
    for _ in range(m_max - 1):
        S_ = g4d.DeviceSplats(G.n, G.sh_degree, G.sh, dev)
        W_ = g4d.RenderWorkspace(G.n, W, H, capacity, dev)
        I_ = torch.empty_like(img)
        s_ = S_.struct()
        keep += [S_, W_, I_, s_]
        slot_ws.append(W_)
        slot_S.append(ctypes.byref(s_))
        slot_W.append(ctypes.byref(W_.ws))
        slot_I.append(I_.data_ptr())
    # slot 0 runs on the current stream, so m slots use m streams (a process
    # has four hardware queues); the others get streams of their own
    slot_streams = [torch.cuda.Stream() for _ in range(m_max - 1)]   # default priority
    slot_sp = [sp] + [x.cuda_stream for x in slot_streams]

    def in_flight(m, n_frames, k0):
        """Enqueue n_frames frames over m slots; returns the host time the
        enqueueing took."""
        t_host = time.perf_counter()
        for k in range(n_frames):
            b = k % m
            ci, t = frames[(k0 + k) % len(frames)]
            r1 = lib.g4d_deform(bG, bP, bM, ctypes.c_float(t), slot_S[b], slot_sp[b])
            r2 = lib.g4d_render(slot_S[b], bC[ci], slot_W[b], slot_I[b], None, None, slot_sp[b])
            if r1 or r2:
                raise g4d.G4DError(r1 or r2, "bench frames in flight")
        return time.perf_counter() - t_host

    flight = {}
    for m in sorted({1, 2, 3, 4, 6, 8, args.in_flight}):
        in_flight(m, args.warmup, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host_s = in_flight(m, K, args.warmup)
        torch.cuda.synchronize()
        flight[m] = time.perf_counter() - t0
        for w_ in slot_ws[:m]:
            st = g4d.read_status(w_)
            assert st.overflow == 0 and st.sort_error == 0
        log(f"{m} in flight: {K / flight[m]:.1f} frames/s (host enqueue {1e6 * host_s / K:.1f} us per frame)")
    wall_pipe = flight[args.in_flight]
    log("stage breakdown")
    # ---- per-stage breakdown (separate pass with events at every boundary)
    n_prof = min(K, 100)
    stage_ev = [[ev.create() for _ in range(9)] for _ in range(n_prof)]
    dfm_ev = [(ev.create(), ev.create()) for _ in range(n_prof)]
    for k in range(n_prof):
        ci, t = frames[(args.warmup + k) % len(frames)]
        ev.record(dfm_ev[k][0], sp)
        g4d.deform(G, P, M, t, S)
        ev.record(dfm_ev[k][1], sp)
        g4d.set_stage_events(stage_ev[k])
        g4d.render(S, cams[ci], ws, img)
        g4d.set_stage_events(None)
    torch.cuda.synchronize()
    stages = {"deform": float(np.mean([ev.elapsed(a, b) for a, b in dfm_ev]))}
    for i, name in enumerate(STAGES):
        stages[name] = float(np.mean([ev.elapsed(e[i], e[i + 1]) for e in stage_ev]))
    # ---- the blend's work over the timed frames: the same frames rendered
    # again with n_contrib and final_T (the variant that counts), not timed
    T_ = torch.empty((H, W), dtype=torch.float32, device=dev)
    nc_ = torch.empty((H, W), dtype=torch.int32, device=dev)
    evals_tot = comp_tot = 0
    for k in range(K):
        ci, t = frames[(args.warmup + k) % len(frames)]
        g4d.deform(G, P, M, t, S)
        g4d.render(S, cams[ci], ws, img, T_, nc_)
        st = g4d.read_status(ws)
        evals_tot += int(st.blend_evals)
        comp_tot += int(st.blend_composited)
    evals_per_frame = evals_tot / K
    comp_per_frame = comp_tot / K

    # ---- roofline of the dominant kernel (the blend: bound by VALU issue).
    # achieved: the method's operations (24 per evaluated pair) per second of
    # the blend's event-timed launch, against the published FP32 peak; the
    # counted figures (VALU instructions per launch from the counter summary)
    # give the issue utilisation beside it
    cnt = blend_counters()
    achieved = evals_per_frame * BLEND_OPS_PER_EVAL / (blend_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_blend<false>", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": int(cnt["traffic_bytes_per_launch"]) if cnt else None,
                "traffic_unit": "bytes/launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                "evaluated_pairs_per_frame": int(evals_per_frame),
                "composited_pairs_per_frame": int(comp_per_frame),
                "ops_per_evaluated_pair": BLEND_OPS_PER_EVAL, "avg_ms": round(blend_ms, 4)}
    if cnt:
        # wave64 VALU instructions of one launch (SQ_INSTS_VALU; a transcendental
        # occupies its SIMD four issue slots) over the issue slots of the launch
        slots = (cnt["valu_instructions_per_launch"] + 3 * cnt["trans_instructions_per_launch"])
        roofline["valu_instructions_per_launch"] = cnt["valu_instructions_per_launch"]
        roofline["valu_issue_utilization"] = round(slots / (PEAK_WAVE_INSTR_PER_S * blend_ms * 1e-3), 4)
        roofline["valu_instructions_per_composited_pair"] = round(
            cnt["valu_instructions_per_launch"] * 64 / max(comp_per_frame, 1), 2)

    # the rasterizer as a whole (counter bytes over its live time per frame)
    rbytes = rasterizer_traffic()
    r_ms = sum(stages[k] for k in STAGES)
    raster_hbm = {"bytes_per_frame": rbytes, "ms_per_frame": round(r_ms, 4),
                  "achieved_GBs": round(rbytes / (r_ms * 1e-3) / 1e9, 1) if rbytes else None,
                  "peak_GBs": PEAK_HBM_GBS,
                  "frac": round(rbytes / (r_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if rbytes else None}

    fps_flight = K / wall_pipe
    out = {"metric": METRIC, "value": round(fps_flight, 2), "unit": "frames/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": round(1e3 * wall_pipe / K, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "100k Gaussians (noisy sphere shell + 10% fill, SH3), HexPlane 64/128 x t25 "
                                  "F32, MLP 64-64-10 FP32, 800x800, 20 ring cameras x 20 timestamps",
                      "gaussians": G.n, "width": W, "height": H, "instances_max": kmax,
                      "capacity": capacity, "layout": args.layout},
           "stages_ms": {k: round(v, 4) for k, v in stages.items()},
           "roofline": roofline, "rasterizer_hbm": raster_hbm,
           "frames_in_flight": args.in_flight,
           "in_flight_frames_per_s": {str(m): round(K / w, 2) for m, w in sorted(flight.items())},
           "sequential": {"frames_per_s": round(fps, 2), "ms_per_frame": round(1e3 * wall / K, 4),
                          "how": "one frame at a time on one stream (deform, then render)"}}
    log("stages done")
    if not args.no_serve:
        out["serving"] = serving_bench(args.serve_seconds, args.serve_rate, args.serve_budget_gb, args.serve_slots,
                                       layout=args.layout)
    # the training direction on its own workload (a few seconds; not part of `value`)
    log("training iteration")
    out["training"] = time_training_step(200, 20)
    log("training iteration, 100k Gaussians")
    out["training_100k"] = time_training_step(50, 5, "100k", args.layout)
    if args.extra:
        out["extra"] = extra_measurements(min(K, 200), 20, args.layout)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(sc, frames, args.cpu_frames, args.cpu_single_frames)
    for e in blend_ev:
        ev.destroy(e[0]); ev.destroy(e[1])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

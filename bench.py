#!/usr/bin/env python
"""Benchmark of the streaming Gaussian-splatting hot path on one MI355X.

One step = one optimisation iteration of the shift stage over every view of a timestep:
  shift_apply (forward) -> render_fwd with the L1 term fused into its blend (all views, one
  launch sequence: loss gradient and error maps) -> render_bwd (full parameter gradients +
  historical positional gradient) -> shift_apply (adjoint) -> adam_step -> densify_append
  (children written into spare rows; the live count is not advanced, so every step sees the
  same scene size).
Inputs are synthetic and resident in device memory before timing starts.

Prints one JSON line (rank 0).  `python bench.py` defaults to one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Hardware queues per process, read when the HIP runtime starts: the serving legs run training
# and three render slots on streams of their own, and with HIP's default of 4 queues one slot
# shares the training stream's queue, where its renders wait behind training kernels (p50/p99
# 15/43 ms against 2.4/5.5 ms with 8 queues on the 500/s workload).  Set before torch loads
# (serving.MIN_HW_QUEUES states the same number for library users).
SERVING_HW_QUEUES = 8
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < SERVING_HW_QUEUES:
    os.environ["GPU_MAX_HW_QUEUES"] = str(SERVING_HW_QUEUES)

PEAK_FP32_FLOPS = 157.3e12   # MI355X fp32 vector, published
PEAK_HBM_BPS = 8.0e12        # MI355X HBM3E, published
# Algorithmic flops per (pixel, list entry) pair of the blend (counted from its definition):
#   alpha test of an entry: pixel offset (2), quadratic form (8), exp (1), opacity scale, clamp,
#   skip test (3) = 14; compositing a blended entry: transmittance update and stop test (3),
#   weight (1), three colour multiply-adds (6) = 10.
FWD_FLOPS_TEST, FWD_FLOPS_BLEND = 14, 10
# Backward, per entry walked from the pixel's last blended entry: alpha recomputed (14); for a
#   blended entry also transmittance recovery (2), colour gradient (4), alpha gradient (9),
#   colour-behind update (12), exponent / opacity gradient (2), mean and conic gradients (17) = 46.
BWD_FLOPS_TEST, BWD_FLOPS_BLEND = 14, 46


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tile_name(t) -> str:
    """'WxH' for 16x16 sub-tiles, 'WxHs8' for 8x8 sub-tiles (one pixel per lane)."""
    return f"{t[0]}x{t[1]}" + ("s8" if len(t) > 2 and int(t[2]) == 8 else "")


# LDS batches of the blend tried by the autotuner, in order of preference
BATCH_CANDIDATES = (128, 64, 256)


def autotune_name(key) -> str:
    """'WxH' (one batch tried) or 'WxH/bB' for an autotuner result key."""
    if len(key) == 2 and isinstance(key[1], int) and isinstance(key[0], tuple):
        return f"{tile_name(key[0])}/b{key[1]}"
    return tile_name(key)


def parse_tile(name: str):
    name = name.lower()
    sub = 8 if name.endswith("s8") else 16
    w, h = (int(x) for x in (name[:-2] if sub == 8 else name).split("x"))
    return (w, h, sub) if sub == 8 else (w, h)


def measured_traffic(kernel: str, workload: str, tile: str, batch: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None if
    there is none for this workload, tile size and blend batch, or the blend source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    src = os.path.join(ROOT, "paper_2411_14847_amd", "csrc", "raster.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if rec.get("kernel") != kernel or rec.get("workload") != workload or tile not in rec.get("by_tile", {}):
        return None
    if int(rec.get("batch", 128)) != int(batch):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("raster_hip_sha256"):
        return None
    return float(rec["by_tile"][tile]["traffic_bytes"])


def count_tile_keys(ctx, g, cams) -> int:
    """Tile keys of one render of g into cams at the context's tile size (sum of the visible
    Gaussians' tile-rectangle areas)."""
    total = 0
    for c in cams:
        pr = ctx.debug_projection(g, c)  # [n][16]: ..., x0, y0, x1, y1, visible
        vis = pr[:, 15] > 0.5
        total += int(((pr[vis, 13] - pr[vis, 11]) * (pr[vis, 14] - pr[vis, 12])).sum().item())
        del pr
    return total


def build_workload(args):
    import torch

    import synth
    from paper_2411_14847_amd import Context, GaussianBuffers, RenderOut
    from paper_2411_14847_amd.api import zeroed_grads

    if args.workload == "multiview":
        scene, cams, _ = synth.multiview_scene(args.seed, n=args.n, n_views=args.views, width=args.width,
                                               height=args.height, with_grads=False)
        name = f"multiview_{args.n // 1000}k_sh3_{args.views}x{args.width}x{args.height}"
        if getattr(args, "ssim_lambda", 0.0) > 0.0:
            name += f"_dssim{args.ssim_lambda:g}"
        if getattr(args, "shift", "direct") == "hash":
            name += "_hashfields"
    else:
        scene, cams, _ = synth.single_view_scene(args.seed)
        name = "single_view_2k_sh0_128x128"
    N = scene.n
    cap = N + args.densify_k
    g = GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh,
                                    scene.sh_degree, capacity=cap)
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    ctx = Context(max_gaussians=cap, max_views=len(cams), max_keys=args.max_keys or int(N * len(cams) * 24) + (1 << 20),
                  max_tiles=tiles)
    dev = "cuda"
    # dynamic group and its ground-truth motion (10% of the base Gaussians)
    motion = synth.timestep_motion(args.seed, 1, N)
    dyn = torch.as_tensor(motion.dynamic, device=dev)
    nd = int(dyn.numel())
    # shifted copy: separate mean/quat planes, the other planes alias the scene's
    gs = GaussianBuffers(torch.zeros_like(g.mean), torch.zeros_like(g.quat), g.log_scale, g.logit, g.sh, g.n,
                         g.n_base, g.sh_degree)
    # targets: the ground truth moved by its motion, rendered once
    ctx.shift_fwd(g, gs, dyn, torch.as_tensor(motion.dpos, device=dev), torch.as_tensor(motion.dquat, device=dev))
    targets = [o.rgb.clone() for o in ctx.render_fwd(gs, cams, args.bg)]
    ctx.sync()
    # the step's accumulators (gradients, loss, historical gradient sums, offset gradients) share
    # one buffer, cleared by one fill per step
    zbuf, zgrads, zextra = zeroed_grads(g, [((1,), torch.float32), ((cap,), torch.float32), ((cap,), torch.int32),
                                            ((3, nd), torch.float32), ((4, nd), torch.float32)])
    st = dict(
        torch=torch, ctx=ctx, g=g, gs=gs, cams=cams, dyn=dyn, targets=targets, name=name, scene=scene,
        outs=[RenderOut.allocate(c) for c in cams],
        dls=[torch.zeros(3, c.height, c.width, device=dev) for c in cams],
        errs=[torch.zeros(c.height, c.width, device=dev) for c in cams],
        ssim_scratch=([torch.empty(9 * c.height * c.width, device=dev) for c in cams]
                      if getattr(args, "ssim_lambda", 0.0) > 0.0 else None),
        zbuf=zbuf, grads=zgrads, loss=zextra[0], gn=zextra[1], cnt=zextra[2], d_dpos=zextra[3], d_drot=zextra[4],
        dpos=torch.zeros(3, nd, device=dev), drot=torch.cat([torch.ones(1, nd), torch.zeros(3, nd)]).to(dev),
        m=[torch.zeros(3, nd, device=dev), torch.zeros(4, nd, device=dev)],
        v=[torch.zeros(3, nd, device=dev), torch.zeros(4, nd, device=dev)],
        n_app=torch.zeros(1, dtype=torch.int32, device=dev), nd=nd, N=N, cap=cap,
    )
    if getattr(args, "shift", "direct") == "hash":
        # H_dyn over the dynamic rows, H_st over the static ones (N3DV table sizes, App. B); offsets
        # laid out [dynamic | static] over all N base rows
        from paper_2411_14847_amd import HashField, geometric_res
        import numpy as np
        st_rows = np.setdiff1d(np.arange(N, dtype=np.int32), motion.dynamic).astype(np.int32)
        rows = torch.as_tensor(np.concatenate([motion.dynamic, st_rows]).astype(np.int32), device=dev)
        lo = (scene.mean.min(axis=1) - 0.1).tolist()
        hi = (scene.mean.max(axis=1) + 0.1).tolist()
        fields = {"dyn": HashField.init(geometric_res(16, 2048, 16), 4, 16, 64, lo, hi, dev, seed=1),
                  "st": HashField.init(geometric_res(16, 2048, 16), 2, 14, 64, lo, hi, dev, seed=2)}
        for f in fields.values():  # a field part-way through its optimisation: a non-zero output layer
            f.w2.normal_(0.0, 1e-3)
        # H_dyn runs on a second stream with its own context (a context's calls may not overlap):
        # its 20k queries cannot fill the GPU alone, so they share it with H_st's 180k
        ctx_dyn = Context(max_gaussians=N, max_views=1, max_keys=1 << 10, max_tiles=16)
        st.update(ctx_dyn=ctx_dyn, side=torch.cuda.Stream())
        st.update(rows=rows, dyn_rows=rows[:nd], st_rows=rows[nd:], ns=N - nd, fields=fields,
                  field_grads={k: f.zeros_like() for k, f in fields.items()},
                  field_mv={k: (f.zeros_like(), f.zeros_like()) for k, f in fields.items()},
                  dpos=torch.zeros(3, N, device=dev), drot=torch.cat([torch.ones(1, N), torch.zeros(3, N)]).to(dev),
                  d_dpos=torch.zeros(3, N, device=dev), d_drot=torch.zeros(4, N, device=dev))
    return st


def train_step(s, it, args, per_view=False, overlap=True):
    """One training step; with `overlap` the H_dyn field runs on a second stream beside H_st,
    without it (graph capture: a captured fork replays on separate hardware queues) on the
    current stream."""
    ctx, g, gs, cams = s["ctx"], s["g"], s["gs"], s["cams"]
    fields = s.get("fields")
    if fields:
        nd, ns = s["nd"], s["ns"]
        torch = s["torch"]
        main = torch.cuda.current_stream()
        side = s["side"] if overlap else main
        for f in s["field_grads"].values():
            for t in f.arrays():
                t.zero_()
        if overlap:
            side.wait_stream(main)
        s["ctx_dyn"].hash_field_fwd(fields["dyn"], g.mean, s["N"], s["dyn_rows"], nd, s["dpos"], s["drot"], col=0,
                                    stream=side)
        ctx.hash_field_fwd(fields["st"], g.mean, s["N"], s["st_rows"], ns, s["dpos"], s["drot"], col=nd)
        if overlap:
            main.wait_stream(side)
        ctx.shift_fwd(g, gs, s["rows"], s["dpos"], s["drot"])
    else:
        ctx.shift_fwd(g, gs, s["dyn"], s["dpos"], s["drot"])
    s["zbuf"].zero_()
    if fields:  # the fields' offset gradients cover every base row (their own buffers)
        s["d_dpos"].zero_()
        s["d_drot"].zero_()
    lam = getattr(args, "ssim_lambda", 0.0)
    if not per_view and lam > 0.0:
        # Eq. (3) with its D-SSIM term: the render, then the fidelity loss over the images
        ctx.render_fwd(gs, cams, args.bg, out=s["outs"])
        ctx.fidelity_loss_grad(cams, [o.rgb for o in s["outs"]], s["targets"], lam, s["dls"], s["errs"], s["loss"],
                               scratch=s["ssim_scratch"])
        ctx.render_bwd(gs, cams, args.bg, s["outs"], s["dls"], s["grads"], s["gn"], s["cnt"])
    elif not per_view:
        # render fused with the L1 term (the step reads only the loss gradient, error maps and the
        # forward's transmittance / contributor counts, so the images are not written)
        ctx.render_fwd_l1(gs, cams, args.bg, s["targets"], s["dls"], s["errs"], s["loss"], out=s["outs"],
                          keep_rgb=False)
        ctx.render_bwd(gs, cams, args.bg, s["outs"], s["dls"], s["grads"], s["gn"], s["cnt"])
    else:
        # plain per-view path: one render_fwd / loss / render_bwd per camera
        V = len(cams)
        for v in range(V):
            ctx.render_fwd(gs, cams[v:v + 1], args.bg, out=s["outs"][v:v + 1])
            if lam > 0.0:
                ctx.fidelity_loss_grad(cams[v:v + 1], [s["outs"][v].rgb], s["targets"][v:v + 1], lam,
                                       s["dls"][v:v + 1], s["errs"][v:v + 1], s["loss"], scratch=[s["ssim_scratch"][v]])
            else:
                ctx.l1_loss_grad(cams[v:v + 1], [s["outs"][v].rgb], s["targets"][v:v + 1], s["dls"][v:v + 1],
                                 s["errs"][v:v + 1], s["loss"])
            s["dls"][v].mul_(1.0 / V)
            ctx.render_bwd(gs, cams[v:v + 1], args.bg, s["outs"][v:v + 1], s["dls"][v:v + 1], s["grads"], s["gn"],
                           s["cnt"])
    if fields:
        ctx.shift_adjoint(g, s["rows"], s["drot"], s["grads"], s["d_dpos"], s["d_drot"])
        if overlap:
            side.wait_stream(main)
        s["ctx_dyn"].hash_field_bwd(fields["dyn"], g.mean, s["N"], s["dyn_rows"], nd, s["d_dpos"], s["d_drot"],
                                    s["field_grads"]["dyn"], col=0, stream=side)
        ctx.hash_field_bwd(fields["st"], g.mean, s["N"], s["st_rows"], ns, s["d_dpos"], s["d_drot"],
                           s["field_grads"]["st"], col=nd)
        if overlap:
            main.wait_stream(side)
        groups = []
        for k, f in fields.items():
            m, v = s["field_mv"][k]
            groups += [(p, gr, mm, vv, args.lr_field) for p, gr, mm, vv in
                       zip(f.arrays(), s["field_grads"][k].arrays(), m.arrays(), v.arrays())]
        ctx.adam_step(groups, step=it)
    else:
        ctx.shift_adjoint(g, s["dyn"], s["drot"], s["grads"], s["d_dpos"], s["d_drot"])
        ctx.adam_step([(s["dpos"], s["d_dpos"], s["m"][0], s["v"][0], args.lr_pos),
                       (s["drot"], s["d_drot"], s["m"][1], s["v"][1], args.lr_rot)], step=it,
                      d_step=s.get("d_step") if it is None else None)
    # (a replayed graph keeps the densify seed of its capture; Adam counts its steps on the device)
    ctx.densify_append(g, s["errs"], cams, s["gn"], s["cnt"], 0.0, 0.0, 0.0, args.densify_k,
                       0 if it is None else it, s["n_app"])


def time_steps(s, args, k, warm, per_view=False):
    torch = s["torch"]
    for i in range(warm):
        train_step(s, i + 1, args, per_view)
    torch.cuda.synchronize()
    s["ctx"].sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for i in range(k):
        train_step(s, warm + i + 1, args, per_view)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s["ctx"].sync()
    return e0.elapsed_time(e1) / k, wall


def time_graph_steps(s, args, k, warm, first_step):
    """The same training step captured once in a HIP graph and replayed k times (after `warm`
    untimed replays): Adam's step count lives on the device and advances per replay."""
    torch = s["torch"]
    s["d_step"] = torch.full((1,), first_step - 1, dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        train_step(s, None, args, overlap=False)  # warm-up on a side stream (also a real step)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        train_step(s, None, args, overlap=False)
    for _ in range(warm):
        graph.replay()
    torch.cuda.synchronize()
    s["ctx"].sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(k):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    s["ctx"].sync()
    del graph
    return e0.elapsed_time(e1) / k


def render_latency(s, args, reps):
    """Latency of one full-resolution novel-view render (view 0) on an idle GPU."""
    torch = s["torch"]
    ctx, gs, cam = s["ctx"], s["gs"], s["cams"][0]
    out = s["outs"][0:1]
    times = []
    for _ in range(5):
        ctx.render_fwd(gs, [cam], args.bg, out=out)
    torch.cuda.synchronize()
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.render_fwd(gs, [cam], args.bg, out=out)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.percentile(times, 50)), float(np.percentile(times, 99))


def fwdbwd_latency(s, args, reps):
    """Mean latency of zeroing the gradients + render_fwd + render_bwd over all views, issued
    eagerly and as one replayed HIP graph (launch overhead vs kernel time at small sizes)."""
    torch = s["torch"]
    ctx, gs, cams, outs, dls, grads = s["ctx"], s["gs"], s["cams"], s["outs"], s["dls"], s["grads"]

    def step():
        for t in grads.planes():
            t.zero_()
        ctx.render_fwd(gs, cams, args.bg, out=outs)
        ctx.render_bwd(gs, cams, args.bg, outs, dls, grads)

    def timed(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    eager = timed(step)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    replay = timed(graph.replay)
    ctx.sync()
    return eager, replay


def feature_render_times(s, args):
    """16-channel identity features of every view from the render's lists (Gaussian Grouping's
    render M, Sec. 3.3) and the dynamics mask built on them, timed with events after one render."""
    torch = s["torch"]
    import synth
    ctx, g, cams = s["ctx"], s["gs"], s["cams"]
    feat, _, cls_w, cls_b = synth.identity_setup(args.seed + 3, s["N"], n_objects=64)
    fdev = torch.zeros(16, g.capacity, device="cuda")
    fdev[:, :s["N"]] = torch.as_tensor(feat, device="cuda")
    # flow above the threshold in a few small discs of the first view only (the other views still
    # run the pixel pass)
    flows = [torch.as_tensor(f, device="cuda") for f in synth.flow_maps(args.seed + 4, cams[:1], frac=0.002)]
    flows += [torch.zeros(c.height, c.width, device="cuda") for c in cams[1:]]
    W, B = torch.as_tensor(cls_w, device="cuda"), torch.as_tensor(cls_b, device="cuda")
    idx = torch.zeros(g.capacity, dtype=torch.int32, device="cuda")
    nd = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.render_fwd(g, cams, args.bg, out=s["outs"])
    out = [torch.empty(16, c.height, c.width, device="cuda") for c in cams]
    ctx.render_features(g, cams, fdev, out=out)
    ctx.dynamic_mask(cams, out, flows, 1.0, W, B, fdev, s["N"], idx, nd)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(args.feature_reps):
        ctx.render_features(g, cams, fdev, out=out)
    e[1].record()
    for _ in range(args.feature_reps):
        ctx.dynamic_mask(cams, out, flows, 1.0, W, B, fdev, s["N"], idx, nd)
    e[2].record()
    torch.cuda.synchronize()
    ms_f = e[0].elapsed_time(e[1]) / args.feature_reps
    ms_m = e[1].elapsed_time(e[2]) / args.feature_reps
    log(f"[bench] identity features (16 ch, {len(cams)} views) {ms_f:.3f} ms; dynamics mask {ms_m:.3f} ms "
        f"({int(nd.item())} dynamic Gaussians)")
    return {"channels": 16, "render_ms_all_views": round(ms_f, 4), "dynamic_mask_ms": round(ms_m, 4),
            "n_objects": 64, "n_dynamic": int(nd.item())}


def host_cpu():
    """(CPU model name, threads this process may use, capped at the 16-thread share of a one-GPU
    host)."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return model, max(1, min(n, 16))


def oracle_fwd_bwd(scene, cam, bg, seed):
    """One fwd+bwd of the oracle on one view with a seeded upstream gradient N(0, 1)."""
    import oracle
    rng = np.random.default_rng(seed)
    dl = rng.normal(0, 1, size=(3, cam.height, cam.width)).astype(np.float32)
    vr = oracle.render_view(scene, cam, bg=bg)
    oracle.render_backward(scene, [cam], [dl], bg=bg, renders=[vr])


def cpu_baseline(s, args):
    """The oracle (float64 C, untuned) on a bounded sample of the same workload: view 0 fwd+bwd
    on one thread, then views 0..T-1 at once on T threads (one view per thread; the oracle's C
    calls release the interpreter lock), T = the host threads this process may use (at most 16).
    Scaled to iterations of all views: value = T views / wall time / n_views."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    scene, cams = s["scene"], s["cams"]
    V = len(cams)
    model, T = host_cpu()
    T = min(T, V)
    oracle.lib()
    t0 = time.perf_counter()
    oracle_fwd_bwd(scene, cams[0], args.bg, args.seed + 7)
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=T) as ex:
        list(ex.map(lambda v: oracle_fwd_bwd(scene, cams[v], args.bg, args.seed + 7 + v), range(T)))
    dtT = time.perf_counter() - t0
    cam = cams[0]
    return {"value": T / dtT / V, "unit": "iters/s", "cores": T, "kind": "oracle",
            "sample": f"views 0..{T - 1} of {V} ({cam.width}x{cam.height}, {scene.n} Gaussians), fwd+bwd, one "
                      f"view per thread on {T} threads: {dtT:.1f} s; value = {T} / ({V} x that time)",
            "cpu": model,
            "single_thread": {"value": 1.0 / (dt1 * V), "cores": 1,
                              "sample": f"view 0 fwd+bwd on one thread: {dt1:.1f} s; value = 1 / ({V} x that time)"}}


def bench_oracle_timings(args):
    """Host-only timings of the oracle (float64 C, untuned) on the other workloads: medians of 5
    runs after one warm-up, on one thread and with one view per thread over T threads.
      single view: 2,000 Gaussians SH0 at 128x128, fwd+bwd;
      streaming: one iteration (shift, 20-view fwd, L1 gradient, 20-view bwd, shift adjoint,
        Adam) of the 2,000-Gaussian scene on the 20-camera 128x128 rig, times 100 per timestep;
      stress sub-scene: the large-footprint generator at 64 Gaussians, four 32x32 views, fwd+bwd;
      serving: one render of the 200k-Gaussian scene at 640x480, 1280x720 and 1920x1080."""
    import oracle
    import synth
    from concurrent.futures import ThreadPoolExecutor
    model, T = host_cpu()
    oracle.lib()
    bg = args.bg

    def median_s(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    res = {}
    scene, cams1, _ = synth.single_view_scene(args.seed)
    res["single_view_2k_sh0_128x128_fwd_bwd_ms"] = 1e3 * median_s(lambda: oracle_fwd_bwd(scene, cams1[0], bg, 1))
    log(f"[oracle] single view {res['single_view_2k_sh0_128x128_fwd_bwd_ms']:.1f} ms")
    rig = synth.streaming_rig(128, 128)
    motion = synth.timestep_motion(args.seed, 1, scene.n)
    rng = np.random.default_rng(args.seed + 11)
    targets = [rng.uniform(0, 1, size=(3, 128, 128)) for _ in rig]
    nd = motion.dynamic.size
    dpos = np.zeros((3, nd)); drot = np.concatenate([np.ones((1, nd)), np.zeros((3, nd))])
    mom = [np.zeros((3, nd)), np.zeros((4, nd))]
    vel = [np.zeros((3, nd)), np.zeros((4, nd))]

    def iteration(threads):
        m, q = oracle.shift_fwd(scene, motion.dynamic, dpos, drot)
        sc = synth.Scene(m.astype(np.float32), q.astype(np.float32), scene.log_scale, scene.logit, scene.sh,
                         scene.sh_degree)
        with ThreadPoolExecutor(max_workers=threads) as ex:
            vrs = list(ex.map(lambda c: oracle.render_view(sc, c, bg=bg), rig))
        _, dls, _ = oracle.l1_loss_grad(np.stack([v.rgb for v in vrs]), np.stack(targets))

        def bwd(v):
            return oracle.render_backward(sc, [rig[v]], [dls[v]], bg=bg, renders=[vrs[v]])[0]
        with ThreadPoolExecutor(max_workers=threads) as ex:
            gs = list(ex.map(bwd, range(len(rig))))
        gm = sum(g.mean for g in gs)
        gq = sum(g.quat for g in gs)
        dm, dq = oracle.shift_adj(sc, motion.dynamic, drot, gm, gq)
        for i, (p, g) in enumerate(((dpos, dm), (drot, dq))):
            oracle.adam(p, g, mom[i], vel[i], 1e-3, 0.9, 0.999, 1e-15, 1)

    for th in (1, T):
        ms = 1e3 * median_s(lambda: iteration(th), reps=3)
        res[f"streaming_iteration_20x128x128_ms_T{th}"] = ms
        res[f"streaming_ms_per_timestep_100_iters_T{th}"] = 100.0 * ms
        log(f"[oracle] streaming iteration {ms:.1f} ms on {th} threads")
    sub, subcams = synth.large_footprint_scene(args.seed, n=64, width=32, height=32)
    res["stress_subscene_64_4x32x32_fwd_bwd_ms"] = 1e3 * median_s(
        lambda: [oracle_fwd_bwd(sub, c, bg, 3) for c in subcams])
    big, _, _ = synth.multiview_scene(args.seed, n=args.n, n_views=1, width=64, height=64, with_grads=False)
    pos = synth.rig_positions()
    for W, H in synth.RESOLUTIONS:
        cam = synth.make_camera(np.eye(3), pos[7], W, H)
        res[f"serving_render_{W}x{H}_ms"] = 1e3 * median_s(lambda: oracle.render_view(big, cam, bg=bg), reps=3)
        log(f"[oracle] render {W}x{H} {res[f'serving_render_{W}x{H}_ms']:.0f} ms")
    line = {"metric": "oracle (float64 C) timings on the host", "value": None, "unit": "ms", "n_gpus": 0,
            "cpu": model, "threads": T, "data": "synthetic",
            "timings_ms": {k: round(v, 3) for k, v in res.items()}}
    print(json.dumps(line), flush=True)


def _scene_buffers(scene, capacity):
    from paper_2411_14847_amd import GaussianBuffers
    return GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh,
                                       scene.sh_degree, capacity=capacity)


def _gt_targets(ctx, gt, gt_next, cams, seed, t, bg):
    """Advances the ground-truth trajectory to timestep t (10% of the base Gaussians moved by a
    seeded position and small-angle rotation delta) and renders its target images once."""
    import torch
    import synth
    m = synth.timestep_motion(seed, t, gt.n_base)
    dyn = torch.as_tensor(m.dynamic, device="cuda")
    ctx.shift_fwd(gt, gt_next, dyn, torch.as_tensor(m.dpos, device="cuda"), torch.as_tensor(m.dquat, device="cuda"))
    for d, s_ in zip(gt.planes(), gt_next.planes()):
        d.copy_(s_)
    imgs = [o.rgb.clone() for o in ctx.render_fwd(gt, cams, bg)]
    return dyn, imgs


def _psnr(outs, targets):
    import math
    mse = sum(float(((o.rgb - t) ** 2).mean().item()) for o, t in zip(outs, targets)) / len(outs)
    return 10.0 * math.log10(1.0 / max(mse, 1e-20))


def bench_streaming(args):
    """Per-timestep streaming optimisation on the 2,000-Gaussian SH0 scene seen by a 20-camera rig
    at 128x128: each timestep moves 10% of the Gaussians, runs `iters` shift/render/loss/adjoint/
    Adam iterations against that timestep's ground-truth renders, then appends up to densify_k
    Gaussians; G^var is erased every 20 timesteps.  Targets are rendered before each timestep's
    timer starts.  Reports ms/timestep for the batched path (HIP-graph replay and eager) and for
    the plain per-view loop."""
    import torch
    import synth
    from paper_2411_14847_amd import Context
    from paper_2411_14847_amd.streaming import StreamConfig, Trainer

    if args.stream_scene == "multiview":
        # the benchmark's full-scale scene: 200k Gaussians (SH3) seen by 20 cameras at 1352x1014
        scene, cams, _ = synth.multiview_scene(args.seed, n=args.n, n_views=args.views, width=args.width,
                                               height=args.height, with_grads=False)
    else:
        scene, cam1, _ = synth.single_view_scene(args.seed)
        cams = synth.streaming_rig(128, 128) if args.stream_views == 20 else cam1
    N = scene.n
    cap = N + 20 * args.densify_k
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    gctx = Context(max_gaussians=N, max_views=len(cams), max_keys=N * len(cams) * 64 + (1 << 20), max_tiles=tiles)
    gt = _scene_buffers(scene, N)
    gt_next = gt.clone()
    targets, dyns = [], []
    for t in range(1, args.timesteps + 1):
        dyn, imgs = _gt_targets(gctx, gt, gt_next, cams, args.seed, t, args.bg)
        dyns.append(dyn)
        targets.append(imgs)
    gctx.sync()
    variants = [("batched_graph", dict(use_graph=True)), ("batched_eager", dict(use_graph=False))]
    if args.per_view_steps > 0:
        variants.append(("per_view_eager", dict(use_graph=False, per_view=True)))
    res = {}
    for name, kw in variants:
        g = _scene_buffers(scene, cap)
        ctx = Context(max_gaussians=cap, max_views=len(cams), max_keys=cap * len(cams) * 8 + (1 << 20),
                      max_tiles=tiles)
        cfg = StreamConfig(iters=args.iters, k_append=args.densify_k, seed=args.seed, shift=args.shift,
                           inherit_iters=args.inherit_iters, **kw)
        tr = Trainer(ctx, g, cams, max_dynamic=int(dyns[0].numel()), cfg=cfg)
        tuned = None
        if args.tile:
            ctx.tile = parse_tile(args.tile)
        elif not args.no_tile_autotune and name != "per_view_eager":
            # tile size from the autotuner on the first timestep's render (one iteration first)
            tr.begin_timestep(1, dyns[0])
            tr.set_targets(targets[0])
            tr.iteration()
            tuned = tr.autotune_tile()
            log(f"[bench] streaming {name}: autotune {tuned}; using {ctx.tile}, batch {ctx.batch}")
        T = args.timesteps if name != "per_view_eager" else min(args.timesteps, args.per_view_timesteps)
        rows = []
        prof_from = T - 2 if name == "batched_eager" and T >= 3 else None
        for t in range(1, T + 1):
            if t == prof_from:
                ctx.profile_begin(max_records=3 * (args.iters + 2))
            r = tr.timestep(t, dyns[t - 1], targets[t - 1])
            r["psnr"] = _psnr(tr.outs, targets[t - 1])
            rows.append(r)
        stages = ctx.profile_end() if prof_from is not None else None
        ctx.sync()
        ms = [r["ms"] for r in rows]
        steady = ms[1:] if len(ms) > 1 else ms
        res[name] = {"timesteps": T, "ms_per_timestep": round(float(np.mean(steady)), 3),
                     "ms_first_timestep": round(ms[0], 3), "n_final": rows[-1]["n"],
                     "loss_first_last_final_t": [rows[-1]["loss_first"], rows[-1]["loss_last"]],
                     "psnr_final_t": round(rows[-1]["psnr"], 2),
                     "mean_loss_drop": float(np.mean([r["loss_first"] - r["loss_last"] for r in rows])),
                     "ms_series": [round(r["ms"], 1) for r in rows], "n_series": [r["n"] for r in rows],
                     "inherited_series": [r["inherited"] for r in rows], "pruned_series": [r["pruned"] for r in rows],
                     "tile": tile_name(ctx.tile), "blend_batch": ctx.batch}
        if stages is not None:
            res[name]["stage_ms_per_timestep_last3"] = {k: round(v[0] / 3.0, 3) for k, v in stages.items()}
        log(f"[bench] streaming {name}: {res[name]}")
        del tr, ctx, g
        torch.cuda.empty_cache()
    main_ = res["batched_graph"]
    line = {
        "metric": (f"streaming ms/timestep ({args.iters} iterations + append) on the "
                   + ("2k-Gaussian scene, 20-view rig 128x128" if args.stream_scene == "rig" else
                      f"{N // 1000}k-Gaussian scene, {len(cams)} views {cams[0].width}x{cams[0].height}")),
        "value": main_["ms_per_timestep"], "unit": "ms/timestep", "n_gpus": 1, "steps": args.timesteps,
        "warmup": 1, "ms_per_step": round(main_["ms_per_timestep"] / max(1, args.iters), 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"streaming_2k_sh0_{len(cams)}x128x128" if args.stream_scene == "rig" else
                                f"streaming_{N // 1000}k_sh3_{len(cams)}x{cams[0].width}x{cams[0].height}")
                               + ("_hashfields" if args.shift == "hash" else "")
                               + (f"_inherit{args.inherit_iters}" if args.inherit_iters else ""),
                   "iters_per_timestep": args.iters, "inherit_iters": args.inherit_iters, "shift": args.shift,
                   "densify_k": args.densify_k, "erase_every": 20, "dynamic_fraction": 0.1},
        "variants": res,
    }
    print(json.dumps(line), flush=True)


def serving_leg(args, n_requests):
    """Continuous-batching render serving of the 200k-Gaussian SH3 scene while a training thread
    runs timesteps of the streaming loop on the 20-view 1352x1014 rig (its own stream) and
    publishes each finished timestep.  Requests arrive Poisson at `rate` from 64 viewers, at
    640x480, 1280x720 or 1920x1080; latency is arrival to completion event.  Returns the
    figures of the open-loop run with training, of a closed batch without training, and the
    training times."""
    import threading
    import torch
    import synth
    from paper_2411_14847_amd import Context
    from paper_2411_14847_amd.serving import RenderServer, Request, SceneSnapshots, serve_requests
    from paper_2411_14847_amd.streaming import StreamConfig, Trainer

    scene, cams, _ = synth.multiview_scene(args.seed, n=args.n, n_views=args.views, width=args.width,
                                           height=args.height, with_grads=False)
    N = scene.n
    cap = N + 20 * args.densify_k
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    ctx = Context(max_gaussians=cap, max_views=len(cams), max_keys=int(cap * len(cams) * 24) + (1 << 20),
                  max_tiles=tiles)
    g = _scene_buffers(scene, cap)
    gt = _scene_buffers(scene, N)
    gt_next = gt.clone()
    cfg = StreamConfig(iters=args.iters, k_append=args.densify_k, seed=args.seed, use_graph=True,
                       max_inflight=args.max_inflight)
    tr = Trainer(ctx, g, cams, max_dynamic=int(round(0.1 * N)), cfg=cfg)
    snaps = SceneSnapshots(g)
    snaps.publish(g)
    server = RenderServer(snaps, max_gaussians=cap, n_slots=args.slots, max_batch=args.max_batch,
                          max_tiles=args.max_batch * 8160, keys_per_tile=args.keys_per_tile)
    reqs = [Request(i, r.arrival_s, r.camera)
            for i, r in enumerate(synth.serving_requests(args.seed, n_requests=n_requests, rate_hz=args.rate))]
    train_stream = torch.cuda.Stream()
    t_state = {"t": 0}

    def train_one():
        t_state["t"] += 1
        t = t_state["t"]
        dyn, imgs = _gt_targets(ctx, gt, gt_next, cams, args.seed, t, args.bg)
        r = tr.timestep(t, dyn, imgs)
        snaps.publish(g, torch.cuda.current_stream())
        return r

    # warm-up: one training timestep alone, then one batch per slot
    with torch.cuda.stream(train_stream):
        alone = [train_one() for _ in range(args.train_alone)]
    torch.cuda.synchronize()
    for slot in server.slots:
        server.launch(slot, reqs[:min(3, len(reqs))])
    torch.cuda.synchronize()
    for slot in server.slots:
        slot.ctx.sync(slot.stream)
        slot.busy, slot.event, slot.batch = False, None, []
    # capacity: every request of a closed batch submitted at t = 0, no training
    cap_reqs = [Request(i, 0.0, r.camera) for i, r in enumerate(reqs[:args.capacity_requests])]
    st_cap = serve_requests(server, cap_reqs)
    server.latencies.clear()
    server.completed = server.retried = 0
    log(f"[bench] serving capacity (closed batch of {len(cap_reqs)}, no training): {st_cap}")
    # open loop with concurrent training
    stop = threading.Event()
    during = []

    def trainer_loop():
        with torch.cuda.stream(train_stream):
            while not stop.is_set():
                during.append(train_one())

    th = threading.Thread(target=trainer_loop)
    th.start()
    st = serve_requests(server, reqs)
    stop.set()
    th.join()
    torch.cuda.synchronize()
    log(f"[bench] serving with training: {st}; training ms/timestep {[round(d['ms'], 1) for d in during]}")
    train_alone_ms = float(np.mean([a["ms"] for a in alone[1:]] or [a["ms"] for a in alone]))
    return {
        "workload": f"serving_{N // 1000}k_sh3_poisson{int(args.rate)}_64viewers_mixedres",
        "requests": len(reqs), "slots": args.slots, "max_batch": args.max_batch,
        "training": f"{len(cams)} views {args.width}x{args.height}, {args.iters} iters/timestep",
        "frames_per_s": round(st["frames_per_s"], 2),
        "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3), "retried": st["retried"],
        "train_ms_per_timestep_concurrent": round(float(np.mean([d["ms"] for d in during])), 2) if during else None,
        "timesteps_during_serving": len(during),
        "train_ms_per_timestep_alone": round(train_alone_ms, 2),
        "capacity_frames_per_s": round(st_cap["frames_per_s"], 2),
        "capacity_p50_ms": round(st_cap["p50_ms"], 3), "capacity_p99_ms": round(st_cap["p99_ms"], 3),
    }


def bench_serving(args):
    """The serving leg alone, with its own JSON line (frames/s, p50/p99)."""
    r = serving_leg(args, args.requests)
    line = {
        "metric": "serving frames/s and p50/p99 latency (Poisson 500/s, mixed 640x480..1920x1080, 200k Gaussians) "
                  "with concurrent training",
        "value": r["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": r["requests"], "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {k: r[k] for k in ("workload", "requests", "slots", "max_batch", "training")},
    }
    line.update({k: v for k, v in r.items() if k not in line["config"] and k != "frames_per_s"})
    print(json.dumps(line), flush=True)


def bench_stress(args):
    """Large-footprint stress: 1,000,000 Gaussians (SH3, log-scales N(-2, 0.5), about 680 tiles
    per Gaussian), four 1920x1080 views; one step = zero gradients + render_fwd + render_bwd with
    upstream gradients N(0, 1), captured once in a HIP graph and replayed."""
    import torch
    import synth
    from paper_2411_14847_amd import Context, RenderOut

    t0 = time.perf_counter()
    scene, cams = synth.large_footprint_scene(args.seed, n=args.stress_n)
    log(f"[bench] stress scene generated in {time.perf_counter() - t0:.1f}s")
    N = scene.n
    g = _scene_buffers(scene, N)
    del scene
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    max_keys = args.max_keys or 0xFFFF0000
    ctx = Context(max_gaussians=N, max_views=len(cams), max_keys=max_keys, max_tiles=tiles)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed)
    dls = [torch.randn(3, c.height, c.width, device="cuda", generator=gen) for c in cams]
    outs = [RenderOut.allocate(c) for c in cams]
    grads = g.zeros_like()

    def step():
        for t in grads.planes():
            t.zero_()
        ctx.render_fwd(g, cams, args.bg, out=outs)
        ctx.render_bwd(g, cams, args.bg, outs, dls, grads)

    tuned = None
    if not args.no_autotune:
        tuned = ctx.autotune_tile(g, cams, args.bg, outs, dls, grads, reps=2, batches=BATCH_CANDIDATES)
        log(f"[bench] stress autotune (ms per fwd+bwd): {tuned}; using {ctx.tile}, batch {ctx.batch}")
    step()
    tile = ctx.tile
    ctx.tile = (16, 16)  # pair counts at 16x16 tiles (see the multi-view benchmark)
    ctx.render_fwd(g, cams, args.bg, out=outs, count_pairs=True)
    ctx.sync()
    evaluated, blended = ctx.pair_counts()
    walked = int(sum(int(o.n_contrib.sum().item()) for o in outs))
    ctx.tile = tile
    total_keys = count_tile_keys(ctx, g, cams)
    log(f"[bench] stress pairs evaluated {evaluated:.3e} blended {blended:.3e} walked {walked:.3e} keys {total_keys}")
    # eager, with stage timers
    for _ in range(args.warmup):
        step()
    ctx.sync()
    ctx.profile_begin(max_records=args.steps + 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    stages = ctx.profile_end()
    ctx.sync()
    eager_ms = e0.elapsed_time(e1) / args.steps
    per_stage = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    # HIP graph of one step, replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ctx.sync()
    graph_ms = e0.elapsed_time(e1) / args.steps
    log(f"[bench] stress eager {eager_ms:.2f} ms/step, graph {graph_ms:.2f} ms/step")
    bwd_flops = BWD_FLOPS_TEST * walked + BWD_FLOPS_BLEND * blended
    fwd_flops = FWD_FLOPS_TEST * evaluated + FWD_FLOPS_BLEND * blended
    line = {
        "metric": "large-footprint fwd+bwd iters/s @1M Gaussians x 4 views 1920x1080 (HIP graph)",
        "value": round(1000.0 / graph_ms, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(graph_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"stress_{N // 1000}k_sh3_4x1920x1080", "tile": tile_name(ctx.tile)},
        "autotune_ms": {autotune_name(t): v for t, v in tuned.items()} if tuned else None, "blend_batch": ctx.batch,
        "eager_ms_per_step": round(eager_ms, 3),
        "stage_ms_per_step": {k: round(v, 4) for k, v in per_stage.items()},
        "pairs": {"evaluated_fwd": evaluated, "blended": blended, "walked_bwd": walked},
        "tile_keys": total_keys,
        "blend_tflops": {"fwd": round(fwd_flops / (per_stage.get("blend_fwd", 0) or 1) * 1e-9, 3),
                         "bwd": round(bwd_flops / (per_stage.get("blend_bwd", 0) or 1) * 1e-9, 3)},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["multiview", "single", "streaming", "serving", "stress", "oracle"],
                    default="multiview")
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--views", type=int, default=20)
    ap.add_argument("--width", type=int, default=1352)
    ap.add_argument("--height", type=int, default=1014)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--densify-k", type=int, default=5000)
    ap.add_argument("--ssim-lambda", type=float, default=0.0,
                    help="weight of the D-SSIM term of the fidelity loss (Eq. 3); 0 = L1 only")
    ap.add_argument("--shift", choices=["direct", "hash"], default="direct",
                    help="shift offsets: per-Gaussian for the dynamic group (direct), or produced by the "
                         "H_dyn / H_st hash-encoded deformation fields over every base Gaussian (Sec. 3.3)")
    ap.add_argument("--lr-field", type=float, default=2e-3)
    ap.add_argument("--inherit-iters", type=int, default=0,
                    help="streaming: selective-inheritance iterations per timestep (s1 = 20 in the paper)")
    ap.add_argument("--max-keys", type=int, default=0)
    ap.add_argument("--lr-pos", type=float, default=1e-3)
    ap.add_argument("--lr-rot", type=float, default=1e-3)
    ap.add_argument("--render-reps", type=int, default=100)
    ap.add_argument("--feature-reps", type=int, default=5,
                    help="multiview: timed 16-channel identity-feature renders and dynamics masks (0 skips)")
    ap.add_argument("--per-view-steps", type=int, default=3)
    ap.add_argument("--graph-steps", type=int, default=20,
                    help="multiview: also time this many steps replayed from one captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters", type=int, default=100, help="iterations per timestep (streaming, serving)")
    ap.add_argument("--timesteps", type=int, default=40, help="timesteps (streaming)")
    ap.add_argument("--per-view-timesteps", type=int, default=10)
    ap.add_argument("--stream-views", type=int, choices=[1, 20], default=20)
    ap.add_argument("--stream-scene", choices=["rig", "multiview"], default="rig",
                    help="streaming: the 2k-Gaussian scene on a 128x128 rig, or the full multi-view scene "
                         "(--n Gaussians, --views cameras at --width x --height)")
    ap.add_argument("--requests", type=int, default=30000, help="requests (serving workload)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="multiview: requests of the serving leg run after the training steps (0: none)")
    ap.add_argument("--rate", type=float, default=500.0)
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--keys-per-tile", type=int, default=1200)
    ap.add_argument("--train-alone", type=int, default=2)
    ap.add_argument("--capacity-requests", type=int, default=500)
    ap.add_argument("--stress-n", type=int, default=1_000_000)
    ap.add_argument("--max-inflight", type=int, default=2,
                    help="training iterations queued at once while serving (0 = unbounded)")
    ap.add_argument("--no-autotune", action="store_true", help="stress: keep 16x16 tiles")
    ap.add_argument("--no-tile-autotune", action="store_true",
                    help="multiview/single: keep 16x16 tiles instead of the native autotuner's choice")
    ap.add_argument("--batch", type=int, default=0, choices=[0, 64, 128, 256],
                    help="blend LDS batch (0: autotuned with the tile size)")
    ap.add_argument("--tile", default="",
                    help="multiview/single: fixed tile size WxH (edges 16, 32 or 64; suffix s8 for 8x8 "
                         "sub-tiles) instead of autotuning")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    args.bg = (0.0, 0.0, 0.0)
    rank = int(os.environ.get("RANK", "0"))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        if rank == 0:
            print("bench.py measures one GPU only: the library has no multi-GPU path (views would shard "
                  "across GPUs with one gradient all-reduce per iteration).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "oracle":  # host only
        return bench_oracle_timings(args)
    import torch
    torch.cuda.set_device(0)
    if args.copy_probe:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "launches": 3}))
        return
    if args.workload == "streaming":
        return bench_streaming(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "stress":
        return bench_stress(args)
    log(f"[bench] building workload {args.workload}")
    s = build_workload(args)
    ctx = s["ctx"]
    train_step(s, 1, args)
    tuned = None
    if args.batch:
        ctx.batch = args.batch
    if args.tile:
        ctx.tile = parse_tile(args.tile)
    elif not args.no_tile_autotune:
        # native autotuner over tile sizes and blend batches on this workload (outside the timed
        # region)
        tuned = ctx.autotune_tile(s["gs"], s["cams"], args.bg, s["outs"], s["dls"], s["grads"], reps=5,
                                  batches=(args.batch,) if args.batch else BATCH_CANDIDATES)
        log(f"[bench] autotune (ms per fwd+bwd): {tuned}; using {ctx.tile}, batch {ctx.batch}")
    # pair counts of the blend (outside the timed region), always at 16x16 tiles: with larger
    # tiles n_contrib counts positions in a longer list whose extra entries are culled per
    # sub-tile, so only the 16x16 counts measure the work the definition asks for
    train_step(s, 1, args)
    tile = ctx.tile
    ctx.tile = (16, 16)
    ctx.render_fwd(s["gs"], s["cams"], args.bg, out=s["outs"], count_pairs=True)
    ctx.sync()
    evaluated, blended = ctx.pair_counts()
    walked = int(sum(int(o.n_contrib.sum().item()) for o in s["outs"]))
    ctx.tile = tile
    tile_keys = count_tile_keys(ctx, s["gs"], s["cams"])
    log(f"[bench] pairs evaluated {evaluated:.3e} blended {blended:.3e} walked-bwd {walked:.3e}; "
        f"{tile_keys} tile keys at {tile_name(ctx.tile)}")
    # timed steps with live stage timers
    log(f"[bench] warmup {args.warmup}, timing {args.steps} steps")
    for i in range(args.warmup):
        train_step(s, i + 2, args)
    ctx.profile_begin(max_records=args.steps + 1)
    ms, wall = time_steps(s, args, args.steps, 0)
    stages = ctx.profile_end()
    log(f"[bench] {ms:.2f} ms/step ({1000.0 / ms:.2f} iters/s), wall {wall:.2f}s")
    per_stage = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    # dominant kernel roofline
    fwd_flops = FWD_FLOPS_TEST * evaluated + FWD_FLOPS_BLEND * blended
    bwd_flops = BWD_FLOPS_TEST * walked + BWD_FLOPS_BLEND * blended
    cand = {"blend_bwd": bwd_flops, "blend_fwd": fwd_flops}
    dom = max(cand, key=lambda k: per_stage.get(k, 0.0))
    dom_ms = per_stage[dom]
    achieved = cand[dom] / (dom_ms * 1e-3) / 1e12
    kname = {"blend_bwd": "k_blend_bwd", "blend_fwd": "k_blend_fwd"}[dom]
    wl_key = f"multiview_{args.n // 1000}k_{args.views}x{args.width}x{args.height}"
    tile_s = tile_name(ctx.tile)
    traffic = measured_traffic(kname, wl_key, tile_s, ctx.batch) if args.workload == "multiview" else None
    roof = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_FLOPS / 1e12,
            "unit": "TFLOP/s", "frac": round(achieved * 1e12 / PEAK_FP32_FLOPS, 4), "traffic": traffic,
            "flops_per_launch": float(cand[dom]), "avg_launch_ms": round(dom_ms, 4)}
    graph_ms = None
    if args.workload == "multiview" and args.shift == "direct" and args.graph_steps > 0:
        graph_ms = time_graph_steps(s, args, args.graph_steps, 2, args.warmup + args.steps + 2)
        log(f"[bench] graph-replayed step {graph_ms:.3f} ms ({1000.0 / graph_ms:.2f} iters/s)")
    p50, p99 = render_latency(s, args, args.render_reps)
    log(f"[bench] render p50 {p50:.3f} ms p99 {p99:.3f} ms")
    feats = feature_render_times(s, args) if args.workload == "multiview" and args.feature_reps > 0 else None
    serving = None
    if args.workload == "multiview" and args.serving_requests > 0:
        serving = serving_leg(args, args.serving_requests)
    lat = None
    if args.workload == "single":
        e_ms, g_ms = fwdbwd_latency(s, args, 200)
        lat = {"eager_us": round(e_ms * 1e3, 2), "graph_us": round(g_ms * 1e3, 2)}
        log(f"[bench] fwd+bwd latency eager {e_ms * 1e3:.1f} us, graph replay {g_ms * 1e3:.1f} us")
    pv_ms = None
    if args.per_view_steps > 0:
        pv_ms, _ = time_steps(s, args, args.per_view_steps, 1, per_view=True)
        log(f"[bench] per-view loop {pv_ms:.2f} ms/step")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(s, args)
        log(f"[bench] cpu baseline {cpu['value']:.3e} iters/s on {cpu['cores']} threads "
            f"({cpu['single_thread']['value']:.3e} on one), {cpu['cpu']}")
    cams = s["cams"]
    line = {
        "metric": ("fwd+bwd iters/s @200k Gaussians x 20 views 1352x1014; render p50/p99 ms"
                   if args.workload == "multiview" else
                   "fwd+bwd iters/s @2k Gaussians x 1 view 128x128 (single-view scene); fwd+bwd latency us"),
        "value": round(1000.0 / ms, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": s["name"], "n_gaussians": s["N"], "sh_degree": int(s["g"].sh_degree),
                   "views": len(cams), "width": cams[0].width, "height": cams[0].height,
                   "tile": tile_name(ctx.tile), "blend_batch": ctx.batch,
                   "n_dynamic": s["nd"], "densify_k": args.densify_k,
                   "loss": "l1" if args.ssim_lambda == 0.0 else f"(1-l) L1 + l D-SSIM, l = {args.ssim_lambda}",
                   "shift": ("direct offsets of the dynamic group" if args.shift == "direct" else
                             "H_dyn (T 2^16, F 4) / H_st (T 2^14, F 2) hash fields, 16 levels, 64 hidden"),
                   "parallelism": "single GPU"},
        "tile_autotune_ms": ({autotune_name(t): v for t, v in tuned.items()} if tuned else None),
        "graph_replay": ({"ms_per_step": round(graph_ms, 3), "iters_per_s": round(1000.0 / graph_ms, 3),
                          "steps": args.graph_steps} if graph_ms else None),
        "render_p50_ms": round(p50, 4), "render_p99_ms": round(p99, 4),
        "serving": serving,
        "identity_features": feats,
        "fwd_bwd_latency": lat,
        "per_view_loop_iters_per_s": round(1000.0 / pv_ms, 3) if pv_ms else None,
        "stage_ms_per_step": {k: round(v, 4) for k, v in per_stage.items()},
        "pairs": {"evaluated_fwd": evaluated, "blended": blended, "walked_bwd": walked},
        "tile_keys": tile_keys,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

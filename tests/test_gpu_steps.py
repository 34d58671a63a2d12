"""GPU parity of the steps around the rasterizer: shift (forward / adjoint), Adam, L1 gradient and
error map, densification, one composed training iteration; plus the autograd wrapper and the
streaming driver."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_grad_close, excluded_pixels, log, make_ctx, to_gpu

pytestmark = pytest.mark.gpu
BG = (0.1, 0.05, 0.0)


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


@pytest.mark.parametrize("n_dyn", [0, 1, 200, 2000])
def test_shift_forward_and_adjoint(n_dyn):
    scene, cams, _ = synth.single_view_scene(1)
    rng = np.random.default_rng(n_dyn)
    dyn = np.sort(rng.choice(scene.n, n_dyn, replace=False)).astype(np.int32)
    if n_dyn == 1:
        dyn[0] = scene.n - 1  # last row
    dpos = rng.normal(0, 0.01, (3, n_dyn)).astype(np.float32)
    drot = rng.normal(size=(4, n_dyn)).astype(np.float32)
    g = to_gpu(scene)
    out = g.zeros_like()
    ctx = make_ctx(scene.n, cams)
    ctx.shift_fwd(g, out, dev(dyn), dev(dpos), dev(drot))
    om, oq = oracle.shift_fwd(scene, dyn, dpos, drot)
    np.testing.assert_allclose(out.mean.cpu().numpy(), om, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(out.quat.cpu().numpy(), oq, rtol=1e-6, atol=1e-7)
    dmean = rng.normal(size=(3, scene.n)).astype(np.float32)
    dquat = rng.normal(size=(4, scene.n)).astype(np.float32)
    d_out = g.zeros_like()
    d_out.mean.copy_(dev(dmean))
    d_out.quat.copy_(dev(dquat))
    d_dpos = torch.zeros(3, max(n_dyn, 1), device="cuda")[:, :n_dyn].contiguous()
    d_drot = torch.zeros(4, max(n_dyn, 1), device="cuda")[:, :n_dyn].contiguous()
    ctx.shift_adjoint(g, dev(dyn), dev(drot), d_out, d_dpos, d_drot)
    ctx.sync()
    ddp, ddr = oracle.shift_adj(scene, dyn, drot, dmean, dquat)
    np.testing.assert_allclose(d_dpos.cpu().numpy(), ddp, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(d_drot.cpu().numpy(), ddr, rtol=1e-5, atol=1e-6)


def test_adam_matches_oracle_host_and_device_step():
    rng = np.random.default_rng(4)
    sizes = [1, 1023, 1024, 5000, 0, 77]
    lrs = [1e-3, 5e-2, 1e-4, 2e-3, 1e-3, 3e-1]
    scene, cams, _ = synth.single_view_scene(0, n=10)
    ctx = make_ctx(10, cams)
    P = [dev(rng.normal(size=n).astype(np.float32)) for n in sizes]
    P2 = [p.clone() for p in P]
    M = [torch.zeros_like(p) for p in P]; V = [torch.zeros_like(p) for p in P]
    M2 = [torch.zeros_like(p) for p in P]; V2 = [torch.zeros_like(p) for p in P]
    ref = [(p.cpu().numpy().astype(np.float64), np.zeros(p.numel()), np.zeros(p.numel())) for p in P]
    d_step = torch.zeros(1, dtype=torch.int32, device="cuda")
    # fp32 rounding bound of the first-moment recurrence, whose terms have mixed signs: each step
    # rounds within 2^-24 of the running sum of |terms| (m_abs), so |m - m_exact| <= c 2^-24 m_abs
    m_abs = [np.zeros(n) for n in sizes]
    for step in range(1, 6):
        G = [dev((rng.normal(size=n) * 10 ** rng.uniform(-4, 1)).astype(np.float32)) for n in sizes]
        m_abs = [0.9 * ma + 0.1 * np.abs(g_.cpu().numpy().astype(np.float64)) for ma, g_ in zip(m_abs, G)]
        ctx.adam_step([(p, g_, m, v, lr) for p, g_, m, v, lr in zip(P, G, M, V, lrs)], 0.9, 0.999, 1e-15, step)
        ctx.adam_step([(p, g_, m, v, lr) for p, g_, m, v, lr in zip(P2, G, M2, V2, lrs)], 0.9, 0.999, 1e-15,
                      d_step=d_step)
        # the entry point takes float32 hyper-parameters; the oracle gets the same values
        f32 = lambda x: float(np.float32(x))
        ref = [oracle.adam(r[0], g_.cpu().numpy(), r[1], r[2], f32(lr), f32(0.9), f32(0.999), f32(1e-15), step)
               for r, g_, lr in zip(ref, G, lrs)]
    ctx.sync()
    assert int(d_step.item()) == 5
    for p, p2, m, v, r, ma in zip(P, P2, M, V, ref, m_abs):
        if p.numel() == 0:
            continue
        np.testing.assert_allclose(p.cpu().numpy(), r[0], rtol=1e-5, atol=1e-6)
        err_m = np.abs(m.cpu().numpy().astype(np.float64) - r[1])
        assert np.all(err_m <= 1e-5 * np.abs(r[1]) + 16 * 2.0 ** -24 * ma), float(np.max(err_m))
        np.testing.assert_allclose(v.cpu().numpy(), r[2], rtol=1e-5, atol=1e-20)
        np.testing.assert_allclose(p2.cpu().numpy(), p.cpu().numpy(), rtol=1e-6, atol=1e-7)


def test_l1_loss_gradient_and_error_maps():
    rng = np.random.default_rng(2)
    cams = [synth.make_camera(np.eye(3), (0, 0, 0), w, h) for w, h in ((64, 48), (37, 29), (128, 128))]
    R = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    T = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    T[0][:, 0, 0] = R[0][:, 0, 0]  # zero difference -> zero gradient
    ctx = make_ctx(10, cams)
    dl = [torch.zeros(3, c.height, c.width, device="cuda") for c in cams]
    err = [torch.zeros(c.height, c.width, device="cuda") for c in cams]
    loss = torch.zeros(1, device="cuda")
    ctx.l1_loss_grad(cams, [dev(r) for r in R], [dev(t) for t in T], dl, err, loss)
    ctx.sync()
    V = len(cams)
    want_loss = 0.0
    for v in range(V):
        l, d, e = oracle.l1_loss_grad(R[v][None], T[v][None])
        want_loss += l / V
        np.testing.assert_allclose(dl[v].cpu().numpy(), d[0] / V, rtol=1e-6)
        np.testing.assert_allclose(err[v].cpu().numpy(), e[0], rtol=1e-6, atol=1e-7)
    assert float(loss.item()) == pytest.approx(want_loss, rel=1e-5)


@pytest.mark.parametrize("tile", [(16, 16), (32, 32), (16, 16, 8)])
def test_fused_forward_l1_matches_render_then_l1(tile):
    """render_fwd_l1 against render_fwd followed by l1_loss_grad (which the oracle pins above):
    images, dL/drgb and error maps bit-identical, loss equal up to float summation order; with
    keep_rgb False the image buffers are left untouched."""
    from test_gpu_parity import small_multiview
    scene, cams, _ = small_multiview(seed=11, n=2500, views=3, W=150, H=110)
    rng = np.random.default_rng(12)
    targets = [dev(rng.uniform(size=(3, c.height, c.width)).astype(np.float32)) for c in cams]
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    ctx.tile = tile
    out = ctx.render_fwd(g, cams, BG)
    dl = [torch.zeros(3, c.height, c.width, device="cuda") for c in cams]
    err = [torch.zeros(c.height, c.width, device="cuda") for c in cams]
    loss = torch.zeros(1, device="cuda")
    ctx.l1_loss_grad(cams, [o.rgb for o in out], targets, dl, err, loss)
    for keep in (True, False):
        out2 = [type(o).allocate(c) for o, c in zip(out, cams)]
        for o in out2:
            o.rgb.fill_(-7.0)
        dl2 = [torch.full_like(d, 5.0) for d in dl]
        err2 = [torch.full_like(e, 5.0) for e in err]
        loss2 = torch.full((1,), 0.25, device="cuda")
        ctx.render_fwd_l1(g, cams, BG, targets, dl2, err2, loss2, out=out2, keep_rgb=keep)
        ctx.sync()
        for v in range(len(cams)):
            if keep:
                assert torch.equal(out2[v].rgb, out[v].rgb)
            else:
                assert bool((out2[v].rgb == -7.0).all())
            assert torch.equal(out2[v].t_final, out[v].t_final)
            assert torch.equal(out2[v].n_contrib, out[v].n_contrib)
            assert torch.equal(dl2[v], dl[v])
            assert torch.equal(err2[v], err[v])
        assert float(loss2.item()) - 0.25 == pytest.approx(float(loss.item()), rel=1e-5)
    # the fused forward also feeds render_bwd like render_fwd does
    grads_a, grads_b = g.zeros_like(), g.zeros_like()
    ctx.render_fwd(g, cams, BG, out=out)
    ctx.render_bwd(g, cams, BG, out, dl, grads_a)
    ctx.render_fwd_l1(g, cams, BG, targets, dl2, None, None, out=out2, keep_rgb=False)
    ctx.render_bwd(g, cams, BG, out2, dl2, grads_b)
    ctx.sync()
    for a, b in zip(grads_a.planes(), grads_b.planes()):
        torch.testing.assert_close(a, b, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_fidelity_loss_with_dssim_matches_oracle(lam):
    """Eq. (3) fidelity term with D-SSIM against the oracle: several views of ragged sizes
    (tiles of 16 with a remainder, images smaller than the window), renders and targets of
    random and smooth content (small local variance, where SSIM's moments cancel most)."""
    rng = np.random.default_rng(31)
    sizes = ((64, 48), (37, 29), (150, 110), (9, 7))
    cams = [synth.make_camera(np.eye(3), (0, 0, 0), w, h) for w, h in sizes]
    R, T = [], []
    for k, c in enumerate(cams):
        if k % 2 == 0:
            r = rng.uniform(size=(3, c.height, c.width))
            t = np.clip(r + rng.normal(0, 0.1, size=r.shape), 0, 1)
        else:
            yy, xx = np.mgrid[0:c.height, 0:c.width]
            r = 0.5 + 0.4 * np.sin(xx / 7.0 + np.arange(3)[:, None, None]) * np.cos(yy / 5.0)
            t = r + 0.02 * rng.normal(size=r.shape)
        R.append(r.astype(np.float32))
        T.append(t.astype(np.float32))
    ctx = make_ctx(10, cams)
    dl = [torch.full((3, c.height, c.width), 7.0, device="cuda") for c in cams]
    err = [torch.zeros(c.height, c.width, device="cuda") for c in cams]
    loss = torch.full((1,), 0.5, device="cuda")
    ctx.fidelity_loss_grad(cams, [dev(r) for r in R], [dev(t) for t in T], lam, dl, err, loss)
    ctx.sync()
    want = [oracle.fidelity_loss_grad(R[v][None], T[v][None], lam) for v in range(len(cams))]
    V = len(cams)
    want_loss = sum(w[0] for w in want) / V
    assert float(loss.item()) - 0.5 == pytest.approx(want_loss, rel=1e-5)
    for v in range(V):
        got = dl[v].cpu().numpy()
        o = want[v][1][0] / V
        # per-tensor bound of the gradient tests: |g - o| <= 1e-3 |o| + 1e-4 max|o|
        bad = np.abs(got - o) > 1e-3 * np.abs(o) + 1e-4 * np.abs(o).max()
        assert not bad.any(), (v, np.abs(got - o).max(), np.abs(o).max())
        np.testing.assert_allclose(err[v].cpu().numpy(), want[v][2][0], rtol=1e-6, atol=1e-7)
    # lambda = 0 is the L1 call, bit for bit
    dl0 = [torch.zeros_like(d) for d in dl]
    dl1 = [torch.zeros_like(d) for d in dl]
    ctx.fidelity_loss_grad(cams, [dev(r) for r in R], [dev(t) for t in T], 0.0, dl0)
    ctx.l1_loss_grad(cams, [dev(r) for r in R], [dev(t) for t in T], dl1)
    ctx.sync()
    for a, b in zip(dl0, dl1):
        assert torch.equal(a, b)


def test_fidelity_loss_with_dssim_fullsize():
    """Two views at the benchmark's 1352x1014, lambda 0.2: every element against the oracle."""
    rng = np.random.default_rng(32)
    cams = [synth.make_camera(np.eye(3), (0, 0, 0), 1352, 1014) for _ in range(2)]
    R = [rng.uniform(size=(3, 1014, 1352)).astype(np.float32) for _ in cams]
    T = [np.clip(r + rng.normal(0, 0.05, size=r.shape), 0, 1).astype(np.float32) for r in R]
    ctx = make_ctx(10, cams)
    dl = [torch.zeros(3, 1014, 1352, device="cuda") for _ in cams]
    err = [torch.zeros(1014, 1352, device="cuda") for _ in cams]
    loss = torch.zeros(1, device="cuda")
    ctx.fidelity_loss_grad(cams, [dev(r) for r in R], [dev(t) for t in T], 0.2, dl, err, loss)
    ctx.sync()
    total = 0.0
    for v in range(2):
        lv, dv, ev = oracle.fidelity_loss_grad(R[v][None], T[v][None], 0.2)
        total += lv / 2
        o = dv[0] / 2
        got = dl[v].cpu().numpy()
        assert not (np.abs(got - o) > 1e-3 * np.abs(o) + 1e-4 * np.abs(o).max()).any()
        np.testing.assert_allclose(err[v].cpu().numpy(), ev[0], rtol=1e-6, atol=1e-7)
    assert float(loss.item()) == pytest.approx(total, rel=1e-5)


def _densify_case(seed, n, views, k_max, extra_cap, tau_pos, tau_err, gamma):
    rng = np.random.default_rng(seed)
    scene, cams, _ = synth.multiview_scene(seed, n=n, n_views=views, width=96, height=72, with_grads=False)
    errs = [rng.uniform(0, 1, size=(c.height, c.width)).astype(np.float32) for c in cams]
    gsum = rng.exponential(1.0, size=n).astype(np.float32)
    cnt = rng.integers(0, 4, size=n).astype(np.int32)
    return scene, cams, errs, gsum, cnt, k_max, n + extra_cap, tau_pos, tau_err, gamma


@pytest.mark.parametrize("case", [
    (1, 800, 4, 5000, 6000, 0.0, 0.0, 0.0),     # |S| < K: children cycle over the ranked parents
    (2, 800, 3, 100, 6000, 1.0, 0.3, 0.5),      # |S| > K: capped at K
    (3, 500, 2, 300, 120, 0.0, 0.0, 0.0),       # capped by capacity
    (4, 300, 2, 50, 100, 1e9, 1e9, 0.5),        # empty S
])
def test_densify_append_matches_oracle(case):
    scene, cams, errs, gsum, cnt, k_max, cap, tp, te, gamma = _densify_case(*case)
    n = scene.n
    seed = 1234 + case[0]
    sel, score, _ = oracle.densify_select(scene.mean, cams, errs, gsum, cnt, gamma, tp, te)
    planes = {k: np.zeros(getattr(scene, k).shape[:-1] + (cap,), np.float32)
              for k in ("mean", "quat", "log_scale", "logit", "sh")}
    for k in planes:
        planes[k][..., :n] = getattr(scene, k)
    n_app, child_mean = oracle.spawn(planes, n, cap, sel, k_max, seed)
    g = to_gpu(scene, capacity=cap)
    ctx = make_ctx(cap, cams)
    n_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.densify_append(g, [dev(e) for e in errs], cams, dev(gsum), dev(cnt), gamma, tp, te, k_max, seed, n_dev)
    ctx.sync()
    log(f"  |S|={sel.size} appended={n_app}")
    assert int(n_dev.item()) == n_app
    if n_app == 0:
        return
    rows = slice(n, n + n_app)
    for k in ("quat", "logit", "sh"):  # copied bit-exactly from the parent
        np.testing.assert_array_equal(getattr(g, k)[..., rows].cpu().numpy(), planes[k][..., rows])
    np.testing.assert_allclose(g.log_scale[:, rows].cpu().numpy(), planes["log_scale"][:, rows], rtol=0, atol=1e-6)
    np.testing.assert_allclose(g.mean[:, rows].cpu().numpy(), child_mean, rtol=1e-6, atol=1e-6)
    # base rows untouched
    np.testing.assert_array_equal(g.mean[:, :n].cpu().numpy(), scene.mean)


def test_one_training_iteration_matches_oracle():
    """shift -> render -> L1 -> render_bwd -> shift adjoint, composed, against the oracle."""
    scene, cams, _ = synth.multiview_scene(11, n=1500, n_views=3, width=96, height=80)
    n = scene.n
    motion = synth.timestep_motion(11, 1, n)
    rng = np.random.default_rng(3)
    dpos = rng.normal(0, 0.01, (3, motion.dynamic.size)).astype(np.float32)
    drot = np.concatenate([np.ones((1, motion.dynamic.size)), rng.normal(0, 0.05, (3, motion.dynamic.size))]
                          ).astype(np.float32)
    targets = [np.full((3, c.height, c.width), 5.0, np.float32) for c in cams]  # render < target everywhere
    # oracle
    om, oq = oracle.shift_fwd(scene, motion.dynamic, dpos, drot)
    shifted = synth.Scene(om.astype(np.float32), oq.astype(np.float32), scene.log_scale, scene.logit, scene.sh,
                          scene.sh_degree)
    renders = [oracle.render_view(shifted, c, bg=BG) for c in cams]
    _, dl, _ = oracle.l1_loss_grad(np.stack([r.rgb for r in renders]).astype(np.float32), np.stack(targets))
    dls = [dl[v].astype(np.float32) for v in range(len(cams))]
    masks = [excluded_pixels(vr, c, grad=True) for vr, c in zip(renders, cams)]
    for d, m in zip(dls, masks):
        d[:, m] = 0.0
    og, _, _, _ = oracle.render_backward(shifted, cams, dls, bg=BG, renders=renders)
    ddp, ddr = oracle.shift_adj(scene, motion.dynamic, drot, og.mean, og.quat)
    # GPU
    g = to_gpu(scene)
    gs = g.zeros_like()
    gs.log_scale, gs.logit, gs.sh = g.log_scale, g.logit, g.sh
    ctx = make_ctx(n, cams)
    dyn = dev(motion.dynamic)
    ctx.shift_fwd(g, gs, dyn, dev(dpos), dev(drot))
    outs = ctx.render_fwd(gs, cams, BG)
    dlg = [torch.zeros(3, c.height, c.width, device="cuda") for c in cams]
    loss = torch.zeros(1, device="cuda")
    ctx.l1_loss_grad(cams, [o.rgb for o in outs], [dev(t) for t in targets], dlg, None, loss)
    for d, m, want in zip(dlg, masks, dls):
        d[:, dev(m)] = 0.0  # the oracle's decision-margin pixels
        np.testing.assert_allclose(d.cpu().numpy(), want, rtol=1e-6)
    grads = g.zeros_like()
    ctx.render_bwd(gs, cams, BG, outs, dlg, grads)
    d_dpos = torch.zeros(3, motion.dynamic.size, device="cuda")
    d_drot = torch.zeros(4, motion.dynamic.size, device="cuda")
    ctx.shift_adjoint(g, dyn, dev(drot), grads, d_dpos, d_drot)
    ctx.sync()
    assert_grad_close("d_dpos", d_dpos.cpu().numpy(), ddp)
    assert_grad_close("d_drot", d_drot.cpu().numpy(), ddr)
    assert_grad_close("sh", grads.sh[:, :n].cpu().numpy(), og.sh)


def test_autograd_function_matches_render_bwd():
    from paper_2411_14847_amd.autograd import rasterize
    scene, cams, dls = synth.multiview_scene(5, n=1200, n_views=2, width=80, height=64)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    params = [t[..., :scene.n].clone().requires_grad_(True) for t in g.planes()]
    imgs = rasterize(*params, ctx, cams, BG, scene.sh_degree)
    loss = sum((img * dev(d)).sum() for img, d in zip(imgs, dls))
    loss.backward()
    outs = ctx.render_fwd(g, cams, BG)
    grads = g.zeros_like()
    ctx.render_bwd(g, cams, BG, outs, [dev(d) for d in dls], grads)
    ctx.sync()
    for p, ref in zip(params, grads.planes()):
        torch.testing.assert_close(p.grad, ref[..., :scene.n], rtol=1e-4, atol=1e-5)
    for img, o in zip(imgs, outs):
        assert torch.equal(img.detach(), o.rgb)


def test_autograd_function_matches_oracle():
    """The autograd path against the float64 oracle: images within the image tolerance, and the
    parameter gradients of L = sum_v <dl_v, image_v> (upstream zeroed where a decision sits within
    rounding of its threshold) within the gradient tolerance."""
    from paper_2411_14847_amd.autograd import rasterize
    from gpu_util import IMG_TOL, assert_grad_close, excluded_pixels
    scene, cams, dls = synth.multiview_scene(6, n=1500, n_views=2, width=96, height=72)
    log("[autograd vs oracle]")
    renders = [oracle.render_view(scene, c, bg=BG) for c in cams]
    dls = [d.copy() for d in dls]
    for d, vr, cam in zip(dls, renders, cams):
        d[:, excluded_pixels(vr, cam, grad=True)] = 0.0
    og, _, _, _ = oracle.render_backward(scene, cams, dls, bg=BG, renders=renders)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    params = [t[..., :scene.n].clone().requires_grad_(True) for t in g.planes()]
    imgs = rasterize(*params, ctx, cams, BG, scene.sh_degree)
    loss = sum((img * dev(d)).sum() for img, d in zip(imgs, dls))
    loss.backward()
    ctx.sync()
    for img, vr, cam in zip(imgs, renders, cams):
        ex = excluded_pixels(vr, cam)
        err = np.abs(img.detach().cpu().numpy() - vr.rgb)[:, ~ex]
        assert err.max() <= IMG_TOL, err.max()
    gflag = np.zeros(scene.n, bool)
    for cam in cams:
        gflag |= (oracle.project(scene, cam).flags & oracle.GAUSS_GRAD_FLAGS) != 0
    for name, p in zip(("mean", "quat", "log_scale", "logit", "sh"), params):
        rel = assert_grad_close(name, p.grad.cpu().numpy(), getattr(og, name), exclude=gflag)
        log(f"  {name}: max rel err (significant) {rel:.2e}")


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("lam", [0.0, 0.2], ids=["l1", "l1_dssim"])
def test_streaming_driver(use_graph, lam):
    from paper_2411_14847_amd import Context, GaussianBuffers
    from paper_2411_14847_amd.streaming import StreamConfig, Trainer
    scene, _, _ = synth.single_view_scene(0, n=600)
    cams = synth.streaming_rig(64, 64)[:4]
    cfg = StreamConfig(iters=25, k_append=80, erase_every=2, use_graph=use_graph, ssim_lambda=lam)
    cap = scene.n + 2 * cfg.k_append
    g = GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh, 0, capacity=cap)
    gt = g.clone()
    ctx = Context(max_gaussians=cap, max_views=len(cams), max_keys=cap * len(cams) * 32, max_tiles=4 * 16)
    tr = Trainer(ctx, g, cams, max_dynamic=scene.n // 10, cfg=cfg)
    gt_ctx = Context(max_gaussians=cap, max_views=len(cams), max_keys=cap * len(cams) * 32, max_tiles=4 * 16)
    ns = []
    for t in range(1, 4):
        m = synth.timestep_motion(0, t, scene.n)
        gt_out = gt.zeros_like()
        gt_ctx.shift_fwd(gt, gt_out, dev(m.dynamic), dev(m.dpos), dev(m.dquat))
        gt.mean.copy_(gt_out.mean); gt.quat.copy_(gt_out.quat)
        targets = [o.rgb.clone() for o in gt_ctx.render_fwd(gt, cams, cfg.bg)]
        st = tr.timestep(t, dev(m.dynamic), targets)
        log(f"  t={t} loss {st['loss_first']:.5f} -> {st['loss_last']:.5f}, appended {st['appended']}, n {st['n']}")
        assert st["loss_last"] < st["loss_first"]
        ns.append(st["n"])
    ctx.sync()
    # erase every 2 timesteps: t=2 erases G^var before its append
    assert ns[0] == scene.n + 80 and ns[1] == scene.n + 80 and ns[2] == scene.n + 160


def test_graph_replay_matches_eager():
    """One captured training iteration replayed three times, with eager work and synchronisation
    between replays; every replay is checked against an eager run from the same state."""
    from paper_2411_14847_amd import Context, GaussianBuffers
    from paper_2411_14847_amd.streaming import StreamConfig, Trainer
    scene, _, _ = synth.single_view_scene(2, n=500)
    cams = synth.streaming_rig(48, 48)[:3]
    cfg = StreamConfig(iters=1, k_append=10)
    g = GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh, 0,
                                    capacity=scene.n + 16)
    ctx = Context(max_gaussians=g.capacity, max_views=3, max_keys=g.capacity * 3 * 32, max_tiles=3 * 9)
    tr = Trainer(ctx, g, cams, max_dynamic=60, cfg=cfg)
    m = synth.timestep_motion(2, 1, scene.n)
    tr.begin_timestep(1, dev(m.dynamic[:60]))
    tr.set_targets([torch.full((3, 48, 48), 0.3, device="cuda") for _ in cams])

    def snapshot():
        return [t.clone() for t in (tr._dpos, tr._drot, tr._m_dpos, tr._v_dpos, tr._m_drot, tr._v_drot, tr.d_step)]

    def restore(snap):
        for dst, src in zip((tr._dpos, tr._drot, tr._m_dpos, tr._v_dpos, tr._m_drot, tr._v_drot, tr.d_step), snap):
            dst.copy_(src)

    s0 = snapshot()
    tr.iteration()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (tr._dpos, tr._drot, tr.loss)]
    restore(s0)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        tr.iteration(stream=side)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    restore(s0)
    with torch.cuda.graph(graph):
        tr.iteration(stream=torch.cuda.current_stream())
    for rep in range(3):
        restore(s0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (tr._dpos, tr._drot, tr.loss)
        for a, b in zip(got, eager):
            torch.testing.assert_close(a, b, rtol=1e-5, atol=1e-7)
        # eager work between replays
        ctx.render_fwd(g, cams, cfg.bg)
        ctx.sync()


def _small_requests(n, seed=0, sizes=((160, 120), (320, 180), (240, 136))):
    reqs = synth.serving_requests(seed, n_requests=n, rate_hz=2000.0, n_viewers=8)
    rng = np.random.default_rng(seed)
    out = []
    for r in reqs:
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        cam = synth.make_camera(r.camera.R.astype(np.float64), r.camera.campos.astype(np.float64), W, H)
        out.append((r.arrival_s, cam))
    return out


def test_serving_batches_match_alone_renders():
    from paper_2411_14847_amd import GaussianBuffers
    from paper_2411_14847_amd.serving import RenderServer, Request, SceneSnapshots
    scene, _, _ = synth.multiview_scene(3, n=20_000, n_views=1, with_grads=False)
    g = GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh, 3)
    snaps = SceneSnapshots(g)
    snaps.publish(g)
    server = RenderServer(snaps, max_gaussians=g.capacity, n_slots=2, max_batch=6, max_tiles=6 * 240,
                          keys_per_tile=2000, max_w=320, max_h=180)
    reqs = [Request(i, a, c) for i, (a, c) in enumerate(_small_requests(6, seed=1))]
    slot = server.slots[1]
    server.launch(slot, reqs)
    slot.stream.synchronize()
    slot.ctx.sync(slot.stream)
    batched = [server._view(o, r.camera).rgb.clone() for o, r in zip(slot.outs, reqs)]
    assert len({(r.camera.width, r.camera.height) for r in reqs}) > 1  # mixed resolutions
    for r, img in zip(reqs, batched):
        alone = server.render_alone(r.camera)
        assert torch.equal(alone.rgb, img)


def test_serving_loop_with_concurrent_training():
    import threading
    from paper_2411_14847_amd import Context, GaussianBuffers
    from paper_2411_14847_amd.serving import RenderServer, Request, SceneSnapshots, serve_requests
    from paper_2411_14847_amd.streaming import StreamConfig, Trainer
    scene, cams, _ = synth.multiview_scene(4, n=20_000, n_views=4, width=160, height=120, with_grads=False)
    cfg = StreamConfig(iters=10, k_append=200)
    cap = scene.n + 400
    g = GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh, 3, capacity=cap)
    snaps = SceneSnapshots(g)
    snaps.publish(g)
    ctx = Context(max_gaussians=cap, max_views=4, max_keys=cap * 4 * 40, max_tiles=4 * 80)
    tr = Trainer(ctx, g, cams, max_dynamic=2000, cfg=cfg)
    targets = [torch.full((3, 120, 160), 0.2, device="cuda") for _ in cams]
    train_stream = torch.cuda.Stream()
    done = []

    def train():
        with torch.cuda.stream(train_stream):
            for t in range(1, 3):
                m = synth.timestep_motion(4, t, scene.n)
                done.append(tr.timestep(t, dev(m.dynamic), targets))
                snaps.publish(g, train_stream)

    th = threading.Thread(target=train)
    th.start()
    server = RenderServer(snaps, max_gaussians=cap, n_slots=3, max_batch=4, max_tiles=4 * 240, keys_per_tile=2000,
                          max_w=320, max_h=180)
    reqs = [Request(i, a, c) for i, (a, c) in enumerate(_small_requests(80, seed=2))]
    st = serve_requests(server, reqs)
    th.join()
    torch.cuda.synchronize()
    log(f"  serving {st}; training {[round(d['ms'], 1) for d in done]} ms/timestep")
    assert st["frames"] == 80 and st["p99_ms"] is not None and st["p50_ms"] <= st["p99_ms"]
    assert len(done) == 2 and snaps.version == 3


@pytest.mark.parametrize("shift", ["direct", "hash"])
def test_bake_applies_the_final_offsets(shift):
    """After k iterations of a timestep, the baked scene equals the shift (Sec. 3.3) of the final
    parameters by the final offsets -- for the hash fields, the offsets the final fields give --
    on every row, G^var included (their means and quaternions keep the last Adam step)."""
    import types
    from oracle import hashfield as HF
    from paper_2411_14847_amd import Context, GaussianBuffers
    from paper_2411_14847_amd.streaming import StreamConfig, Trainer
    scene, _, _ = synth.single_view_scene(0, n=600)
    cams = synth.streaming_rig(64, 64)[:4]
    cfg = StreamConfig(iters=6, k_append=80, erase_every=100, prune_min_opacity=0.0, shift=shift,
                       field_dyn=(8, 4, 12, 64, 4, 64), field_st=(8, 2, 10, 32, 4, 32))
    cap = scene.n + 2 * cfg.k_append
    g = GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh, 0, capacity=cap)
    gt = g.clone()
    ctx = Context(max_gaussians=cap, max_views=len(cams), max_keys=cap * len(cams) * 32, max_tiles=4 * 16)
    tr = Trainer(ctx, g, cams, max_dynamic=scene.n // 10, cfg=cfg)
    for t in (1, 2):
        m = synth.timestep_motion(0, t, scene.n)
        gt_out = gt.zeros_like()
        ctx.shift_fwd(gt, gt_out, dev(m.dynamic), dev(m.dpos), dev(m.dquat))
        gt.mean.copy_(gt_out.mean); gt.quat.copy_(gt_out.quat)
        targets = [o.rgb.clone() for o in ctx.render_fwd(gt, cams, cfg.bg)]
        if t == 1:
            tr.timestep(t, dev(m.dynamic), targets)  # leaves 80 G^var rows
            continue
        log(f"[bake] {shift}: timestep 2, n {g.n} (n_base {g.n_base})")
        tr.set_targets(targets)
        tr.begin_timestep(t, dev(m.dynamic))
        tr.iteration()
        tr.run_iterations(cfg.iters - 1)
        torch.cuda.synchronize()
        n = g.n
        assert n > g.n_base
        fin = synth.Scene(g.mean[:, :n].cpu().numpy(), g.quat[:, :n].cpu().numpy(), g.log_scale[:, :n].cpu().numpy(),
                          g.logit[:n].cpu().numpy(), g.sh[:, :n].cpu().numpy(), 0)
        rows = tr._shift_idx.cpu().numpy()
        if shift == "direct":
            dpos, drot = tr._dpos.cpu().numpy(), tr._drot.cpu().numpy()
        else:
            parts = []
            for k, idx in (("dyn", tr._dyn), ("st", tr._st)):
                f = tr.fields[k]
                p = types.SimpleNamespace(res=f.res, features=f.features, log2_table=f.log2_table,
                                          aabb_min=np.array(f.aabb_min), aabb_max=np.array(f.aabb_max),
                                          **{a: t_.cpu().numpy() for a, t_ in zip(("table", "w1", "b1", "w2", "b2"),
                                                                                  f.arrays())})
                parts.append(HF.field_fwd(HF.from_params(p), fin.mean[:, idx.cpu().numpy()].astype(np.float64)))
            dpos = np.concatenate([parts[0][0], parts[1][0]], 1)
            drot = np.concatenate([parts[0][1], parts[1][1]], 1)
        om, oq = oracle.shift_fwd(fin, rows, dpos, drot)
        tr.end_timestep(t)
        torch.cuda.synchronize()
        np.testing.assert_allclose(g.mean[:, :n].cpu().numpy(), om, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(g.quat[:, :n].cpu().numpy(), oq, rtol=1e-5, atol=1e-6)
        # G^var rows were not shifted: they hold exactly their final parameters
        np.testing.assert_array_equal(g.mean[:, g.n_base:n].cpu().numpy(), fin.mean[:, g.n_base:])

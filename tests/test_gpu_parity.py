"""Parity of the HIP path (through the C ABI) with the CPU oracle, on seeded synthetic inputs.

Bar: tile keys, values, ranges and n_contrib bit-exact; images within 1e-4 absolute;
gradients within |g - o| <= 1e-3 |o| + 1e-4 max|o| per tensor.  Pixels where the oracle
reports a decision (skip / stop / exponent sign) within rounding of its threshold, and
Gaussians whose radius is within rounding of an integer, are excluded and counted.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (IMG_TOL, assert_grad_close, excluded_pixels, log, make_ctx, to_gpu)

pytestmark = pytest.mark.gpu

BG = (0.05, 0.1, 0.15)


def gpu_render(scene, cams, bg=BG, ctx=None):
    g = to_gpu(scene)
    ctx = ctx or make_ctx(scene.n, cams)
    out = ctx.render_fwd(g, cams, bg)
    ctx.sync()
    return ctx, g, out


def small_multiview(seed=3, n=3000, views=3, W=200, H=150, deg=3):
    scene, cams, dls = synth.multiview_scene(seed, n=n, n_views=views, width=W, height=H)
    if deg != 3:
        K = (deg + 1) ** 2
        scene = synth.Scene(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh[:3 * K].copy(), deg)
    return scene, cams, dls


def large_footprint_sub(seed=0):
    """64 Gaussians from the large-footprint generator (SH3, log-scales N(-2, 0.5)), its four
    cameras at 32x32, upstream gradients N(0, 1)."""
    scene, cams = synth.large_footprint_scene(seed, n=64, width=32, height=32)
    rng = np.random.default_rng(seed + 1)
    return scene, cams, [rng.normal(size=(3, 32, 32)).astype(np.float32) for _ in cams]


def off_frustum(seed=11, n=200, W=96, H=72, views=2):
    """Gaussians beside the field of view whose footprints reach the image, seen by a yawed and
    pitched two-view rig (SH3): in every view tens of visible Gaussians lie beyond the Jacobian
    clamp (1.3x the half field of view), so the clipped J and its zero derivative are exercised."""
    return synth.off_frustum_scene(seed, n, W, H, n_views=views)


def opaque_clamp(seed=7):
    """240 small Gaussians behind 12 nearly opaque wide ones (SH1, 64x48): alpha meets the 0.99
    clamp near the opaque centres, so the clamped forward and its zero derivative are exercised."""
    return synth.opaque_scene(seed)


CASES = {
    "single_view_2000": lambda: synth.single_view_scene(0),
    "multiview_sh3_ragged": lambda: small_multiview(),
    "multiview_sh1": lambda: small_multiview(seed=5, n=1500, views=2, W=97, H=61, deg=1),
    "tiny_dense": lambda: synth.tiny_scene(2, 300, 40, 36, sh_degree=2, log_scale_mu=-2.0),
    "large_footprint_64_4x32x32": large_footprint_sub,
    "off_frustum_clamp_2x96x72": off_frustum,
    "opaque_alpha_clamp_64x48": opaque_clamp,
}


@pytest.mark.parametrize("case", list(CASES))
def test_projection_matches_oracle(case):
    scene, cams, _ = CASES[case]()
    log(f"[projection] {case} n={scene.n} views={len(cams)}")
    ctx, g, _ = gpu_render(scene, cams)
    for cam in cams:
        got = ctx.debug_projection(g, cam)
        p = oracle.project(scene, cam)
        vis = got[:, 15] > 0.5
        flag = (p.flags & oracle.FLAG_RADIUS) != 0
        np.testing.assert_array_equal(vis[~flag], p.visible[~flag])
        v = p.visible & ~flag
        np.testing.assert_allclose(got[v, 0:2], p.uv[v], rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(got[v, 2:5], p.conic[v], rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(got[v, 5], p.opacity[v], rtol=1e-12)
        np.testing.assert_allclose(got[v, 6:9], p.rgb[v], rtol=1e-9, atol=1e-12)
        np.testing.assert_array_equal(got[v, 10].astype(np.int32), p.radius[v])
        np.testing.assert_array_equal(got[v, 11:15].astype(np.int32), p.rect[v])
        assert flag.sum() <= max(2, scene.n // 1000)


@pytest.mark.parametrize("case", list(CASES))
def test_keys_values_ranges_bit_exact(case):
    scene, cams, _ = CASES[case]()
    log(f"[keys] {case}")
    ctx, g, _ = gpu_render(scene, cams)
    for v, cam in enumerate(cams):
        p = oracle.project(scene, cam)
        assert not np.any(p.flags & oracle.FLAG_RADIUS), "radius within rounding of an integer"
        k, val, r = oracle.keys(p, cam)
        TX, TY = oracle.tiles_of(cam, (16, 16))
        gk, gv, gr = ctx.debug_keys(v, k.size + 16, TX * TY)
        assert gk.size == k.size
        np.testing.assert_array_equal(gk, k)
        np.testing.assert_array_equal(gv, val)
        np.testing.assert_array_equal(gr, r)


@pytest.mark.parametrize("case", list(CASES))
def test_images_match_oracle(case):
    scene, cams, _ = CASES[case]()
    log(f"[image] {case}")
    ctx, g, out = gpu_render(scene, cams)
    for v, cam in enumerate(cams):
        vr = oracle.render_view(scene, cam, bg=BG)
        ex = excluded_pixels(vr, cam)
        rgb = out[v].rgb.cpu().numpy()
        T = out[v].t_final.cpu().numpy()
        nc = out[v].n_contrib.cpu().numpy()
        err = np.abs(rgb - vr.rgb)[:, ~ex]
        log(f"  view {v}: max |rgb| err {err.max():.2e}, excluded px {ex.sum()} / {ex.size}")
        assert err.max() <= IMG_TOL
        assert np.abs(T - vr.t_final)[~ex].max() <= IMG_TOL
        np.testing.assert_array_equal(nc[~ex], vr.n_contrib[~ex])
        assert ex.mean() <= 0.01


@pytest.mark.parametrize("case", list(CASES))
def test_gradients_match_oracle(case):
    scene, cams, dls = CASES[case]()
    log(f"[grad] {case}")
    renders = [oracle.render_view(scene, c, bg=BG) for c in cams]
    # upstream gradient zeroed where a decision sits within rounding of its threshold
    dls = [d.copy() for d in dls]
    for d, vr, cam in zip(dls, renders, cams):
        d[:, excluded_pixels(vr, cam, grad=True)] = 0.0
    og, _, ogn, ocnt = oracle.render_backward(scene, cams, dls, bg=BG, renders=renders)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    out = ctx.render_fwd(g, cams, BG)
    grads = g.zeros_like()
    gn = torch.zeros(g.capacity, device="cuda")
    cnt = torch.zeros(g.capacity, dtype=torch.int32, device="cuda")
    ctx.render_bwd(g, cams, BG, out, [torch.as_tensor(d, device="cuda") for d in dls], grads, gn, cnt)
    ctx.sync()
    gflag = np.zeros(scene.n, bool)
    for cam in cams:
        gflag |= (oracle.project(scene, cam).flags & oracle.GAUSS_GRAD_FLAGS) != 0
    for name in ("mean", "quat", "log_scale", "logit", "sh"):
        got = getattr(grads, name)[..., :scene.n].cpu().numpy()
        rel = assert_grad_close(name, got, getattr(og, name), exclude=gflag)
        log(f"  {name}: max rel err (significant) {rel:.2e}")
    np.testing.assert_array_equal(cnt[:scene.n].cpu().numpy(), ocnt)
    assert_grad_close("gradnorm", gn[:scene.n].cpu().numpy(), ogn, exclude=gflag)


def test_forward_is_deterministic_and_batch_independent():
    scene, cams, _ = small_multiview(seed=8, n=2500, views=3)
    log("[determinism]")
    ctx, g, out1 = gpu_render(scene, cams)
    out2 = ctx.render_fwd(g, cams, BG)
    ctx.sync()
    for a, b in zip(out1, out2):
        assert torch.equal(a.rgb, b.rgb) and torch.equal(a.t_final, b.t_final) and torch.equal(a.n_contrib, b.n_contrib)
    # each view alone equals the same view inside the batched launch
    for v, cam in enumerate(cams):
        ctx1 = make_ctx(scene.n, [cam])
        alone = ctx1.render_fwd(g, [cam], BG)
        ctx1.sync()
        assert torch.equal(alone[0].rgb, out1[v].rgb)
        assert torch.equal(alone[0].n_contrib, out1[v].n_contrib)


def test_edge_cases_empty_culled_and_huge():
    cam = synth.make_camera(np.eye(3), (0, 0, 0), 70, 45)
    bgt = torch.tensor(BG, device="cuda").view(3, 1, 1)
    # no Gaussians: background everywhere
    empty = synth.Scene(np.zeros((3, 0), np.float32), np.zeros((4, 0), np.float32), np.zeros((3, 0), np.float32),
                        np.zeros(0, np.float32), np.zeros((3, 0), np.float32), 0)
    log("[edge] empty")
    ctx, g, out = gpu_render(empty, [cam])
    assert torch.allclose(out[0].rgb, bgt.expand_as(out[0].rgb))
    assert torch.all(out[0].n_contrib == 0) and torch.all(out[0].t_final == 1)
    # every Gaussian behind the camera or at the near plane
    rng = np.random.default_rng(0)
    behind = synth.Scene(np.stack([rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50), rng.uniform(-5, 0.2, 50)]
                                  ).astype(np.float32), synth._quats(rng, 50),
                         np.full((3, 50), -2.0, np.float32), np.zeros(50, np.float32), np.zeros((3, 50), np.float32), 0)
    log("[edge] culled")
    ctx, g, out = gpu_render(behind, [cam])
    assert torch.allclose(out[0].rgb, bgt.expand_as(out[0].rgb))
    # one Gaussian covering every tile, plus a few small ones in front of it
    big = synth.Scene(np.array([[0.0, 0.05, -0.1], [0.0, 0.02, 0.03], [3.0, 1.0, 1.2]], np.float32),
                      np.array([[1, 1, 1], [0, 0, 0], [0, 0, 0], [0, 0, 0]], np.float32),
                      np.log(np.array([[2.0, 0.02, 0.03], [2.0, 0.02, 0.01], [2.0, 0.02, 0.02]], np.float32)),
                      np.array([2.0, 0.0, 1.0], np.float32),
                      ((np.array([[0.9, 0.1, 0.4], [0.2, 0.8, 0.4], [0.1, 0.1, 0.9]]) - 0.5) / synth.Y00
                       ).astype(np.float32), 0)
    log("[edge] huge")
    ctx, g, out = gpu_render(big, [cam])
    vr = oracle.render_view(big, cam, bg=BG)
    assert vr.proj.rect[0].tolist() == [0, 0, 5, 3]
    ex = excluded_pixels(vr, cam)
    assert np.abs(out[0].rgb.cpu().numpy() - vr.rgb)[:, ~ex].max() <= IMG_TOL


def test_key_overflow_is_reported():
    from paper_2411_14847_amd import Context, DassError
    scene, cams, _ = synth.single_view_scene(0)
    ctx = Context(max_gaussians=scene.n, max_views=1, max_keys=1000, max_tiles=64)
    g = to_gpu(scene)
    ctx.render_fwd(g, cams, BG)
    with pytest.raises(DassError) as e:
        ctx.sync()
    assert "DASS_E_CAPACITY" in str(e.value)
    ctx.sync()  # cleared


def test_invalid_arguments_are_rejected():
    from paper_2411_14847_amd import Context, DassError
    scene, cams, _ = synth.single_view_scene(0, n=10)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    g.sh_degree = 4
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_fwd(g, cams, BG)
    g.sh_degree = 0
    g.n = g.capacity + 1
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_fwd(g, cams, BG)
    g.n = scene.n
    with pytest.raises(DassError, match="DASS_E_CAPACITY"):
        ctx.render_fwd(g, cams * 2, BG)  # more views than reserved
    small = Context(max_gaussians=5, max_views=1, max_keys=100, max_tiles=64)
    with pytest.raises(DassError, match="DASS_E_CAPACITY"):
        small.render_fwd(g, cams, BG)
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_bwd(g, cams, BG, [], [], g.zeros_like())  # no matching forward yet on a fresh context


def test_backward_must_match_the_forward_cameras_and_background():
    """render_bwd walks the lists of the last render_fwd: a call with other poses of the same image
    size, or another background, is refused instead of chaining stale records."""
    from paper_2411_14847_amd import DassError
    scene, cams, dls = small_multiview(seed=4, n=400, views=2, W=64, H=48)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    out = ctx.render_fwd(g, cams, BG)
    dl = [torch.as_tensor(d, device="cuda") for d in dls]
    moved = [synth.make_camera(c.R.astype(np.float64), c.campos.astype(np.float64) + np.array([0.01, 0, 0]),
                               c.width, c.height) for c in cams]
    log("[bwd check] moved cameras, other background")
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_bwd(g, moved, BG, out, dl, g.zeros_like())
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_bwd(g, cams, (0.5, 0.5, 0.5), out, dl, g.zeros_like())
    grads = g.zeros_like()
    ctx.render_bwd(g, cams, BG, out, dl, grads)  # the matching call still runs
    ctx.sync()
    assert torch.isfinite(grads.mean).all() and grads.mean.abs().sum() > 0

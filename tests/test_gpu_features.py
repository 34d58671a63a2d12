"""GPU parity of identity-feature rendering (dass_render_features: the C-channel blend with the
colour render's weights) and of the dynamics mask built on it (dass_dynamic_mask, Sec. 3.3)
against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import IMG_TOL, excluded_pixels, log, make_ctx, to_gpu

pytestmark = pytest.mark.gpu
BG = (0.1, 0.05, 0.0)


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


@pytest.mark.parametrize("tile", [(16, 16), (32, 32), (32, 32, 8), (64, 32)])
@pytest.mark.parametrize("channels", [16, 5])
def test_feature_render_matches_oracle(tile, channels):
    scene, cams, _ = synth.multiview_scene(31, n=2500, n_views=3, width=100, height=84, with_grads=False)
    feat, _, _, _ = synth.identity_setup(32, scene.n, channels=channels)
    log(f"feature render tile {tile} channels {channels}")
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    ctx.tile = tile
    outs = ctx.render_fwd(g, cams, BG)
    fdev = torch.zeros(channels, g.capacity, device="cuda")
    fdev[:, :scene.n] = dev(feat)
    F = ctx.render_features(g, cams, fdev)
    ctx.sync()
    for v, c in enumerate(cams):
        vr = oracle.render_view(scene, c, bg=BG, tile=tile[:2])
        want = oracle.render_features(vr, c, feat, tile=tile[:2])
        keep = ~excluded_pixels(vr, c, tile=tile[:2])
        got = F[v].cpu().numpy()
        err = np.abs(got - want)[:, keep].max()
        assert err <= IMG_TOL, (v, err)
        # with every feature 1 the image is the coverage 1 - T_final of the same render
    ones = torch.ones(channels, g.capacity, device="cuda")
    F1 = ctx.render_features(g, cams, ones)
    ctx.sync()
    for v in range(len(cams)):
        cov = 1.0 - outs[v].t_final.cpu().numpy()
        assert np.abs(F1[v].cpu().numpy() - cov[None]).max() <= 1e-5


def test_feature_render_requires_matching_forward():
    from paper_2411_14847_amd import DassError
    scene, cams, _ = synth.multiview_scene(33, n=500, n_views=2, width=64, height=48, with_grads=False)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    f = torch.zeros(16, g.capacity, device="cuda")
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_features(g, cams, f)          # no render_fwd yet
    ctx.render_fwd(g, cams, BG)
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_features(g, cams[:1], f)      # other cameras
    with pytest.raises(DassError, match="DASS_E_INVALID"):
        ctx.render_features(g, cams, torch.zeros(17, g.capacity, device="cuda"))


def _margin(cls_w, cls_b, x):
    s = np.asarray(cls_w, np.float64) @ np.asarray(x, np.float64) + np.asarray(cls_b, np.float64)[:, None]
    top = np.sort(s, axis=0)
    return top[-1] - top[-2]


@pytest.mark.parametrize("n_objects", [8, 200])
def test_dynamic_mask_matches_oracle(n_objects):
    """Flow-thresholded pixels -> objects of the rendered identity features -> Gaussians of those
    objects.  Pixels whose classification is within 1e-2 of a tie, and pixels where
    the oracle flags a float decision, get no flow (they decide nothing); Gaussians within 1e-3
    may go either way."""
    scene, cams, _ = synth.multiview_scene(34, n=3000, n_views=3, width=100, height=84, with_grads=False)
    feat, obj, cls_w, cls_b = synth.identity_setup(35, scene.n, n_objects=n_objects)
    flows = synth.flow_maps(36, cams, frac=0.002)
    gamma = 1.0
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    ctx.render_fwd(g, cams, BG)
    fdev = torch.zeros(16, g.capacity, device="cuda")
    fdev[:, :scene.n] = dev(feat)
    F = ctx.render_features(g, cams, fdev)
    oimgs = []
    for v, c in enumerate(cams):
        vr = oracle.render_view(scene, c, bg=BG)
        oimg = oracle.render_features(vr, c, feat)
        oimgs.append(oimg)
        amb = excluded_pixels(vr, c) | (_margin(cls_w, cls_b, oimg.reshape(16, -1)) < 1e-2).reshape(c.height, c.width)
        flows[v][amb] = 0.0
    dyn_obj, want = oracle.dynamic_gaussians(oimgs, flows, gamma, cls_w, cls_b, feat)
    log(f"dynamic objects {dyn_obj.sum()} of {n_objects}, dynamic Gaussians {want.size}")
    idx = torch.full((scene.n,), -1, dtype=torch.int32, device="cuda")
    nd = torch.zeros(1, dtype=torch.int32, device="cuda")
    objs = torch.zeros(n_objects, dtype=torch.int32, device="cuda")
    ctx.dynamic_mask(cams, F, [dev(f) for f in flows], gamma, dev(cls_w), dev(cls_b), fdev, scene.n, idx, nd,
                     dyn_objects=objs)
    ctx.sync()
    np.testing.assert_array_equal(objs.cpu().numpy().astype(bool), dyn_obj)
    k = int(nd.item())
    got = idx[:k].cpu().numpy()
    assert np.all(np.diff(got) > 0)
    amb_g = set(np.nonzero(_margin(cls_w, cls_b, feat) < 1e-3)[0].tolist())
    assert set(got.tolist()) ^ set(want.tolist()) <= amb_g
    assert 0 < k <= scene.n
    if n_objects > 8:
        assert 0 < dyn_obj.sum() < n_objects and k < scene.n  # a proper subset


def test_dynamic_mask_degenerate_cases():
    """No flow above the threshold: no dynamic object and no dynamic Gaussian; no Gaussians at
    all: an empty list with the count written."""
    scene, cams, _ = synth.multiview_scene(37, n=800, n_views=2, width=64, height=48, with_grads=False)
    feat, _, cls_w, cls_b = synth.identity_setup(38, scene.n, n_objects=5)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams)
    ctx.render_fwd(g, cams, BG)
    fdev = torch.zeros(16, g.capacity, device="cuda")
    fdev[:, :scene.n] = dev(feat)
    F = ctx.render_features(g, cams, fdev)
    flows = [torch.zeros(c.height, c.width, device="cuda") for c in cams]
    idx = torch.full((scene.n,), -1, dtype=torch.int32, device="cuda")
    nd = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    objs = torch.full((5,), 9, dtype=torch.int32, device="cuda")
    ctx.dynamic_mask(cams, F, flows, 1.0, dev(cls_w), dev(cls_b), fdev, scene.n, idx, nd, dyn_objects=objs)
    ctx.sync()
    assert int(nd.item()) == 0 and int(objs.abs().sum()) == 0
    ctx.dynamic_mask(cams, F, flows, 1.0, dev(cls_w), dev(cls_b), fdev, 0, idx, nd)
    ctx.sync()
    assert int(nd.item()) == 0

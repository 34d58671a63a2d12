"""Parity at the full multi-view workload (200,000 Gaussians, SH degree 3, 20 views at 1352x1014,
all views in one render call as the benchmark runs them), on outputs the oracle computes one
by one: complete sorted keys / ranges of two views, sampled tiles of the images, and complete
gradients of sampled Gaussians (the oracle blends only the tiles those Gaussians touch, which
is all their gradients depend on).  Run at 16x16 tiles and at every size the tile autotuner finds
within a few percent of the best for this workload on MI355X (32x32, 32x64, 64x32, 64x64)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import IMG_TOL, assert_grad_close, excluded_pixels, log, make_ctx, to_gpu

pytestmark = pytest.mark.gpu

BG = (0.0, 0.0, 0.0)


@pytest.fixture(scope="module", params=[(16, 16), (32, 32), (32, 64), (64, 32), (64, 64)],
                ids=["tile16x16", "tile32x32", "tile32x64", "tile64x32", "tile64x64"])
def full(request):
    tile = request.param
    log(f"[fullsize] generating 200k-Gaussian, 20-view scene (tile {tile[0]}x{tile[1]})")
    scene, cams, dls = synth.multiview_scene(0, n=200_000, n_views=20)
    g = to_gpu(scene)
    ctx = make_ctx(scene.n, cams, keys_per_gaussian=24)
    ctx.tile = tile
    out = ctx.render_fwd(g, cams, BG)
    ctx.sync()
    log("[fullsize] GPU forward done")
    projs = [oracle.project(scene, c, tile) for c in cams]
    keys = [oracle.keys(p, c, tile) for p, c in zip(projs, cams)]
    log("[fullsize] oracle projections and keys done")
    return dict(scene=scene, cams=cams, dls=dls, g=g, ctx=ctx, out=out, projs=projs, keys=keys, tile=tile)


@pytest.mark.parametrize("view", [0, 19])
def test_fullsize_keys_bit_exact(full, view):
    cam, p = full["cams"][view], full["projs"][view]
    k, v, r = full["keys"][view]
    flagged = np.nonzero(p.flags & oracle.FLAG_RADIUS)[0]
    TX, TY = oracle.tiles_of(cam, full["tile"])
    gk, gv, gr = full["ctx"].debug_keys(view, k.size + 4096, TX * TY)
    log(f"  view {view}: {k.size} keys, radius-flagged Gaussians {flagged.size}")
    if flagged.size == 0:
        np.testing.assert_array_equal(gk, k)
        np.testing.assert_array_equal(gv, v)
        np.testing.assert_array_equal(gr, r)
    else:  # compare the tiles no flagged Gaussian touches
        bad = np.zeros(TX * TY, bool)
        for gidx in flagged:
            x0, y0, x1, y1 = p.rect[gidx]
            for ty in range(max(0, y0 - 1), min(TY, y1 + 1)):
                bad[ty * TX + max(0, x0 - 1): ty * TX + min(TX, x1 + 1)] = True
        for t in np.nonzero(~bad)[0]:
            np.testing.assert_array_equal(gk[gr[t, 0]:gr[t, 1]], k[r[t, 0]:r[t, 1]])
            np.testing.assert_array_equal(gv[gr[t, 0]:gr[t, 1]], v[r[t, 0]:r[t, 1]])


@pytest.mark.parametrize("view", [0, 7, 19])
def test_fullsize_sampled_tiles_match(full, view):
    cam, tile = full["cams"][view], full["tile"]
    TX, TY = oracle.tiles_of(cam, tile)
    rng = np.random.default_rng(100 + view)
    n_pick = max(4, 20 * 256 // (tile[0] * tile[1]))
    tiles = np.concatenate([rng.choice(TX * TY, n_pick, replace=False), [TX * TY - 1, TX - 1]])  # + ragged corners
    vr = oracle.render_view(full["scene"], cam, bg=BG, tile=tile, tiles=tiles, proj=full["projs"][view],
                            key_data=full["keys"][view])
    m = vr.computed & ~excluded_pixels(vr, cam, tile=tile)
    o = full["out"][view]
    err = np.abs(o.rgb.cpu().numpy() - vr.rgb)[:, m].max()
    log(f"  view {view}: {m.sum()} pixels compared, max |rgb| err {err:.2e}")
    assert err <= IMG_TOL
    assert np.abs(o.t_final.cpu().numpy() - vr.t_final)[m].max() <= IMG_TOL
    np.testing.assert_array_equal(o.n_contrib.cpu().numpy()[m], vr.n_contrib[m])


def test_fullsize_sampled_gaussian_gradients(full):
    scene, cams, projs, tile = full["scene"], full["cams"], full["projs"], full["tile"]
    n = scene.n
    rng = np.random.default_rng(7)
    nvis = np.sum([p.visible for p in projs], axis=0)
    gflag = np.zeros(n, bool)
    for p in projs:
        gflag |= (p.flags & oracle.GAUSS_GRAD_FLAGS) != 0
    cand = np.nonzero((nvis >= 10) & ~gflag)[0]
    sample = rng.choice(cand, 12, replace=False)
    only = np.zeros(n, np.int32)
    only[sample] = 1
    # per view: the tiles the sampled Gaussians touch; upstream gradient zeroed at flagged pixels
    dls = [d.copy() for d in full["dls"]]
    renders, tile_lists = [], []
    for v, (cam, p) in enumerate(zip(cams, projs)):
        TX, _ = oracle.tiles_of(cam, tile)
        ts = set()
        for gidx in sample:
            if p.visible[gidx]:
                x0, y0, x1, y1 = p.rect[gidx]
                ts.update(ty * TX + tx for ty in range(y0, y1) for tx in range(x0, x1))
        tl = np.array(sorted(ts), np.int32)
        tile_lists.append(tl)
        vr = oracle.render_view(scene, cam, bg=BG, tile=tile, tiles=tl, proj=p, key_data=full["keys"][v])
        dls[v][:, vr.computed & excluded_pixels(vr, cam, grad=True, tile=tile)] = 0.0
        renders.append(vr)
    log(f"  oracle backward over {sum(t.size for t in tile_lists)} tiles")
    og, _, ogn, ocnt = oracle.render_backward(scene, cams, dls, bg=BG, tile=tile, renders=renders, tiles=tile_lists,
                                              only=only)
    ctx, g = full["ctx"], full["g"]
    grads = g.zeros_like()
    gn = torch.zeros(g.capacity, device="cuda")
    cnt = torch.zeros(g.capacity, dtype=torch.int32, device="cuda")
    ctx.render_fwd(g, cams, BG, out=full["out"])
    ctx.render_bwd(g, cams, BG, full["out"], [torch.as_tensor(d, device="cuda") for d in dls], grads, gn, cnt)
    ctx.sync()
    for name in ("mean", "quat", "log_scale", "logit", "sh"):
        got = getattr(grads, name)[..., :n].cpu().numpy()[..., sample]
        want = getattr(og, name)[..., sample]
        rel = assert_grad_close(name, got, want)
        log(f"  {name}: max rel err (significant) {rel:.2e}")
    np.testing.assert_array_equal(cnt.cpu().numpy()[sample], ocnt[sample])
    assert_grad_close("gradnorm", gn.cpu().numpy()[sample], ogn[sample])


def test_large_footprint_fullsize_sampled_tiles():
    """The large-footprint workload at full size (1,000,000 Gaussians, SH3, log-scales N(-2, 0.5),
    four 1920x1080 views) at the 64x64 tiles the autotuner picks for it: sampled tiles of two
    views against the oracle (keys of those views computed by the oracle at the same tile size)."""
    tile = (64, 64)
    log("[stress fullsize] generating the 1M-Gaussian scene")
    scene, cams = synth.large_footprint_scene(0)
    g = to_gpu(scene)
    from paper_2411_14847_amd import Context
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    ctx = Context(max_gaussians=scene.n, max_views=len(cams), max_keys=400_000_000, max_tiles=tiles)
    ctx.tile = tile
    out = ctx.render_fwd(g, cams, BG)
    ctx.sync()
    log("[stress fullsize] GPU forward done")
    for view in (0, 3):
        cam = cams[view]
        p = oracle.project(scene, cam, tile)
        k, v, r = oracle.keys(p, cam, tile)
        TX, TY = oracle.tiles_of(cam, tile)
        rng = np.random.default_rng(300 + view)
        picks = np.concatenate([rng.choice(TX * TY, 3, replace=False), [TX * TY - 1]])  # + ragged corner
        vr = oracle.render_view(scene, cam, bg=BG, tile=tile, tiles=picks, proj=p, key_data=(k, v, r))
        m = vr.computed & ~excluded_pixels(vr, cam, tile=tile)
        o = out[view]
        err = np.abs(o.rgb.cpu().numpy() - vr.rgb)[:, m].max()
        log(f"  view {view}: {k.size} keys, {m.sum()} pixels compared, max |rgb| err {err:.2e}")
        assert err <= IMG_TOL
        assert np.abs(o.t_final.cpu().numpy() - vr.t_final)[m].max() <= IMG_TOL
        np.testing.assert_array_equal(o.n_contrib.cpu().numpy()[m], vr.n_contrib[m])
        gk, gv, gr = ctx.debug_keys(view, k.size + 4096, TX * TY)
        for t in picks:  # the sampled tiles' sorted key lists, bit-exact
            np.testing.assert_array_equal(gk[gr[t, 0]:gr[t, 1]], k[r[t, 0]:r[t, 1]])
            np.testing.assert_array_equal(gv[gr[t, 0]:gr[t, 1]], v[r[t, 0]:r[t, 1]])


def test_fullsize_sampled_feature_tiles(full):
    """16-channel identity features of the full workload (same render call), sampled tiles of
    two views against the oracle's blend of the same lists."""
    scene, cams, tile, ctx, g = full["scene"], full["cams"], full["tile"], full["ctx"], full["g"]
    feat, _, _, _ = synth.identity_setup(40, scene.n)
    ctx.render_fwd(g, cams, BG)
    fdev = torch.zeros(16, g.capacity, device="cuda")
    fdev[:, :scene.n] = torch.as_tensor(feat, device="cuda")
    F = ctx.render_features(g, cams, fdev)
    ctx.sync()
    for view in (0, 13):
        cam = cams[view]
        TX, TY = oracle.tiles_of(cam, tile)
        rng = np.random.default_rng(200 + view)
        n_pick = max(3, 8 * 256 // (tile[0] * tile[1]))
        tiles = np.concatenate([rng.choice(TX * TY, n_pick, replace=False), [TX * TY - 1]])
        vr = oracle.render_view(scene, cam, bg=BG, tile=tile, tiles=tiles, proj=full["projs"][view],
                                key_data=full["keys"][view])
        want = oracle.render_features(vr, cam, feat, tile=tile, tiles=tiles)
        m = vr.computed & ~excluded_pixels(vr, cam, tile=tile)
        err = np.abs(F[view].cpu().numpy() - want)[:, m].max()
        log(f"  features view {view}: {m.sum()} pixels, max err {err:.2e}")
        assert err <= IMG_TOL

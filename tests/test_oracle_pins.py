"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: closed forms,
library routines (scipy, numpy, torch CPU), invariants, a brute-force
per-pixel blend, central finite differences, published known answers and
hand-evaluated fixtures under tests/golden/.
"""
import math
import os

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_gaussian_scene(mean, quat, log_scale, logit, colour=None, sh=None, deg=0):
    K = (deg + 1) ** 2
    if sh is None:
        sh = np.zeros((3 * K, 1), np.float32)
        c = np.asarray(colour if colour is not None else (0.2, 0.5, 0.8), np.float64)
        sh[0:3, 0] = (c - 0.5) / synth.Y00
    return synth.Scene(np.asarray(mean, np.float32).reshape(3, 1), np.asarray(quat, np.float32).reshape(4, 1),
                       np.asarray(log_scale, np.float32).reshape(3, 1), np.asarray([logit], np.float32),
                       np.asarray(sh, np.float32).reshape(3 * K, -1), deg)


def axis_camera(W=64, H=48, campos=(0.0, 0.0, 0.0)):
    """Camera looking down +z with R = I (x right, y down)."""
    return synth.make_camera(np.eye(3), campos, W, H)


# ------------------------------------------------------------------------------------------
# Projection (App. A.1: Sigma = R S S^T R^T, Sigma_2D = J W Sigma W^T J^T)
# ------------------------------------------------------------------------------------------
def test_isotropic_closed_form_footprint():
    """An isotropic Gaussian of scale s on the optical axis at depth z projects to the principal
    point with Sigma_2D = ((f s / z)^2 + 0.3) I, hence r = ceil(3 sqrt(.)), for any rotation."""
    cam = axis_camera(64, 48)
    rng = np.random.default_rng(1)
    for z, s in [(2.0, 0.01), (3.0, 0.05), (7.5, 0.2), (1.0, 0.003)]:
        q = rng.normal(size=4)
        sc = one_gaussian_scene((0, 0, z), q, np.log([s, s, s]), 0.3)
        p = oracle.project(sc, cam)
        z32, s32 = float(np.float32(z)), float(np.exp(np.float64(np.float32(np.log(s)))))
        var = (cam.fx * s32 / z32) ** 2 + float(np.float32(0.3))
        assert p.uv[0] == pytest.approx([cam.cx, cam.cy], abs=1e-12)
        assert p.conic[0] == pytest.approx([1.0 / var, 0.0, 1.0 / var], rel=1e-10, abs=1e-14)
        assert p.radius[0] == math.ceil(3.0 * math.sqrt(var))
        assert p.depth[0] == pytest.approx(z32, abs=0)


def numeric_jacobian(f, x, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3); e[k] = h
        J[:, k] = (f(x + e) - f(x - e)) / (2 * h)
    return J


@pytest.mark.parametrize("seed", range(6))
def test_projection_matches_numeric_jacobian_and_scipy_rotation(seed):
    """Sigma_2D from a numerically differentiated pinhole map and scipy's rotation matrix."""
    rng = np.random.default_rng(seed)
    R_cam = Rotation.from_rotvec(rng.normal(scale=0.2, size=3)).as_matrix()
    campos = rng.normal(scale=0.3, size=3)
    cam = synth.make_camera(R_cam, campos, 96, 80)
    # a point in front of the camera, within the clamp
    xc = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 1.0]) * rng.uniform(2, 6)
    Rw = cam.R.astype(np.float64)
    mean = Rw.T @ (xc - cam.t.astype(np.float64))
    q = rng.normal(size=4).astype(np.float32)
    ls = rng.normal(-2.5, 0.5, size=3).astype(np.float32)
    sc = one_gaussian_scene(mean, q, ls, 0.0)
    p = oracle.project(sc, cam)
    # expected, from library rotation (scalar-last) and numeric derivative of the pinhole map
    qd = q.astype(np.float64)
    Rq = Rotation.from_quat([qd[1], qd[2], qd[3], qd[0]]).as_matrix()
    S = np.diag(np.exp(ls.astype(np.float64)))
    Sigma = Rq @ S @ S.T @ Rq.T
    m64 = sc.mean[:, 0].astype(np.float64)
    tcam = Rw @ m64 + cam.t.astype(np.float64)

    def pin(x):
        return np.array([cam.fx * x[0] / x[2] + cam.cx, cam.fy * x[1] / x[2] + cam.cy])

    J = numeric_jacobian(pin, tcam)
    S2 = J @ Rw @ Sigma @ Rw.T @ J.T + float(np.float32(0.3)) * np.eye(2)
    conic = np.linalg.inv(S2)
    assert p.uv[0] == pytest.approx(pin(tcam), rel=1e-12)
    np.testing.assert_allclose([conic[0, 0], conic[0, 1], conic[1, 1]], p.conic[0], rtol=1e-6, atol=1e-9)
    lam = np.linalg.eigvalsh(S2).max()
    assert p.radius[0] == math.ceil(3 * math.sqrt(lam))


def clip_ratio_limits(cam):
    """1.3 x the half field-of-view tangents (the float32 constant 1.3 widened)."""
    c = float(np.float32(1.3))
    return c * cam.width / (2.0 * cam.fx), c * cam.height / (2.0 * cam.fy)


def clamped_visible(p, cam):
    """Visible Gaussians whose centre lies beyond the Jacobian clamp in x or y (from the pixel
    mean: (u - c_x) / f_x = t_x / t_z)."""
    limx, limy = clip_ratio_limits(cam)
    rx = (p.uv[:, 0] - cam.cx) / cam.fx
    ry = (p.uv[:, 1] - cam.cy) / cam.fy
    return p.visible & ((np.abs(rx) > limx) | (np.abs(ry) > limy))


@pytest.mark.parametrize("ax,ay", [(1.55, 0.2), (-1.7, -0.4), (0.3, 1.6), (-0.5, -1.45), (1.5, -1.5)])
def test_jacobian_clamp_closed_form(ax, ay):
    """A Gaussian whose centre lies beyond 1.3x the half field of view (App. A.1's J evaluated with
    t_x/t_z and t_y/t_z clipped) but whose footprint reaches the image: Sigma_2D equals the
    numerically differentiated pinhole map taken at the clipped point (lim t_z in place of t_x),
    while the pixel mean stays the unclipped projection.  The unclipped Jacobian gives a
    different footprint, so the clip is what is pinned."""
    W, H = 64, 48
    rng = np.random.default_rng(int(1000 * (ax + 3 * ay)) % 2**31)
    R_cam = Rotation.from_rotvec(rng.normal(scale=0.1, size=3)).as_matrix()
    cam = synth.make_camera(R_cam, rng.normal(scale=0.2, size=3), W, H)
    z = 3.0
    xc = np.array([ax * (W / 2) / cam.fx * z, ay * (H / 2) / cam.fy * z, z])
    Rw = cam.R.astype(np.float64)
    mean = Rw.T @ (xc - cam.t.astype(np.float64))
    q = rng.normal(size=4).astype(np.float32)
    ls = np.log(np.array([0.35, 0.3, 0.25]) * z * (W / 2) / cam.fx).astype(np.float32)
    sc = one_gaussian_scene(mean, q, ls, 1.0)
    p = oracle.project(sc, cam)
    assert p.visible[0], "the footprint must reach the image"
    assert clamped_visible(p, cam)[0]
    qd = q.astype(np.float64)
    Rq = Rotation.from_quat([qd[1], qd[2], qd[3], qd[0]]).as_matrix()
    S = np.diag(np.exp(ls.astype(np.float64)))
    Sigma = Rq @ S @ S.T @ Rq.T
    tcam = Rw @ sc.mean[:, 0].astype(np.float64) + cam.t.astype(np.float64)
    limx, limy = clip_ratio_limits(cam)
    tclip = np.array([np.clip(tcam[0] / tcam[2], -limx, limx) * tcam[2],
                      np.clip(tcam[1] / tcam[2], -limy, limy) * tcam[2], tcam[2]])

    def pin(x):
        return np.array([cam.fx * x[0] / x[2] + cam.cx, cam.fy * x[1] / x[2] + cam.cy])

    def conic_at(point):
        J = numeric_jacobian(pin, point)
        S2 = J @ Rw @ Sigma @ Rw.T @ J.T + float(np.float32(0.3)) * np.eye(2)
        c = np.linalg.inv(S2)
        return np.array([c[0, 0], c[0, 1], c[1, 1]]), np.linalg.eigvalsh(S2).max()

    want, lam = conic_at(tclip)
    np.testing.assert_allclose(p.conic[0], want, rtol=1e-6, atol=1e-12)
    assert p.radius[0] == math.ceil(3 * math.sqrt(lam))
    unclipped, _ = conic_at(tcam)
    assert np.abs(unclipped - want).max() > 1e-3 * np.abs(want).max()
    assert p.uv[0] == pytest.approx(pin(tcam), rel=1e-12)


def test_off_frustum_parity_fixture_reaches_the_clamp():
    """The GPU parity cases beside the field of view do exercise the clipped Jacobian: in every view
    at least 20 visible Gaussians lie beyond the clamp and receive gradient."""
    from test_gpu_parity import off_frustum
    sc, cams, dls = off_frustum()
    _, g2ds, _, _ = oracle.render_backward(sc, cams, dls, bg=(0.05, 0.1, 0.15))
    for cam, g2d in zip(cams, g2ds):
        hit = clamped_visible(oracle.project(sc, cam), cam) & (np.abs(g2d).sum(axis=1) > 0)
        assert hit.sum() >= 20


def test_opaque_parity_fixture_reaches_the_alpha_clamp():
    """The nearly opaque GPU parity case does blend entries at the 0.99 alpha clamp: walked by the
    per-pixel definition, at least 50 of its pixels blend an entry whose unclamped alpha is 0.99
    or more (alpha clamped, no derivative through it)."""
    from test_gpu_parity import opaque_clamp
    sc, cams, _ = opaque_clamp()
    cam = cams[0]
    p = oracle.project(sc, cam)
    amax, amin, tstop = float(np.float32(0.99)), float(np.float32(1 / 255)), float(np.float32(1e-4))
    order = sorted(np.nonzero(p.visible)[0], key=lambda g: (np.float32(p.depth[g]), g))
    hits = 0
    for py in range(cam.height):
        for px in range(cam.width):
            tx, ty, T, hit = px // 16, py // 16, 1.0, False
            for g in order:
                if not (p.rect[g, 0] <= tx < p.rect[g, 2] and p.rect[g, 1] <= ty < p.rect[g, 3]):
                    continue
                dx, dy = p.uv[g, 0] - px, p.uv[g, 1] - py
                A, B, C_ = p.conic[g]
                P = -0.5 * (A * dx * dx + C_ * dy * dy) - B * dx * dy
                if P > 0:
                    continue
                araw = p.opacity[g] * math.exp(P)
                a = min(amax, araw)
                if a < amin:
                    continue
                if T * (1 - a) < tstop:
                    break
                hit = hit or araw >= amax
                T *= 1 - a
            hits += hit
    assert hits >= 50


def test_rotation_invariants_via_isotropy():
    """Isotropic s makes Sigma = s^2 I for every q (R R^T = I), so the footprint ignores q."""
    cam = axis_camera(64, 64)
    rng = np.random.default_rng(3)
    base = oracle.project(one_gaussian_scene((0.1, -0.2, 3), (1, 0, 0, 0), np.log([0.04] * 3), 0.0), cam)
    for _ in range(10):
        p = oracle.project(one_gaussian_scene((0.1, -0.2, 3), rng.normal(size=4), np.log([0.04] * 3), 0.0), cam)
        np.testing.assert_allclose(p.conic, base.conic, rtol=1e-12)


def test_cull_near_plane_and_behind():
    cam = axis_camera(64, 64)
    for z, vis in [(0.1, False), (0.2, False), (0.2001, True), (-3.0, False)]:
        p = oracle.project(one_gaussian_scene((0, 0, z), (1, 0, 0, 0), np.log([0.001] * 3), 0.0), cam)
        assert bool(p.visible[0]) == vis


# ------------------------------------------------------------------------------------------
# SH colour (App. A.1 "view-dependent color property"; basis choice documented)
# ------------------------------------------------------------------------------------------
def sphere_grid(nt=200, nphi=400):
    th = (np.arange(nt) + 0.5) * np.pi / nt
    ph = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    T, Pp = np.meshgrid(th, ph, indexing="ij")
    w = np.sin(T) * (np.pi / nt) * (2 * np.pi / nphi)
    d = np.stack([np.sin(T) * np.cos(Pp), np.sin(T) * np.sin(Pp), np.cos(T)], -1).reshape(-1, 3)
    return d, w.reshape(-1), T.reshape(-1), Pp.reshape(-1)


def test_sh_orthonormal_by_quadrature():
    d, w, _, _ = sphere_grid()
    Y = oracle.sh_eval(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=2e-4)


def test_sh_matches_scipy_real_combinations():
    from scipy.special import sph_harm_y
    d, _, th, ph = sphere_grid(20, 30)
    Y = oracle.sh_eval(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            if m == 0:
                ref = sph_harm_y(l, 0, th, ph).real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, m, th, ph).real
            else:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, th, ph).imag
            np.testing.assert_allclose(Y[:, l * l + m + l], ref, atol=1e-12, err_msg=f"l={l} m={m}")


def test_degree0_colour_and_clamp():
    cam = axis_camera()
    for c, want in [((0.2, 0.5, 0.9), (0.2, 0.5, 0.9)), ((-0.3, 0.0, 1.4), (0.0, 0.0, 1.4))]:
        p = oracle.project(one_gaussian_scene((0, 0, 3), (1, 0, 0, 0), np.log([0.05] * 3), 0.0, colour=c), cam)
        np.testing.assert_allclose(p.rgb[0], want, atol=1e-7)


# ------------------------------------------------------------------------------------------
# Blend (App. A.1: C = sum c_i a_i prod_{j<i} (1 - a_j); thresholds documented)
# ------------------------------------------------------------------------------------------
def test_single_gaussian_closed_form():
    cam = axis_camera(64, 48)
    bg = (0.1, 0.2, 0.3)
    for logit in (-1.0, 2.0, 8.0):
        sc = one_gaussian_scene((0.05, -0.03, 2.0), (0.9, 0.1, 0.3, -0.2), np.log([0.03, 0.02, 0.01]), logit,
                                colour=(0.9, 0.4, 0.1))
        vr = oracle.render_view(sc, cam, bg=bg)
        p = vr.proj
        TX, TY = oracle.tiles_of(cam, (16, 16))
        ys, xs = np.mgrid[0:48, 0:64]
        dx = p.uv[0, 0] - xs; dy = p.uv[0, 1] - ys
        A, B, Cc = p.conic[0]
        P = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        a = np.minimum(float(np.float32(0.99)), p.opacity[0] * np.exp(P))
        x0, y0, x1, y1 = p.rect[0]
        inside = (xs // 16 >= x0) & (xs // 16 < x1) & (ys // 16 >= y0) & (ys // 16 < y1)
        use = inside & (a >= float(np.float32(1 / 255))) & (P <= 0)
        for ch in range(3):
            want = np.where(use, p.rgb[0, ch] * a + (1 - a) * bg[ch], bg[ch])
            np.testing.assert_allclose(vr.rgb[ch], want, atol=1e-15)


def test_two_gaussians_closed_form_depth_order():
    cam = axis_camera(32, 32)
    mean = np.array([[0.0, 0.01], [0.0, 0.0], [2.0, 1.5]], np.float32)  # second is nearer
    sc = synth.Scene(mean, np.array([[1, 1], [0, 0], [0, 0], [0, 0]], np.float32),
                     np.log(np.full((3, 2), 0.05, np.float32)), np.array([0.5, -0.5], np.float32),
                     ((np.array([[0.9, 0.1], [0.2, 0.7], [0.3, 0.3]]) - 0.5) / synth.Y00).astype(np.float32), 0)
    bg = (0.05, 0.1, 0.15)
    vr = oracle.render_view(sc, cam, bg=bg)
    p = vr.proj
    ys, xs = np.mgrid[0:32, 0:32]

    def alpha(g):
        dx = p.uv[g, 0] - xs; dy = p.uv[g, 1] - ys
        A, B, Cc = p.conic[g]
        P = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        a = np.minimum(float(np.float32(0.99)), p.opacity[g] * np.exp(P))
        return np.where(a >= float(np.float32(1 / 255)), a, 0.0)

    a1, a2 = alpha(1), alpha(0)  # nearer first
    for ch in range(3):
        want = p.rgb[1, ch] * a1 + p.rgb[0, ch] * a2 * (1 - a1) + (1 - a1) * (1 - a2) * bg[ch]
        np.testing.assert_allclose(vr.rgb[ch], want, atol=1e-13)


def brute_force_pixel(p, gids, px, py, bg):
    """Per-pixel definition: the Gaussians whose rectangle holds this pixel's tile, sorted by
    (float32 depth, index), walked front to back with the documented thresholds."""
    order = sorted(gids, key=lambda g: (np.float32(p.depth[g]), g))
    T, Cc, last = 1.0, np.zeros(3), 0
    amax, amin, tstop = float(np.float32(0.99)), float(np.float32(1 / 255)), float(np.float32(1e-4))
    for i, g in enumerate(order):
        dx, dy = p.uv[g, 0] - px, p.uv[g, 1] - py
        A, B, C_ = p.conic[g]
        P = -0.5 * (A * dx * dx + C_ * dy * dy) - B * dx * dy
        if P > 0:
            continue
        a = min(amax, p.opacity[g] * math.exp(P))
        if a < amin:
            continue
        Tn = T * (1 - a)
        if Tn < tstop:
            break
        Cc += p.rgb[g] * a * T
        T = Tn
        last = i + 1
    return Cc + T * np.asarray(bg), T, last


@pytest.mark.parametrize("seed,deg", [(0, 0), (1, 1), (2, 3)])
def test_tiled_blend_equals_brute_force(seed, deg):
    sc, cams, _ = synth.tiny_scene(seed, 40, 40, 36, sh_degree=deg, log_scale_mu=-2.2)
    cam = cams[0]
    bg = (0.3, 0.1, 0.2)
    vr = oracle.render_view(sc, cam, bg=bg)
    p = vr.proj
    TX, TY = oracle.tiles_of(cam, (16, 16))
    for py in range(0, 36, 3):
        for px in range(0, 40, 3):
            tx, ty = px // 16, py // 16
            gids = [g for g in range(sc.n) if p.visible[g] and p.rect[g, 0] <= tx < p.rect[g, 2]
                    and p.rect[g, 1] <= ty < p.rect[g, 3]]
            C_, T, last = brute_force_pixel(p, gids, float(px), float(py), bg)
            np.testing.assert_allclose(vr.rgb[:, py, px], C_, atol=1e-14)
            assert vr.t_final[py, px] == pytest.approx(T, abs=1e-15)
            assert vr.n_contrib[py, px] == last


def white_scene(sc):
    out = sc.copy()
    out.sh[:] = 0
    out.sh[0:3] = (1.0 - 0.5) / synth.Y00
    return out


@pytest.mark.parametrize("seed", [0, 5])
def test_blend_invariants(seed):
    """sum_i a_i T_i + T_final = 1 (render white with black background); T_final >= 1e-4;
    a pixel whose walk stopped early has T_final < 1e-2 (since alpha <= 0.99)."""
    sc, cams, _ = synth.single_view_scene(seed)
    sc = white_scene(sc)
    vr = oracle.render_view(sc, cams[0], bg=(0, 0, 0))
    np.testing.assert_allclose(vr.rgb[0] + vr.t_final, 1.0, atol=1e-12)
    assert vr.t_final.min() >= float(np.float32(1e-4))
    # dense pile-up: many opaque Gaussians at one pixel stop early
    n = 60
    dense = synth.Scene(np.tile(np.array([[0.0], [0.0], [0.0]], np.float32), (1, n)) +
                        np.linspace(0, 0.5, n, dtype=np.float32)[None] * np.array([[0], [0], [1]], np.float32),
                        np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
                        np.full((3, n), np.log(0.3), np.float32), np.full(n, 3.0, np.float32),
                        np.full((3, n), 0.5 / synth.Y00, np.float32), 0)
    vr2 = oracle.render_view(dense, cams[0], bg=(0, 0, 0))
    lens = vr2.ranges[:, 1] - vr2.ranges[:, 0]
    centre_tile = (64 // 16) * 8 + 64 // 16
    assert vr2.n_contrib[64, 64] < lens[centre_tile]
    assert vr2.t_final[64, 64] < 1e-2
    assert vr2.t_final[64, 64] >= float(np.float32(1e-4))


def test_transmittance_monotone_along_lists():
    sc, cams, _ = synth.tiny_scene(4, 50, 32, 32, log_scale_mu=-2.0)
    vr = oracle.render_view(white_scene(sc), cams[0])
    # T after k entries is non-increasing in k: check via prefix renders with truncated lists
    Ts = []
    for cut in range(0, 60, 5):
        r = vr.ranges.copy()
        r[:, 1] = np.minimum(r[:, 1], r[:, 0] + cut)
        vrk = oracle.render_view(white_scene(sc), cams[0], key_data=(vr.keys, vr.vals, r))
        Ts.append(vrk.t_final)
    for a, b in zip(Ts, Ts[1:]):
        assert np.all(b <= a + 1e-15)


# ------------------------------------------------------------------------------------------
# Keys, sort, ranges
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
def test_keys_sort_ranges_against_numpy(seed):
    sc, cams, _ = synth.single_view_scene(seed)
    cam = cams[0]
    p = oracle.project(sc, cam)
    k, v, r = oracle.keys(p, cam)
    TX, TY = oracle.tiles_of(cam, (16, 16))
    # library sort of the same (key, value) multiset
    raw = []
    for g in range(sc.n):
        if not p.visible[g]:
            continue
        x0, y0, x1, y1 = p.rect[g]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                raw.append(((ty * TX + tx) << 32) | int(p.depth_bits[g]))
    raw_v = []
    for g in range(sc.n):
        if p.visible[g]:
            x0, y0, x1, y1 = p.rect[g]
            raw_v += [g] * ((x1 - x0) * (y1 - y0))
    raw = np.array(raw, np.uint64); raw_v = np.array(raw_v, np.uint32)
    order = np.argsort(raw, kind="stable")
    np.testing.assert_array_equal(k, raw[order])
    np.testing.assert_array_equal(v, raw_v[order])
    tiles = (k >> np.uint64(32)).astype(np.int64)
    lo = np.searchsorted(tiles, np.arange(TX * TY), side="left")
    hi = np.searchsorted(tiles, np.arange(TX * TY), side="right")
    empty = lo == hi
    lo[empty] = 0; hi[empty] = 0
    np.testing.assert_array_equal(r[:, 0], lo)
    np.testing.assert_array_equal(r[:, 1], hi)
    # depth bits are the float32 camera-space depth
    assert np.all(p.depth_bits[p.visible] == p.depth[p.visible].astype(np.float32).view(np.uint32))


# ------------------------------------------------------------------------------------------
# Gradients: central finite differences of L = sum dl * render
# ------------------------------------------------------------------------------------------
def _loss_and_sig(sc, cam, dl, bg):
    vr = oracle.render_view(sc, cam, bg=bg)
    return float(np.sum(vr.rgb * dl)), (vr.keys.tobytes(), vr.signature.tobytes())


# Fourth-order central differences, f'(x) = (8 (f(x+h) - f(x-h)) - (f(x+2h) - f(x-2h))) / 12h with
# h = 1e-4 max(1, |x|): truncation O(h^4) and rounding ~1e-16 |L| / h both stay near 1e-10, so the
# oracle is held to 1e-6 relative (errors seen: below 2e-8).  When one of the four points crosses a
# discrete decision the step drops to 1e-5 (errors seen there: below 3e-7).  The second-order
# stencil at h = 1e-6 has rounding noise of ~1e-9 absolute, 1e-6 of the smallest gradients kept.
FD_STEPS, FD_REL, FD_FLOOR = (1e-4, 1e-5), 1e-6, 1e-3


def fd4(loss_sig, arr, idx):
    """Fourth-order central difference of loss_sig()[0] in arr[idx]; None when at every step some
    perturbation changes a discrete decision (the signatures differ)."""
    x = arr[idx]
    for step in FD_STEPS:
        h = step * max(1.0, abs(x))
        vals, sigs = [], []
        for k in (2, 1, -1, -2):
            arr[idx] = x + k * h
            val, sig = loss_sig()
            vals.append(val)
            sigs.append(sig)
        arr[idx] = x
        if all(sg == sigs[0] for sg in sigs[1:]):
            return (8.0 * (vals[1] - vals[2]) - (vals[0] - vals[3])) / (12.0 * h)
    return None


def assert_fd(name, idx, ana, fd):
    assert abs(ana - fd) <= FD_REL * max(abs(fd), FD_FLOOR), f"{name}{idx}: analytic {ana} fd {fd}"


def float64_scene(sc):
    """The scene with float64 planes, so perturbations are exact."""
    return synth.Scene(sc.mean.astype(np.float64), sc.quat.astype(np.float64), sc.log_scale.astype(np.float64),
                       sc.logit.astype(np.float64), sc.sh.astype(np.float64), sc.sh_degree)


def decision_trace(vr, cam):
    """The discrete decisions of one render: each key's tile and the order of the values (the depth
    bits themselves move with every perturbation of a depth and decide nothing else), which side of
    the Jacobian clamp each centre lies on, which colour channels the clamp at 0 holds, and each
    pixel's blended entries."""
    limx, limy = clip_ratio_limits(cam)
    p = vr.proj
    clip = np.stack([np.abs((p.uv[:, 0] - cam.cx) / cam.fx) > limx, np.abs((p.uv[:, 1] - cam.cy) / cam.fy) > limy])
    dark = np.asarray(p.rgb) <= 0.0
    return ((vr.keys >> np.uint64(32)).tobytes() + vr.vals.tobytes() + clip.tobytes() + dark.tobytes() +
            vr.signature.tobytes())


def check_all_fd(sc, cams, dls, bg):
    """Every parameter element of sc against fd4 of L = sum_v <dl_v, render_v>; returns (checked,
    skipped)."""
    g, _, _, _ = oracle.render_backward(sc, cams, dls, bg=bg)
    sc64 = float64_scene(sc)

    def loss_sig():
        tot, sig = 0.0, []
        for cam, dl in zip(cams, dls):
            vr = oracle.render_view(sc64, cam, bg=bg)
            tot += float(np.sum(vr.rgb * dl))
            sig.append(decision_trace(vr, cam))
        return tot, sig

    checked = skipped = 0
    for name in ("mean", "quat", "log_scale", "logit", "sh"):
        arr = getattr(sc64, name)
        ana = getattr(g, name)
        for idx in np.ndindex(arr.shape):
            fd = fd4(loss_sig, arr, idx)
            if fd is None:
                skipped += 1
                continue
            assert_fd(name, idx, ana[idx], fd)
            checked += 1
    return checked, skipped


@pytest.mark.parametrize("seed,deg", [(0, 1), (1, 3), (2, 0)])
def test_gradients_match_finite_differences(seed, deg):
    sc, cams, dls = synth.tiny_scene(seed, 6, 32, 32, sh_degree=deg, log_scale_mu=-2.0, spread=0.4)
    checked, skipped = check_all_fd(sc, cams, [dls[0].astype(np.float64)], (0.2, 0.1, 0.05))
    assert checked > 0.9 * (checked + skipped)


@pytest.mark.parametrize("seed,deg", [(1, 1), (4, 3)])
def test_gradients_beyond_the_jacobian_clamp_match_finite_differences(seed, deg):
    """Gaussians centred beside the field of view (beyond 1.3x the half field of view in x or y)
    whose footprints reach the image: the adjoint of the clipped Jacobian (the clipped
    coordinate is lim t_z, so t_z carries it and t_x / t_y do not) against central differences,
    over two views turned by yaw and pitch."""
    sc, cams, dls = synth.off_frustum_scene(seed, 8, 40, 32, n_views=2, sh_degree=deg)
    for cam in cams:
        assert clamped_visible(oracle.project(sc, cam), cam).sum() >= 2
    checked, skipped = check_all_fd(sc, cams, [d.astype(np.float64) for d in dls], (0.1, 0.2, 0.3))
    assert checked > 0.9 * (checked + skipped)


def test_large_footprint_subscene_gradients_match_finite_differences():
    """64 Gaussians of the large-footprint generator (SH3, log-scales N(-2, 0.5)) seen by its four
    cameras at 32x32: the summed-over-views gradient of L = sum_v <dl_v, render_v> against central
    differences, on a seeded sample of 240 parameter elements."""
    sc, cams = synth.large_footprint_scene(0, n=64, width=32, height=32)
    rng = np.random.default_rng(17)
    # upstream gradients are float32 at the boundary (the oracle takes them as float32 too)
    dls = [rng.normal(size=(3, 32, 32)).astype(np.float32).astype(np.float64) for _ in cams]
    bg = (0.1, 0.2, 0.3)
    g, _, _, _ = oracle.render_backward(sc, cams, dls, bg=bg)
    sc64 = float64_scene(sc)

    def loss_sig():
        tot, sig = 0.0, []
        for cam, dl in zip(cams, dls):
            vr = oracle.render_view(sc64, cam, bg=bg)
            tot += float(np.sum(vr.rgb * dl))
            sig.append(decision_trace(vr, cam))
        return tot, sig

    names = ("mean", "quat", "log_scale", "logit", "sh")
    sizes = [getattr(sc64, nm).size for nm in names]
    picks = rng.choice(sum(sizes), size=240, replace=False)
    checked = skipped = 0
    for flat in picks:
        k = int(np.searchsorted(np.cumsum(sizes), flat, side="right"))
        name = names[k]
        arr = getattr(sc64, name)
        idx = np.unravel_index(int(flat - (np.cumsum(sizes)[k - 1] if k else 0)), arr.shape)
        fd = fd4(loss_sig, arr, idx)
        if fd is None:
            skipped += 1
            continue
        assert_fd(name, idx, getattr(g, name)[idx], fd)
        checked += 1
    assert checked > 0.9 * (checked + skipped)


# ------------------------------------------------------------------------------------------
# Shift (Sec. 3.3): p' = p + mu_n, q' = norm(q) x norm(sigma_n)
# ------------------------------------------------------------------------------------------
def test_shift_zero_offsets_is_identity():
    sc, _, _ = synth.single_view_scene(0, n=50)
    dyn = np.arange(0, 50, 3, dtype=np.int32)
    dpos = np.zeros((3, dyn.size)); drot = np.tile([[1.0], [0], [0], [0]], (1, dyn.size))
    m, q = oracle.shift_fwd(sc, dyn, dpos, drot)
    np.testing.assert_array_equal(m, sc.mean.astype(np.float64))
    qn = sc.quat.astype(np.float64) / np.linalg.norm(sc.quat.astype(np.float64), axis=0)
    np.testing.assert_allclose(q[:, dyn], qn[:, dyn], atol=1e-15)


def test_shift_rotation_composes_like_scipy():
    rng = np.random.default_rng(7)
    sc, _, _ = synth.single_view_scene(1, n=20)
    sc.quat = (sc.quat * rng.uniform(0.5, 2.0, size=(1, 20))).astype(np.float32)  # unnormalised input
    dyn = np.arange(20, dtype=np.int32)
    dpos = rng.normal(0, 0.01, size=(3, 20)); drot = rng.normal(size=(4, 20))
    m, q = oracle.shift_fwd(sc, dyn, dpos, drot)
    for j in range(20):
        a = sc.quat[:, j].astype(np.float64); b = drot[:, j]
        Ra = Rotation.from_quat([a[1], a[2], a[3], a[0]])
        Rb = Rotation.from_quat([b[1], b[2], b[3], b[0]])
        Rq = Rotation.from_quat([q[1, j], q[2, j], q[3, j], q[0, j]])
        np.testing.assert_allclose(Rq.as_matrix(), (Ra * Rb).as_matrix(), atol=1e-12)
        assert np.linalg.norm(q[:, j]) == pytest.approx(1.0, abs=1e-14)
    np.testing.assert_allclose(m, sc.mean.astype(np.float64) + dpos, atol=0)


def test_shift_adjoint_finite_differences():
    rng = np.random.default_rng(11)
    sc, _, _ = synth.single_view_scene(2, n=12)
    dyn = np.array([1, 4, 7, 11], np.int32)
    dpos = rng.normal(0, 0.01, size=(3, 4)); drot = rng.normal(size=(4, 4))
    wm = rng.normal(size=(3, 12)); wq = rng.normal(size=(4, 12))
    ddp, ddr = oracle.shift_adj(sc, dyn, drot, wm, wq)

    def L(dp, dr):
        m, q = oracle.shift_fwd(sc, dyn, dp, dr)
        return float(np.sum(m * wm) + np.sum(q * wq))

    for arr, ana in ((dpos, ddp), (drot, ddr)):
        for idx in np.ndindex(arr.shape):
            x = arr[idx]; h = 1e-6
            arr[idx] = x + h; lp = L(dpos, drot)
            arr[idx] = x - h; lm = L(dpos, drot)
            arr[idx] = x
            assert ana[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-8)


# ------------------------------------------------------------------------------------------
# Adam (textbook, bias-corrected)
# ------------------------------------------------------------------------------------------
def test_adam_matches_torch_over_ten_steps():
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=257)
    grads = [rng.normal(size=257) * 10 ** rng.uniform(-3, 1) for _ in range(10)]
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-15
    t = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad(); t.grad = torch.tensor(g, dtype=torch.float64); opt.step()
        p, m, v = oracle.adam(p, g, m, v, lr, b1, b2, eps, k)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-4, 0.0])
    p, _, _ = oracle.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 0.01, 0.9, 0.999, 1e-15, 1)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-15), rtol=1e-12)


# ------------------------------------------------------------------------------------------
# L1 fidelity term and error map (Eqs. 2/3, Sec. 3.4)
# ------------------------------------------------------------------------------------------
def test_l1_against_torch():
    rng = np.random.default_rng(0)
    r = rng.uniform(size=(3, 3, 9, 11)).astype(np.float32)
    t = rng.uniform(size=(3, 3, 9, 11)).astype(np.float32)
    t[0, 0, 0, 0] = r[0, 0, 0, 0]
    loss, dl, err = oracle.l1_loss_grad(r, t)
    rt = torch.tensor(r, dtype=torch.float64, requires_grad=True)
    lt = torch.nn.functional.l1_loss(rt, torch.tensor(t, dtype=torch.float64))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(dl, rt.grad.numpy(), rtol=1e-12)
    np.testing.assert_allclose(err, np.abs(r.astype(np.float64) - t).mean(1), rtol=1e-12)


# ------------------------------------------------------------------------------------------
# Densification (Sec. 3.4, Alg. 1, Eq. 4)
# ------------------------------------------------------------------------------------------
def test_alg1_golden_fixture():
    rows = np.loadtxt(os.path.join(GOLDEN, "alg1_pixels.txt"), comments="#")
    cam = synth.make_camera(np.diag([1.0, -1.0, -1.0]), (0, 0, 4), 128, 128)
    xy, ok = oracle.alg1(rows[:, 0:3].T, cam)
    for i, row in enumerate(rows):
        assert ok[i] == bool(row[5])
        if ok[i]:
            assert tuple(xy[i]) == (int(row[3]), int(row[4]))


def test_alg1_equals_rounded_pinhole_mean():
    sc, cams, _ = synth.multiview_scene(0, n=3000, n_views=3, width=320, height=240, with_grads=False)
    for cam in cams:
        p = oracle.project(sc, cam)
        xy, ok = oracle.alg1(sc.mean, cam)
        u, v = p.uv[:, 0], p.uv[:, 1]
        inside = (np.floor(u + 0.5) >= 0) & (np.floor(u + 0.5) < cam.width) & (np.floor(v + 0.5) >= 0) & \
                 (np.floor(v + 0.5) < cam.height) & (p.depth > 0)
        far = (np.abs(u - np.floor(u) - 0.5) > 1e-6) & (np.abs(v - np.floor(v) - 0.5) > 1e-6)
        np.testing.assert_array_equal(ok[far], inside[far])
        sel = far & ok
        np.testing.assert_array_equal(xy[sel, 0], np.floor(u[sel] + 0.5).astype(np.int32))
        np.testing.assert_array_equal(xy[sel, 1], np.floor(v[sel] + 0.5).astype(np.int32))


def test_densify_selection_matches_set_definition():
    rng = np.random.default_rng(5)
    sc, cams, _ = synth.multiview_scene(1, n=800, n_views=4, width=64, height=48, with_grads=False)
    errs = [rng.uniform(0, 1, size=(48, 64)).astype(np.float32) for _ in cams]
    gsum = rng.exponential(1.0, size=800).astype(np.float32)
    cnt = rng.integers(0, 5, size=800).astype(np.int32)
    gamma, tp, te = 0.6, 1.5, 0.4
    sel, score, in_err = oracle.densify_select(sc.mean, cams, errs, gsum, cnt, gamma, tp, te)
    # set-level restatement of Eq. (4) from the Alg. 1 pixels
    S_err = set()
    best = np.zeros(800, np.float32)
    for c, cam in enumerate(cams):
        xy, ok = oracle.alg1(sc.mean, cam)
        for g in np.nonzero(ok)[0]:
            e = errs[c][xy[g, 1], xy[g, 0]]
            best[g] = max(best[g], e)
            if e > np.float32(gamma):
                S_err.add(int(g))
    gbar = np.where(cnt > 0, gsum / np.maximum(cnt, 1).astype(np.float32), np.float32(0)).astype(np.float32)
    S_pos = {int(g) for g in range(800) if gbar[g] > np.float32(tp)}
    S_low = {int(g) for g in range(800) if gbar[g] > np.float32(te)}
    S = S_pos | (S_err & S_low)
    assert set(sel.tolist()) == S
    want = sorted(S, key=lambda g: (-best[g], g))
    assert sel.tolist() == want


def test_splitmix64_known_answers():
    for line in open(os.path.join(GOLDEN, "splitmix64_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, i, val = line.split()
        assert oracle.splitmix64(int(seed), int(i)) == int(val, 16)


def _planes(sc, cap):
    def pad(a):
        out = np.zeros(a.shape[:-1] + (cap,), np.float32)
        out[..., :a.shape[-1]] = a
        return out
    return dict(mean=pad(sc.mean), quat=pad(sc.quat), log_scale=pad(sc.log_scale), logit=pad(sc.logit), sh=pad(sc.sh))


def test_spawn_invariants():
    sc, _, _ = synth.single_view_scene(0, n=100)
    cap = 300
    sel = np.array([5, 17, 3], np.int32)
    pl = _planes(sc, cap)
    before = {k: v.copy() for k, v in pl.items()}
    n_app, cm = oracle.spawn(pl, 100, cap, sel, 250, seed=9)
    assert n_app == 200  # capped by capacity
    for k in pl:
        np.testing.assert_array_equal(pl[k][..., :100], before[k][..., :100])
    for j in range(n_app):
        parent, child = sel[j % 3], 100 + j
        np.testing.assert_array_equal(pl["quat"][:, child], pl["quat"][:, parent])
        np.testing.assert_array_equal(pl["sh"][:, child], pl["sh"][:, parent])
        assert pl["logit"][child] == pl["logit"][parent]
        np.testing.assert_allclose(pl["log_scale"][:, child], pl["log_scale"][:, parent] - np.log(1.6), atol=1e-6)
        s = np.exp(pl["log_scale"][:, parent].astype(np.float64))
        assert np.linalg.norm(cm[:, j] - pl["mean"][:, parent]) <= 6 * np.linalg.norm(s) + 1e-9
    pl2 = _planes(sc, cap)
    n2, cm2 = oracle.spawn(pl2, 100, cap, sel, 250, seed=9)
    np.testing.assert_array_equal(cm, cm2)
    assert oracle.spawn(_planes(sc, cap), 100, cap, np.zeros(0, np.int32), 250, seed=9)[0] == 0
    assert oracle.spawn(_planes(sc, cap), 100, cap, sel, 50, seed=9)[0] == 50


def test_child_normals_distribution():
    from scipy import stats
    z = np.array([oracle.child_normals(123, j) for j in range(4000)])
    for k in range(3):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.06


# ---- D-SSIM term of the fidelity loss (Eq. 3) ----------------------------------------------
def test_ssim_window_and_window_sum_brute_force():
    """The window is the normalised 11-tap Gaussian (sigma 1.5) outer product, and the window
    sum is the zero-padded 'same' correlation, checked by explicit loops on a tiny image."""
    w = oracle.ssim_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    g = np.exp(-((np.arange(11) - 5.0) ** 2) / 4.5)
    np.testing.assert_allclose(w, np.outer(g, g) / g.sum() ** 2, rtol=1e-14)
    rng = np.random.default_rng(21)
    img = rng.uniform(size=(9, 7))
    want = np.zeros_like(img)
    H, W = img.shape
    for py in range(H):
        for px in range(W):
            for dy in range(-5, 6):
                for dx in range(-5, 6):
                    qy, qx = py + dy, px + dx
                    if 0 <= qy < H and 0 <= qx < W:
                        want[py, px] += w[dy + 5, dx + 5] * img[qy, qx]
    np.testing.assert_allclose(oracle.ssim_window_sum(img), want, rtol=1e-13, atol=1e-15)


def test_ssim_constant_images_closed_form():
    """Constant images a, b: away from the border the window sees no variance, so the SSIM
    map is the luminance term (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    S = oracle.ssim_terms(np.full((31, 31), a), np.full((31, 31), b))[0]
    want = (2 * a * b + oracle.SSIM_C1) / (a * a + b * b + oracle.SSIM_C1)
    np.testing.assert_allclose(S[5:-5, 5:-5], want, rtol=1e-12)
    assert not np.allclose(S[0, 0], want)  # the zero padding changes the border, as defined


def test_fidelity_loss_identity_symmetry_and_lambda_zero():
    rng = np.random.default_rng(22)
    r = rng.uniform(size=(2, 3, 13, 11))
    t = rng.uniform(size=(2, 3, 13, 11))
    # SSIM(x, x) = 1: no loss, no gradient (a maximum of SSIM, and the L1 kink at 0 has sign 0)
    S = oracle.ssim_terms(r[0, 0], r[0, 0])[0]
    np.testing.assert_allclose(S, 1.0, rtol=1e-13)
    L, dl, err = oracle.fidelity_loss_grad(r, r, 0.4)
    assert abs(L) < 1e-13
    assert np.abs(dl).max() < 1e-13 and np.abs(err).max() == 0.0
    # symmetric in its two images
    assert oracle.fidelity_loss_grad(r, t, 0.4)[0] == pytest.approx(oracle.fidelity_loss_grad(t, r, 0.4)[0], rel=1e-13)
    # lambda = 0 is the L1 term of the C oracle
    L0, dl0, err0 = oracle.fidelity_loss_grad(r.astype(np.float32), t.astype(np.float32), 0.0)
    L1, dl1, err1 = oracle.l1_loss_grad(r.astype(np.float32), t.astype(np.float32))
    assert L0 == pytest.approx(L1, rel=1e-12)
    np.testing.assert_allclose(dl0, dl1, rtol=1e-12, atol=0)
    np.testing.assert_allclose(err0, err1, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_fidelity_gradient_matches_finite_differences(lam):
    rng = np.random.default_rng(23)
    r = rng.uniform(size=(2, 3, 10, 12))
    t = rng.uniform(size=(2, 3, 10, 12))
    _, dl, _ = oracle.fidelity_loss_grad(r, t, lam)
    idx = [tuple(rng.integers(0, s) for s in r.shape) for _ in range(40)]
    checked = 0
    for i in idx:
        if abs(r[i] - t[i]) < 1e-3:  # the L1 kink
            continue
        h = 1e-6
        rp, rm = r.copy(), r.copy()
        rp[i] += h
        rm[i] -= h
        fd = (oracle.fidelity_loss_grad(rp, t, lam)[0] - oracle.fidelity_loss_grad(rm, t, lam)[0]) / (2 * h)
        assert dl[i] == pytest.approx(fd, rel=1e-6, abs=1e-12)
        checked += 1
    assert checked >= 30


# ------------------------------------------------------------------------------------------
# Hash-encoded deformation fields (Sec. 3.3, App. B)
# ------------------------------------------------------------------------------------------
from oracle import hashfield as HF  # noqa: E402


def _field(res, features, log2_table, hidden, seed=0, **kw):
    p = synth.hash_field_params(seed, levels=len(res), features=features, log2_table=log2_table,
                                hidden=hidden, **kw)
    p.res = list(res)
    return HF.from_params(p)


def test_hash_encoding_reproduces_linear_functions_on_dense_levels():
    """Trilinear interpolation is exact for functions linear in the grid coordinates: with
    every dense level's rows set to a.c + b at corner c, the encoding at p is a.(p N_l) + b."""
    f = _field([3, 5, 7], 2, 10, 8)  # (N+1)^3 = 64, 216, 512 <= 1024: all dense
    a = np.array([[0.7, -1.3, 2.1], [-0.4, 0.9, 0.25]])
    b = np.array([0.3, -0.8])
    for l, n in enumerate(f.res):
        g = np.arange(n + 1)
        cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
        c = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], -1)
        f.table[l][:] = 0.0
        f.table[l][HF.corner_index(f, l, c)] = c @ a.T + b
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, size=(50, 3))
    p[0] = 1.0                                   # top corner of the box (the clamped cell)
    p[1] = [0.0, 1.0, 0.5]
    enc = HF.encode(f, p)
    for l, n in enumerate(f.res):
        np.testing.assert_allclose(enc[:, 2 * l:2 * l + 2], (p * n) @ a.T + b, rtol=0, atol=1e-12)


def test_hash_dense_index_is_x_fastest():
    f = _field([3], 1, 8, 4)
    assert HF.corner_index(f, 0, [[1, 0, 0]])[0] == 1
    assert HF.corner_index(f, 0, [[0, 1, 0]])[0] == 4
    assert HF.corner_index(f, 0, [[0, 0, 1]])[0] == 16
    assert HF.corner_index(f, 0, [[3, 3, 3]])[0] == 63


def test_spatial_hash_on_grid_vertices():
    """On a hashed level, a query exactly on a grid vertex reads that vertex's row alone; with
    row r holding the feature r, the encoding returns the hash (x*1 xor y*2654435761 xor
    z*805459861) mod T, whose primes are the published ones of the multi-resolution encoding."""
    T = 1 << 12
    f = _field([100], 1, 12, 4)  # 101^3 > 4096: hashed
    f.table[0][:, 0] = np.arange(T)
    coords = [(37, 0, 0), (0, 1, 0), (0, 0, 1), (0, 2, 0), (5, 7, 11)]
    p = np.array(coords, np.float64) / 100.0
    enc = np.rint(HF.encode(f, p)[:, 0])        # vertex weight 1 up to the rounding of p N
    assert enc[0] == 37                        # prime 1 on x: identity along the x axis
    assert enc[1] == 2654435761 % T           # = 0x9E3779B1 mod 2^12 = 0x9B1
    assert enc[1] == 0x9B1
    assert enc[2] == 805459861 % T            # = 0x30025795 mod 2^12 = 0x795
    assert enc[2] == 0x795
    assert enc[3] == (2 * 2654435761) % T
    assert enc[4] == (5 ^ (7 * 2654435761 % 2**32) ^ (11 * 805459861 % 2**32)) % T


def test_hash_field_identity_and_mlp_closed_form():
    """A zero output layer is the identity shift (dpos 0, drot (1,0,0,0)); with one level, an
    identity first layer and non-negative features, the MLP is the affine map W2 enc + b2."""
    f = _field([4], 4, 10, 4)
    rng = np.random.default_rng(5)
    mean = rng.uniform(-1.4, 1.4, size=(3, 20))
    f.w2[:] = 0.0
    f.b2[:] = 0.0
    dp, dr = HF.field_fwd(f, mean)
    assert np.all(dp == 0.0) and np.all(dr[0] == 1.0) and np.all(dr[1:] == 0.0)
    f.table[:] = np.abs(f.table)
    f.w1[:] = np.eye(4)
    f.b1[:] = 0.0
    f.w2[:] = rng.normal(size=(7, 4))
    f.b2[:] = rng.normal(size=7)
    enc = HF.encode(f, HF.normalised(f, mean))
    dp, dr = HF.field_fwd(f, mean)
    out = enc @ f.w2.T + f.b2
    np.testing.assert_allclose(dp, out[:, :3].T, atol=1e-14)
    np.testing.assert_allclose(dr, out[:, 3:].T + np.array([[1.0], [0], [0], [0]]), atol=1e-14)
    # ReLU: a negative bias beyond every pre-activation leaves only b2
    f.b1[:] = -10.0
    dp, dr = HF.field_fwd(f, mean)
    np.testing.assert_allclose(dp, np.repeat(f.b2[:3, None], 20, 1), atol=0)


def test_hash_field_clamps_to_the_box():
    f = _field([4, 9], 2, 8, 8)
    inside = np.array([[1.5, -0.3, 0.2], [-1.5, 1.5, 0.9]]).T        # on the box faces
    outside = np.array([[4.0, -0.3, 0.2], [-9.0, 7.5, 0.9]]).T
    for a, b in zip(HF.field_fwd(f, inside), HF.field_fwd(f, outside)):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("res,features,log2_table", [([2, 5, 11], 2, 7), ([3, 40], 4, 9)])
def test_hash_field_gradients_match_finite_differences(res, features, log2_table):
    """Every parameter group, dense and hashed levels: central differences of
    <d_dpos, dpos> + <d_drot, drot>."""
    f = _field(res, features, log2_table, 16, seed=2)
    mean, idx, ddp, ddr = synth.field_queries(7, 40, 40)
    mean = mean.astype(np.float64)
    g = HF.field_bwd(f, mean, ddp, ddr)

    def obj():
        a, b = HF.field_fwd(f, mean)
        return float((a * ddp).sum() + (b * ddr).sum())

    rng = np.random.default_rng(1)
    h = 1e-6
    for name in ("table", "w1", "b1", "w2", "b2"):
        arr = getattr(f, name)
        if name == "table":
            used = np.argwhere(np.abs(g["table"]) > 0)
            picks = [tuple(used[i]) for i in rng.choice(len(used), 6, replace=False)]
            picks.append(tuple(np.argwhere(g["table"] == 0)[0]))       # an unused row: zero
        else:
            picks = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
        for ix in picks:
            old = arr[ix]
            arr[ix] = old + h
            fp = obj()
            arr[ix] = old - h
            fm = obj()
            arr[ix] = old
            fd = (fp - fm) / (2 * h)
            assert abs(g[name][ix] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, ix, g[name][ix], fd)


# ------------------------------------------------------------------------------------------
# Selective inheritance (Sec. 3.2, STE of App. B) and pruning of G^var (Sec. 3.4)
# ------------------------------------------------------------------------------------------
from oracle import inherit as INH  # noqa: E402
from scipy.special import expit  # noqa: E402


def test_quant_mask_is_rounding_of_the_sigmoid():
    """Quant(sigmoid(m)) with 1/2 rounding up equals m >= 0 (values where float64 sigmoid is not
    itself rounded to 1/2, |m| > 1e-16, or m = 0)."""
    m = np.concatenate([synth.inheritance_logits(3, 400), [0.0, -0.0, 1e-12, -1e-12, 40.0, -40.0]])
    np.testing.assert_array_equal(INH.quant_mask(m), expit(m.astype(np.float64)) >= 0.5)


def _var_scene(seed, n_base=30, n_var=30, W=40, H=32):
    scene, cams, dls = synth.tiny_scene(seed, n_base + n_var, W, H, log_scale_mu=-2.2)
    scene.n_base = n_base
    return scene, cams, dls


def _eff_scene(scene, lg, ls):
    return synth.Scene(scene.mean.astype(np.float64), scene.quat.astype(np.float64), ls, lg,
                       scene.sh.astype(np.float64), scene.sh_degree, scene.n_base)


def test_masked_gaussians_are_not_drawn():
    """Rendering with the inheritance mask equals rendering without the masked rows."""
    scene, cams, _ = _var_scene(4)
    m = synth.inheritance_logits(5, scene.n - scene.n_base, frac_masked=0.5)
    lg, ls = INH.inherit_planes(scene.logit, scene.log_scale, scene.n_base, m)
    img = oracle.render(_eff_scene(scene, lg, ls), cams)[0].rgb
    keep = INH.keep_rows(scene.logit, scene.n_base, m)
    sub = scene.subset(np.concatenate([np.arange(scene.n_base), scene.n_base + np.nonzero(keep)[0]]))
    ref = oracle.render(sub, cams)[0].rgb
    assert keep.sum() < keep.size
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-12)
    # unmasked rows keep their parameters exactly
    on = scene.n_base + np.nonzero(INH.quant_mask(m))[0]
    np.testing.assert_array_equal(lg[on], scene.logit[on].astype(np.float64))


def test_inheritance_gradient_matches_finite_differences_of_the_mask():
    """The straight-through gradient: for an unmasked Gaussian, dL/dM at M = 1 by central
    differences of the rendered loss with o_r = M o and s_r = M s; masked ones get the mask
    loss only; the mask loss's own value and gradient in closed form."""
    scene, cams, dls = _var_scene(6)
    nv = scene.n - scene.n_base
    m = synth.inheritance_logits(7, nv, frac_masked=0.3)
    lam = 0.05
    lg, ls = INH.inherit_planes(scene.logit, scene.log_scale, scene.n_base, m)
    eff = _eff_scene(scene, lg, ls)
    grads, _, _, _ = oracle.render_backward(eff, cams, dls)
    dm, loss = INH.inherit_grad(scene.logit, scene.n_base, m, grads.logit, grads.log_scale, lam)
    sp = expit(m.astype(np.float64)) * (1 - expit(m.astype(np.float64)))
    assert loss == pytest.approx(lam * expit(m.astype(np.float64)).sum(), rel=1e-14)
    M = INH.quant_mask(m)
    np.testing.assert_allclose(dm[~M], lam * sp[~M], rtol=1e-14)

    def L(i, Mi):
        o = expit(float(scene.logit[i]))
        lg2, ls2 = lg.copy(), ls.copy()
        lg2[i] = np.log(Mi * o / (1.0 - Mi * o))
        ls2[:, i] = scene.log_scale[:, i].astype(np.float64) + np.log(Mi)
        return float((oracle.render(_eff_scene(scene, lg2, ls2), cams)[0].rgb * dls[0]).sum())

    checked = 0
    for j in np.nonzero(M)[0]:
        i = scene.n_base + j
        dM = (dm[j] - lam * sp[j]) / sp[j]
        if abs(dM) < 1e-3:
            continue
        h = 1e-6
        fd = (L(i, 1 + h) - L(i, 1 - h)) / (2 * h)
        assert abs(dM - fd) <= 1e-4 * max(1.0, abs(fd)), (i, dM, fd)
        checked += 1
    assert checked >= 5


def test_compaction_and_pruning_brute_force():
    rng = np.random.default_rng(8)
    n_base, nv = 7, 50
    n = n_base + nv
    planes = {"mean": rng.normal(size=(3, n)), "logit": rng.normal(0, 3, size=n), "sh": rng.normal(size=(12, n))}
    m = synth.inheritance_logits(9, nv)
    for mm, floor in ((m, 0.0), (None, 0.05), (m, 0.05)):
        keep = INH.keep_rows(planes["logit"], n_base, mm, floor)
        want = []
        for j in range(nv):
            ok = True
            if mm is not None:
                ok &= expit(float(mm[j])) >= 0.5
            if floor > 0:
                ok &= expit(planes["logit"][n_base + j]) >= floor
            want.append(ok)
        np.testing.assert_array_equal(keep, want)
        out = INH.compact(planes, n_base, keep)
        rows = list(range(n_base)) + [n_base + j for j in range(nv) if want[j]]
        for k in planes:
            np.testing.assert_array_equal(out[k], planes[k][..., rows])


# ------------------------------------------------------------------------------------------
# Identity-feature rendering and the dynamics mask (Sec. 3.3)
# ------------------------------------------------------------------------------------------
class _FeatProj:
    def __init__(self, p, vals):
        self.uv, self.conic, self.opacity, self.depth, self.rgb = p.uv, p.conic, p.opacity, p.depth, vals


def test_feature_render_equals_brute_force():
    sc, cams, _ = synth.tiny_scene(3, 40, 40, 36, log_scale_mu=-2.2)
    cam = cams[0]
    vr = oracle.render_view(sc, cam)
    p = vr.proj
    feat = np.random.default_rng(4).normal(size=(5, sc.n))
    F = oracle.render_features(vr, cam, feat)
    for py in range(0, 36, 3):
        for px in range(0, 40, 3):
            tx, ty = px // 16, py // 16
            gids = [g for g in range(sc.n) if p.visible[g] and p.rect[g, 0] <= tx < p.rect[g, 2]
                    and p.rect[g, 1] <= ty < p.rect[g, 3]]
            for c0 in (0, 3):
                vals = np.zeros((sc.n, 3))
                k = min(3, 5 - c0)
                vals[:, :k] = feat[c0:c0 + k].T
                want, _, _ = brute_force_pixel(_FeatProj(p, vals), gids, float(px), float(py), (0.0, 0.0, 0.0))
                np.testing.assert_allclose(F[c0:c0 + k, py, px], want[:k], atol=1e-14)


def test_feature_render_of_ones_is_coverage():
    """With every feature 1 the image is sum_i alpha_i T_i = 1 - T_final."""
    sc, cams, _ = synth.tiny_scene(5, 60, 48, 40, log_scale_mu=-2.0)
    vr = oracle.render_view(sc, cams[0])
    F = oracle.render_features(vr, cams[0], np.ones((4, sc.n)))
    for c in range(4):
        np.testing.assert_allclose(F[c], 1.0 - vr.t_final, atol=1e-13)


def test_dynamic_gaussians_brute_force():
    rng = np.random.default_rng(6)
    K, Cn, n = 6, 5, 300
    cls_w, cls_b = rng.normal(size=(K, Cn)), rng.normal(size=K)
    feat = rng.normal(size=(Cn, n))
    imgs = [rng.normal(size=(Cn, 7, 9)) for _ in range(2)]
    flows = [rng.uniform(0, 1, size=(7, 9)) for _ in range(2)]
    dyn_obj, idx = oracle.dynamic_gaussians(imgs, flows, 0.8, cls_w, cls_b, feat)
    want_obj = np.zeros(K, bool)
    for F, fl in zip(imgs, flows):
        for y in range(7):
            for x in range(9):
                if fl[y, x] > 0.8:
                    s = [float(cls_w[k] @ F[:, y, x] + cls_b[k]) for k in range(K)]
                    want_obj[max(range(K), key=lambda k: (s[k], -k))] = True
    np.testing.assert_array_equal(dyn_obj, want_obj)
    want_idx = [g for g in range(n) if want_obj[max(range(K), key=lambda k: (float(cls_w[k] @ feat[:, g] + cls_b[k]), -k))]]
    np.testing.assert_array_equal(idx, want_idx)


def test_hash_field_weight_orientation():
    """w1[h][k] maps feature k to hidden unit h and w2[o][h] hidden unit h to output o: with a
    single 1 at w1[5][2] and w2[1][5], the y offset is the ReLU of encoding feature 2 and every
    other output is zero (a misread index would take another feature or write another output)."""
    f = _field([6], 4, 10, 8)
    f.table[:] = np.abs(f.table) + 0.1
    f.w1[:] = 0.0
    f.w1[5, 2] = 1.0
    f.b1[:] = 0.0
    f.w2[:] = 0.0
    f.w2[1, 5] = 1.0
    f.b2[:] = 0.0
    mean = np.random.default_rng(12).uniform(-1.4, 1.4, size=(3, 30))
    enc = HF.encode(f, HF.normalised(f, mean))
    dp, dr = HF.field_fwd(f, mean)
    np.testing.assert_allclose(dp[1], enc[:, 2], rtol=0, atol=1e-15)
    assert np.all(dp[0] == 0) and np.all(dp[2] == 0) and np.all(dr[1:] == 0) and np.all(dr[0] == 1)
    assert np.abs(enc[:, 2] - enc[:, 1]).max() > 1e-3  # features differ, so a wrong index shows

"""Helpers shared by the GPU parity tests (HIP path through the C ABI vs the CPU oracle)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

IMG_TOL = 1e-4           # images: absolute, float32 path vs float64 definition
GRAD_REL, GRAD_ABS = 1e-3, 1e-4  # |g - o| <= GRAD_REL |o| + GRAD_ABS max|o|, per tensor


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(scene, capacity=None, n_base=None):
    from paper_2411_14847_amd import GaussianBuffers
    return GaussianBuffers.from_arrays(scene.mean, scene.quat, scene.log_scale, scene.logit, scene.sh,
                                       scene.sh_degree, capacity=capacity, n_base=n_base)


def make_ctx(n, cams, keys_per_gaussian=64, extra_keys=1 << 16):
    from paper_2411_14847_amd import Context
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    return Context(max_gaussians=max(n, 1), max_views=len(cams),
                   max_keys=int(max(n, 1) * len(cams) * keys_per_gaussian + extra_keys), max_tiles=tiles)


def tile_pixel_mask(cam, tiles, tile=16):
    TX = (cam.width + tile - 1) // tile
    m = np.zeros((cam.height, cam.width), bool)
    for t in tiles:
        tx, ty = int(t) % TX, int(t) // TX
        m[ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile] = True
    return m


def radius_flag_pixels(proj, cam, tile=(16, 16)):
    """Pixels of tiles on or next to the rectangle of a Gaussian whose radius sits within rounding
    of an integer (its rectangle may differ by one tile between float64 implementations)."""
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    TX = (cam.width + tw - 1) // tw
    TY = (cam.height + th - 1) // th
    m = np.zeros((cam.height, cam.width), bool)
    for g in np.nonzero(proj.flags & oracle.FLAG_RADIUS)[0]:
        x0, y0, x1, y1 = proj.rect[g]
        if not proj.visible[g]:
            continue
        xs = slice(max(0, x0 - 1) * tw, min(TX, x1 + 1) * tw)
        ys = slice(max(0, y0 - 1) * th, min(TY, y1 + 1) * th)
        m[ys, xs] = True
    return m


def excluded_pixels(vr, cam, grad=False, tile=(16, 16)):
    flags = oracle.PIXEL_GRAD_FLAGS if grad else oracle.PIXEL_VALUE_FLAGS
    return ((vr.flags & flags) != 0) | radius_flag_pixels(vr.proj, cam, tile)


def assert_grad_close(name, got, want, exclude=None):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    if exclude is not None:
        got = got[..., ~exclude]
        want = want[..., ~exclude]
    if want.size == 0:
        return 0.0
    scale = np.abs(want).max()
    err = np.abs(got - want)
    bound = GRAD_REL * np.abs(want) + GRAD_ABS * scale
    bad = err > bound
    big = np.abs(want) >= 1e-2 * scale
    rel = (err[big] / np.abs(want[big])).max() if big.any() else 0.0
    assert not bad.any(), (f"{name}: {bad.sum()} of {bad.size} elements outside tolerance; worst err "
                           f"{err.max():.3e} (scale {scale:.3e}); max rel on significant {rel:.3e}")
    return rel

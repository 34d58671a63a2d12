"""CPU oracle for the DASS hot path -- TEST INFRASTRUCTURE, not part of the product.

A plain double-precision definition (``dass_oracle.c``) of what the GPU path
computes, driven from NumPy.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP path and imports nothing from the product package.

Inputs are the float32 arrays of :mod:`synth` (scenes, cameras, upstream
gradients); every computation is in float64 unless a float decides an integer
(the float32 depth bits of a tile key, the float32 historical-gradient and
error thresholds of Eq. (4)), where the float32 value is used, as the kernel
does.  Each function names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dass_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FLAG_RADIUS, FLAG_CLIP, FLAG_RGB, FLAG_SKIP, FLAG_STOP, FLAG_PSIGN, FLAG_CLAMP = 1, 2, 4, 8, 16, 32, 64
GAUSS_GRAD_FLAGS = FLAG_RADIUS | FLAG_CLIP | FLAG_RGB
PIXEL_VALUE_FLAGS = FLAG_SKIP | FLAG_STOP | FLAG_PSIGN
PIXEL_GRAD_FLAGS = PIXEL_VALUE_FLAGS | FLAG_CLAMP


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Cam(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("campos", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32)]


def cam_struct(cam) -> Cam:
    c = Cam()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(-1)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32)]
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.campos[:] = [float(x) for x in np.asarray(cam.campos, np.float32)]
    c.width, c.height = int(cam.width), int(cam.height)
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.orc_count_keys.restype = C.c_int64
        _lib.orc_l1.restype = C.c_double
        _lib.orc_densify_select.restype = C.c_int32
        _lib.orc_spawn.restype = C.c_int32
        _lib.orc_splitmix64.restype = C.c_uint64
        _lib.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def tiles_of(cam, tile):
    tw, th = tile
    return (cam.width + tw - 1) // tw, (cam.height + th - 1) // th


# ------------------------------------------------------------------------------------------
# Projection (App. A.1)
# ------------------------------------------------------------------------------------------
@dataclass
class Projection:
    uv: np.ndarray
    conic: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray
    depth: np.ndarray
    radius: np.ndarray
    rect: np.ndarray
    depth_bits: np.ndarray
    visible: np.ndarray
    flags: np.ndarray


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _scene_arrays(scene):
    """Parameter planes widened to float64 (exact for float32 inputs)."""
    return (_f64(scene.mean), _f64(scene.quat), _f64(scene.log_scale), _f64(scene.logit), _f64(scene.sh))


def project(scene, cam, tile=(16, 16)) -> Projection:
    n = scene.n
    mean, quat, ls, lg, sh = _scene_arrays(scene)
    uv = np.zeros((n, 2)); conic = np.zeros((n, 3)); op = np.zeros(n); rgb = np.zeros((n, 3))
    depth = np.zeros(n); radius = np.zeros(n, np.int32); rect = np.zeros((n, 4), np.int32)
    dbits = np.zeros(n, np.uint32); vis = np.zeros(n, np.int32); flags = np.zeros(n, np.int32)
    cs = cam_struct(cam)
    lib().orc_project(C.c_int32(n), _p(mean), _p(quat), _p(ls), _p(lg), _p(sh), C.c_int32(scene.sh_degree),
                      C.c_int64(n), C.byref(cs), C.c_int32(tile[0]), C.c_int32(tile[1]), _p(uv), _p(conic),
                      _p(op), _p(rgb), _p(depth), _p(radius), _p(rect), _p(dbits), _p(vis), _p(flags))
    return Projection(uv, conic, op, rgb, depth, radius, rect, dbits, vis.astype(bool), flags)


# ------------------------------------------------------------------------------------------
# Keys, sort, ranges ("tile-based" rasterization, Sec. 1 / Sec. 4.2)
# ------------------------------------------------------------------------------------------
def keys(proj: Projection, cam, tile=(16, 16)):
    """Returns (sorted keys uint64, sorted values uint32, ranges int64 [tiles,2])."""
    n = proj.uv.shape[0]
    TX, TY = tiles_of(cam, tile)
    vis = proj.visible.astype(np.int32)
    rect = np.ascontiguousarray(proj.rect, np.int32)
    cnt = lib().orc_count_keys(C.c_int32(n), _p(rect), _p(vis))
    k = np.zeros(cnt, np.uint64)
    v = np.zeros(cnt, np.uint32)
    lib().orc_emit_keys(C.c_int32(n), _p(rect), _p(vis), _p(np.ascontiguousarray(proj.depth_bits)),
                        C.c_int32(TX), _p(k), _p(v))
    lib().orc_sort_pairs(C.c_int64(cnt), _p(k), _p(v))
    ranges = np.zeros((TX * TY, 2), np.int64)
    lib().orc_ranges(C.c_int64(cnt), _p(k), C.c_int32(TX * TY), _p(ranges))
    return k, v, ranges


# ------------------------------------------------------------------------------------------
# Blend (App. A.1) and its adjoint
# ------------------------------------------------------------------------------------------
@dataclass
class ViewRender:
    rgb: np.ndarray        # (3,H,W) float64
    t_final: np.ndarray    # (H,W)
    n_contrib: np.ndarray  # (H,W) int32
    flags: np.ndarray      # (H,W) int32 decision-margin flags
    signature: np.ndarray  # (H,W) uint64 hash of each pixel's blended entries (decision trace)
    computed: np.ndarray   # (H,W) bool, pixels covered by the tile list
    proj: Projection
    keys: np.ndarray
    vals: np.ndarray
    ranges: np.ndarray


def _tile_arr(tiles):
    if tiles is None:
        return 0, None
    t = np.ascontiguousarray(np.asarray(tiles, np.int32))
    return int(t.size), t


def render_view(scene, cam, bg=(0.0, 0.0, 0.0), tile=(16, 16), tiles=None, proj=None,
                key_data=None) -> ViewRender:
    proj = proj if proj is not None else project(scene, cam, tile)
    k, v, ranges = key_data if key_data is not None else keys(proj, cam, tile)
    W, H = cam.width, cam.height
    out = np.zeros((3, H, W)); T = np.ones((H, W)); nc = np.zeros((H, W), np.int32)
    fl = np.zeros((H, W), np.int32)
    sig = np.zeros((H, W), np.uint64)
    nl, tl = _tile_arr(tiles)
    bgd = np.asarray(bg, np.float64)
    lib().orc_blend_fwd(C.c_int32(W), C.c_int32(H), C.c_int32(tile[0]), C.c_int32(tile[1]), _p(ranges), _p(v),
                        _p(proj.uv), _p(proj.conic), _p(proj.opacity), _p(proj.rgb), _p(bgd), C.c_int32(nl),
                        _p(tl) if tl is not None else None, _p(out), _p(T), _p(nc), _p(fl), _p(sig))
    computed = np.zeros((H, W), bool)
    TX, TY = tiles_of(cam, tile)
    for t in (range(TX * TY) if tiles is None else tiles):
        tx, ty = int(t) % TX, int(t) // TX
        computed[ty * tile[1]:(ty + 1) * tile[1], tx * tile[0]:(tx + 1) * tile[0]] = True
    return ViewRender(out, T, nc, fl, sig, computed, proj, k, v, ranges)


@dataclass
class Grads:
    mean: np.ndarray
    quat: np.ndarray
    log_scale: np.ndarray
    logit: np.ndarray
    sh: np.ndarray

    @staticmethod
    def zeros(n, sh_planes):
        return Grads(np.zeros((3, n)), np.zeros((4, n)), np.zeros((3, n)), np.zeros(n), np.zeros((sh_planes, n)))


def blend_backward(vr: ViewRender, cam, dl, bg=(0.0, 0.0, 0.0), tile=(16, 16), tiles=None):
    """Per-Gaussian 2D gradients g2d[n][9] = (du,dv,dA,dB,dC,do,dr,dg,db) of one view."""
    n = vr.proj.uv.shape[0]
    g2d = np.zeros((n, 9))
    nl, tl = _tile_arr(tiles)
    bgd = np.asarray(bg, np.float64)
    p = vr.proj
    lib().orc_blend_bwd(C.c_int32(cam.width), C.c_int32(cam.height), C.c_int32(tile[0]), C.c_int32(tile[1]),
                        _p(vr.ranges), _p(vr.vals), _p(p.uv), _p(p.conic), _p(p.opacity), _p(p.rgb), _p(bgd),
                        _p(_f32(dl)), C.c_int32(nl), _p(tl) if tl is not None else None, _p(g2d))
    return g2d


def project_backward(scene, cam, g2d, grads: Grads, gradnorm, count, tile=(16, 16), only=None):
    n = scene.n
    mean, quat, ls, lg, sh = _scene_arrays(scene)
    onl = None if only is None else np.ascontiguousarray(only, np.int32)
    cs = cam_struct(cam)
    lib().orc_project_bwd(C.c_int32(n), _p(mean), _p(quat), _p(ls), _p(lg), _p(sh), C.c_int32(scene.sh_degree),
                          C.c_int64(n), C.byref(cs), C.c_int32(tile[0]), C.c_int32(tile[1]),
                          _p(np.ascontiguousarray(g2d)), _p(onl) if onl is not None else None,
                          _p(grads.mean), _p(grads.quat), _p(grads.log_scale), _p(grads.logit), _p(grads.sh),
                          _p(gradnorm), _p(count))


def render(scene, cams, bg=(0.0, 0.0, 0.0), tile=(16, 16), tiles=None):
    return [render_view(scene, c, bg, tile, None if tiles is None else tiles[i]) for i, c in enumerate(cams)]


def render_backward(scene, cams, dls, bg=(0.0, 0.0, 0.0), tile=(16, 16), renders=None, tiles=None, only=None):
    """Gradients of sum_v <dl_v, render_v> w.r.t. all parameters, summed over views.

    Returns (Grads, [g2d per view], gradnorm_sum, count)."""
    n = scene.n
    renders = renders if renders is not None else render(scene, cams, bg, tile, tiles)
    grads = Grads.zeros(n, scene.sh.shape[0])
    gn = np.zeros(n)
    cnt = np.zeros(n, np.int32)
    g2ds = []
    for i, (cam, dl, vr) in enumerate(zip(cams, dls, renders)):
        g2d = blend_backward(vr, cam, dl, bg, tile, None if tiles is None else tiles[i])
        g2ds.append(g2d)
        project_backward(scene, cam, g2d, grads, gn, cnt, tile, only)
    return grads, g2ds, gn, cnt


# ------------------------------------------------------------------------------------------
# Shift (Sec. 3.3), Adam, L1 (Eqs. 2/3), densification (Sec. 3.4, Alg. 1, Eq. 4)
# ------------------------------------------------------------------------------------------
def shift_fwd(scene, dyn_idx, dpos, drot):
    n = scene.n
    om = np.zeros((3, n)); oq = np.zeros((4, n))
    di = np.ascontiguousarray(dyn_idx, np.int32)
    lib().orc_shift_fwd(C.c_int32(n), C.c_int64(n), _p(_f64(scene.mean)), _p(_f64(scene.quat)),
                        C.c_int32(di.size), _p(di), _p(_f64(dpos)), _p(_f64(drot)), _p(om), _p(oq))
    return om, oq


def shift_adj(scene, dyn_idx, drot, dmean, dquat):
    n = scene.n
    di = np.ascontiguousarray(dyn_idx, np.int32)
    ddp = np.zeros((3, di.size)); ddr = np.zeros((4, di.size))
    lib().orc_shift_adj(C.c_int32(n), C.c_int64(n), _p(_f64(scene.quat)), C.c_int32(di.size), _p(di),
                        _p(_f64(drot)), _p(np.ascontiguousarray(dmean, np.float64)),
                        _p(np.ascontiguousarray(dquat, np.float64)), _p(ddp), _p(ddr))
    return ddp, ddr


def adam(p, g, m, v, lr, beta1, beta2, eps, step):
    p = np.array(p, np.float64, copy=True); m = np.array(m, np.float64, copy=True)
    v = np.array(v, np.float64, copy=True); g = np.ascontiguousarray(g, np.float64)
    lib().orc_adam(C.c_int64(p.size), _p(p), _p(g), _p(m), _p(v), C.c_double(lr), C.c_double(beta1),
                   C.c_double(beta2), C.c_double(eps), C.c_int32(step))
    return p, m, v


def l1_loss_grad(renders, targets):
    """renders/targets: (V,3,H,W) float32.  Returns (loss, dl (V,3,H,W), err (V,H,W))."""
    r = _f32(renders); t = _f32(targets)
    V, _, H, W = r.shape
    dl = np.zeros(r.shape); err = np.zeros((V, H, W))
    loss = lib().orc_l1(C.c_int32(V), C.c_int64(H * W), _p(r), _p(t), _p(dl), _p(err))
    return loss, dl, err


# ---- D-SSIM term of the fidelity loss (Eq. 3) ----------------------------------------------
# Readings (the paper names "the fidelity loss in the vanilla 3DGS": L1 plus D-SSIM): single-scale
# SSIM with an 11x11 Gaussian window (sigma 1.5, weights normalised to sum 1), images in [0, 1]
# so C1 = 0.01^2 and C2 = 0.03^2, window sums with zero padding ("same" size), the SSIM map
# averaged over the three channels and all pixels, D-SSIM = 1 - SSIM.
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window() -> np.ndarray:
    """The 11x11 window: outer product of the normalised 1-D Gaussian (sigma 1.5)."""
    k = np.arange(11, dtype=np.float64) - 5.0
    g = np.exp(-(k * k) / (2.0 * 1.5 * 1.5))
    g /= g.sum()
    return np.outer(g, g)


def ssim_window_sum(img) -> np.ndarray:
    """sum_q w(q - p) img(q) at every pixel p of an (H, W) image, zero outside it."""
    from scipy.ndimage import correlate
    return correlate(np.asarray(img, np.float64), ssim_window(), mode="constant", cval=0.0)


def ssim_terms(x, y):
    """SSIM map of two (H, W) images and its partial derivatives with respect to the window
    moments mu_x = w*x, E_xx = w*(x^2), E_xy = w*(x y) (the others held fixed)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = ssim_window_sum(x), ssim_window_sum(y)
    exx, eyy, exy = ssim_window_sum(x * x), ssim_window_sum(y * y), ssim_window_sum(x * y)
    A = 2.0 * mx * my + SSIM_C1               # luminance numerator
    B = 2.0 * (exy - mx * my) + SSIM_C2       # 2 sigma_xy + C2
    Cc = mx * mx + my * my + SSIM_C1          # luminance denominator
    D = (exx - mx * mx) + (eyy - my * my) + SSIM_C2  # sigma_x^2 + sigma_y^2 + C2
    S = (A * B) / (Cc * D)
    dS_dmx = (2.0 * my * B - 2.0 * my * A) / (Cc * D) - S * (2.0 * mx / Cc - 2.0 * mx / D)
    dS_dexx = -S / D
    dS_dexy = 2.0 * A / (Cc * D)
    return S, dS_dmx, dS_dexx, dS_dexy


def fidelity_loss_grad(renders, targets, lam: float):
    """Eq. (3) fidelity term over V views: L = (1/V) sum_v [(1 - lam) mean|r - t| + lam (1 -
    mean SSIM(r, t))], means over channels and pixels.  renders/targets (V,3,H,W).  Returns
    (L, dL/drender (V,3,H,W), error map (V,H,W) = mean over channels of |r - t|)."""
    r = np.asarray(renders, np.float64)
    t = np.asarray(targets, np.float64)
    V, _, H, W = r.shape
    n = 3.0 * H * W
    loss = 0.0
    dl = np.zeros(r.shape)
    err = np.zeros((V, H, W))
    for v in range(V):
        loss += lam / V  # the 1 of 1 - SSIM
        for c in range(3):
            x, y = r[v, c], t[v, c]
            d = x - y
            S, dmx, dexx, dexy = ssim_terms(x, y)
            loss += ((1.0 - lam) * np.abs(d).sum() / n - lam * S.sum() / n) / V
            # adjoint of the window sums: the window is symmetric, so it is the same sum
            gS = -lam / (n * V)
            dssim = ssim_window_sum(gS * dmx) + 2.0 * x * ssim_window_sum(gS * dexx) + \
                y * ssim_window_sum(gS * dexy)
            dl[v, c] = (1.0 - lam) * np.sign(d) / (n * V) + dssim
            err[v] += np.abs(d) / 3.0
    return loss, dl, err


def _cams_array(cams):
    arr = (Cam * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = cam_struct(c)
    return arr


def alg1(mean, cam):
    """Alg. 1 pixel of each column of mean (3,N); returns (xy int32 (N,2), ok bool)."""
    m = _f64(mean)
    n = m.shape[1]
    xy = np.zeros((n, 2), np.int32); ok = np.zeros(n, np.int32)
    cs = cam_struct(cam)
    lib().orc_alg1(C.c_int32(n), C.c_int64(n), _p(m), C.byref(cs), _p(xy), _p(ok))
    return xy, ok.astype(bool)


def densify_select(mean_base, cams, err_maps, gradnorm_sum, grad_count, gamma_err, tau_pos, tau_err):
    """Eq. (4) set S ranked by (max error at the Alg. 1 pixel desc, index asc)."""
    m = _f64(mean_base)
    n = m.shape[1]
    err = np.concatenate([_f32(e).reshape(-1) for e in err_maps])
    sel = np.zeros(max(n, 1), np.int32); score = np.zeros(max(n, 1), np.float32)
    in_err = np.zeros(max(n, 1), np.int32)
    ca = _cams_array(cams)
    ns = lib().orc_densify_select(C.c_int32(n), C.c_int64(n), _p(m), C.c_int32(len(cams)), ca, _p(err),
                                  _p(_f32(gradnorm_sum)), _p(np.ascontiguousarray(grad_count, np.int32)),
                                  C.c_float(gamma_err), C.c_float(tau_pos), C.c_float(tau_err),
                                  _p(sel), _p(score), _p(in_err))
    return sel[:ns].copy(), score[:n], in_err[:n].astype(bool)


def spawn(planes: dict, n: int, capacity: int, sel, k_max: int, seed: int):
    """planes: dict of float32 arrays with capacity columns (mean(3,cap), quat(4,cap), log_scale(3,cap),
    logit(cap), sh(P,cap)), modified in place.  Returns (n_app, child_mean float64 (3,n_app))."""
    sel = np.ascontiguousarray(sel, np.int32)
    sh = planes["sh"]
    cm = np.zeros((3, max(k_max, 1)))
    n_app = lib().orc_spawn(C.c_int32(n), C.c_int32(capacity), C.c_int64(capacity), _p(planes["mean"]),
                            _p(planes["quat"]), _p(planes["log_scale"]), _p(planes["logit"]), _p(sh),
                            C.c_int32(sh.shape[0]), _p(sel), C.c_int32(sel.size), C.c_int32(k_max),
                            C.c_uint64(seed), _p(cm))
    return n_app, cm[:, :n_app] if n_app > 0 else np.zeros((3, 0))


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed), C.c_uint64(i)))


def child_normals(seed: int, j: int):
    z = np.zeros(3)
    lib().orc_child_normals(C.c_uint64(seed), C.c_int64(j), _p(z))
    return z


def sh_eval(deg, dirs):
    d = np.ascontiguousarray(dirs, np.float64)
    K = (deg + 1) ** 2
    out = np.zeros((d.shape[0], K))
    lib().orc_sh_eval(C.c_int32(deg), C.c_int32(d.shape[0]), _p(d), _p(out))
    return out


# hash-encoded deformation fields (Sec. 3.3, App. B)
from .hashfield import Field as HashField, field_bwd as hash_field_bwd, field_fwd as hash_field_fwd  # noqa: E402

# selective inheritance and pruning of G^var (Sec. 3.2, App. B, Sec. 3.4)
from . import inherit  # noqa: E402,F401


# ------------------------------------------------------------------------------------------
# Identity-feature rendering and the 3D half of the dynamics mask (Sec. 3.3; the Gaussian
# Grouping identity encodings of App. A)
# ------------------------------------------------------------------------------------------
def render_features(vr: "ViewRender", cam, feat, tile=(16, 16), tiles=None):
    """C-channel image F_c(p) = sum_i e_{i,c} alpha_i T_i of one view: the blend of the colour
    render (same lists, same alpha and transmittance) with the Gaussians' identity features
    feat (C, n) in place of their colours and no background.  The blend is linear in the
    per-Gaussian values, so the colour blend is run on three channels at a time."""
    feat = np.asarray(feat, np.float64)
    Cn, n = feat.shape
    W, H = cam.width, cam.height
    out = np.zeros((Cn, H, W))
    zero_bg = np.zeros(3)
    p = vr.proj
    nl, tl = _tile_arr(tiles)
    for c0 in range(0, Cn, 3):
        k = min(3, Cn - c0)
        vals3 = np.zeros((n, 3))
        vals3[:, :k] = feat[c0:c0 + k].T
        img = np.zeros((3, H, W)); T = np.ones((H, W)); nc = np.zeros((H, W), np.int32)
        fl = np.zeros((H, W), np.int32)
        lib().orc_blend_fwd(C.c_int32(W), C.c_int32(H), C.c_int32(tile[0]), C.c_int32(tile[1]), _p(vr.ranges),
                            _p(vr.vals), _p(p.uv), _p(p.conic), _p(p.opacity), _p(np.ascontiguousarray(vals3)),
                            _p(zero_bg), C.c_int32(nl), _p(tl) if tl is not None else None, _p(img), _p(T), _p(nc),
                            _p(fl), None)
        out[c0:c0 + k] = img[:k]
    return out


def object_ids(cls_w, cls_b, x):
    """Gaussian Grouping's classification of identity features x (C, m): argmax_k of
    cls_w x + cls_b (first index on ties)."""
    logits = np.asarray(cls_w, np.float64) @ np.asarray(x, np.float64) + np.asarray(cls_b, np.float64)[:, None]
    return np.argmax(logits, axis=0)


def dynamic_gaussians(feat_imgs, flows, gamma_op, cls_w, cls_b, feat):
    """Sec. 3.3: pixels whose optical flow exceeds gamma_op are dynamic areas; the objects the
    rendered segmentation shows there are the dynamic objects; the dynamic Gaussians are those
    whose own identity is a dynamic object.  Returns (dynamic object flags (K,), sorted
    Gaussian indices)."""
    K = np.asarray(cls_w).shape[0]
    dyn_obj = np.zeros(K, bool)
    for F, fl in zip(feat_imgs, flows):
        Cn = F.shape[0]
        sel = np.asarray(fl, np.float64).reshape(-1) > gamma_op
        ids = object_ids(cls_w, cls_b, np.asarray(F, np.float64).reshape(Cn, -1)[:, sel])
        dyn_obj[ids] = True
    gid = object_ids(cls_w, cls_b, feat)
    return dyn_obj, np.nonzero(dyn_obj[gid])[0].astype(np.int32)

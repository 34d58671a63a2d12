"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws random
Gaussians, places pinhole cameras and draws upstream gradients, with NumPy's
PCG64 generator and a fixed draw order (means, log-scales, quaternions,
opacity logits, colour coefficients, then upstream gradients).  The same
float32 bytes feed both the CPU oracle and the HIP path.

The paper's workloads are multi-view video datasets (N3DV: 18-21 views at
1352x1014; MeetRoom: 13 views at 1280x720, Sec. 4.1).  No dataset is used:
these scenes stand in for them with the same view counts, resolutions and a
small per-timestep motion (most offsets below 0.01, Sec. 3.3 / Fig. 3).

Conventions: camera frame x right, y down, z forward; R and t map world to
camera (x_cam = R x_world + t); principal point at the image centre
((W-1)/2, (H-1)/2); 60 degree horizontal field of view with fy = fx.
Colour coefficients are stored as planes sh[k*3 + c] (basis index k,
channel c); the degree-0 basis value is 1/(2 sqrt(pi)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Y00 = 0.28209479177387814  # 1 / (2 sqrt(pi)); converts an RGB colour to the degree-0 coefficient


def n_sh_coeffs(degree: int) -> int:
    return (degree + 1) * (degree + 1)


@dataclass
class Camera:
    R: np.ndarray        # (3,3) float32, world -> camera rotation
    t: np.ndarray        # (3,)  float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    campos: np.ndarray   # (3,) float32, camera centre in world space

    def as_dict(self):
        return dict(R=self.R, t=self.t, fx=self.fx, fy=self.fy, cx=self.cx, cy=self.cy,
                    width=self.width, height=self.height, campos=self.campos)


@dataclass
class Scene:
    mean: np.ndarray       # (3,N) float32
    quat: np.ndarray       # (4,N) float32, (w,x,y,z), not normalised
    log_scale: np.ndarray  # (3,N) float32
    logit: np.ndarray      # (N,)  float32, opacity = sigmoid(logit)
    sh: np.ndarray         # (3*K,N) float32, plane k*3+c
    sh_degree: int
    n_base: int = -1

    def __post_init__(self):
        if self.n_base < 0:
            self.n_base = self.n

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[:, idx].copy(), self.quat[:, idx].copy(), self.log_scale[:, idx].copy(),
                     self.logit[idx].copy(), self.sh[:, idx].copy(), self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.mean.copy(), self.quat.copy(), self.log_scale.copy(), self.logit.copy(),
                     self.sh.copy(), self.sh_degree, self.n_base)


def focal_from_fov(width: int, fov_deg: float = 60.0) -> float:
    return width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))


def look_at(campos, target, up=(0.0, 1.0, 0.0)):
    """World->camera rotation for a camera at campos looking at target (x right, y down, z forward)."""
    campos = np.asarray(campos, np.float64)
    f = np.asarray(target, np.float64) - campos
    f /= np.linalg.norm(f)
    right = np.cross(f, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f])


def make_camera(R, campos, width, height, fov_deg=60.0) -> Camera:
    R = np.asarray(R, np.float64)
    campos = np.asarray(campos, np.float64)
    t = -R @ campos
    f = focal_from_fov(width, fov_deg)
    R32 = R.astype(np.float32)
    t32 = t.astype(np.float32)
    # campos recomputed from the stored float32 R and t so both agree to float32 rounding
    cpos = (-(R32.astype(np.float64).T @ t32.astype(np.float64))).astype(np.float32)
    return Camera(R32, t32, float(np.float32(f)), float(np.float32(f)),
                  float((width - 1) / 2.0), float((height - 1) / 2.0), int(width), int(height), cpos)


def _colour_coeffs(rng, n, degree, hi_std):
    K = n_sh_coeffs(degree)
    sh = np.zeros((3 * K, n), np.float32)
    colours = rng.uniform(0.0, 1.0, size=(3, n))
    sh[0:3] = ((colours - 0.5) / Y00).astype(np.float32)
    if degree > 0:
        sh[3:] = rng.normal(0.0, hi_std, size=(3 * (K - 1), n)).astype(np.float32)
    return sh


def _quats(rng, n):
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


# --------------------------------------------------------------------------------------------
# Workload 1: plain single view, 2,000 Gaussians, SH degree 0, 128x128, 16x16 tiles
# --------------------------------------------------------------------------------------------
def single_view_scene(seed: int = 0, n: int = 2000, width: int = 128, height: int = 128):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, size=(3, n)).astype(np.float32)
    log_scale = rng.normal(-3.5, 0.3, size=(3, n)).astype(np.float32)
    quat = _quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    sh = _colour_coeffs(rng, n, 0, 0.0)
    scene = Scene(mean, quat, log_scale, logit, sh, 0)
    cam = make_camera(np.diag([1.0, -1.0, -1.0]), (0.0, 0.0, 4.0), width, height)
    dl = rng.normal(0.0, 1.0, size=(3, height, width)).astype(np.float32)
    return scene, [cam], [dl]


# --------------------------------------------------------------------------------------------
# Workload 2: multi-view batch, 200,000 Gaussians, SH degree 3, 20 views at 1352x1014
# --------------------------------------------------------------------------------------------
def rig_positions(rows=4, cols=5, spacing=0.1, centre=(0.0, 0.0, 0.0)):
    out = []
    for j in range(rows):
        for i in range(cols):
            out.append((centre[0] + (i - (cols - 1) / 2.0) * spacing,
                        centre[1] + (j - (rows - 1) / 2.0) * spacing,
                        centre[2]))
    return out


def frustum_scene(seed: int, n: int, sh_degree: int, log_scale_mu: float, log_scale_sd: float,
                  box: bool = False, rng=None):
    rng = rng if rng is not None else np.random.default_rng(seed)
    z = rng.uniform(2.0, 10.0, size=n)
    lat = rng.uniform(-4.0, 4.0, size=(2, n))
    if not box:
        lat = lat * (z / 10.0)
    mean = np.stack([lat[0], lat[1], z]).astype(np.float32)
    log_scale = rng.normal(log_scale_mu, log_scale_sd, size=(3, n)).astype(np.float32)
    quat = _quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    sh = _colour_coeffs(rng, n, sh_degree, 0.2)
    return Scene(mean, quat, log_scale, logit, sh, sh_degree), rng


def multiview_rig(width=1352, height=1014, rows=4, cols=5, spacing=0.1):
    return [make_camera(np.eye(3), p, width, height) for p in rig_positions(rows, cols, spacing)]


def multiview_scene(seed: int = 0, n: int = 200_000, n_views: int = 20, width: int = 1352,
                    height: int = 1014, with_grads: bool = True, box: bool = False):
    scene, rng = frustum_scene(seed, n, 3, -4.0, 0.5, box=box)
    cams = multiview_rig(width, height)[:n_views]
    dls = None
    if with_grads:
        dls = [rng.normal(0.0, 1.0, size=(3, height, width)).astype(np.float32) for _ in cams]
    return scene, cams, dls


# --------------------------------------------------------------------------------------------
# Workload 4: large footprint, 1,000,000 Gaussians, 4 views at 1920x1080
# --------------------------------------------------------------------------------------------
def large_footprint_scene(seed: int = 0, n: int = 1_000_000, width: int = 1920, height: int = 1080):
    scene, rng = frustum_scene(seed, n, 3, -2.0, 0.5)
    pos = rig_positions(4, 5, 0.1)
    sel = [pos[r * 5 + c] for r in (1, 2) for c in (1, 2)]
    cams = [make_camera(np.eye(3), p, width, height) for p in sel]
    return scene, cams


# --------------------------------------------------------------------------------------------
# Workload 3: streaming; the single-view scene seen by a 20-camera rig at 128x128
# --------------------------------------------------------------------------------------------
def streaming_rig(width=128, height=128):
    out = []
    for p in rig_positions(4, 5, 0.1, centre=(0.0, 0.0, 4.0)):
        out.append(make_camera(look_at(p, (0.0, 0.0, 0.0)), p, width, height))
    return out


@dataclass
class TimestepMotion:
    dynamic: np.ndarray      # int32 indices of the Gaussians marked dynamic (sorted)
    dpos: np.ndarray         # (3, n_dyn) float32 ground-truth position delta
    dquat: np.ndarray        # (4, n_dyn) float32 ground-truth rotation delta (unit)


def timestep_motion(seed: int, t: int, n_base: int, frac: float = 0.10,
                    pos_sd: float = 0.01, ang_sd: float = 0.02) -> TimestepMotion:
    rng = np.random.default_rng([seed, t])
    n_dyn = int(round(frac * n_base))
    dyn = np.sort(rng.choice(n_base, size=n_dyn, replace=False)).astype(np.int32)
    dpos = rng.normal(0.0, pos_sd, size=(3, n_dyn)).astype(np.float32)
    axis = rng.normal(0.0, 1.0, size=(3, n_dyn))
    axis /= np.linalg.norm(axis, axis=0, keepdims=True)
    ang = rng.normal(0.0, ang_sd, size=n_dyn)
    dq = np.concatenate([np.cos(ang / 2)[None], axis * np.sin(ang / 2)[None]], 0).astype(np.float32)
    return TimestepMotion(dyn, dpos, dq)


# --------------------------------------------------------------------------------------------
# Workload 5: serving requests
# --------------------------------------------------------------------------------------------
RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080))


@dataclass
class Request:
    arrival_s: float
    viewer: int
    camera: Camera


def serving_requests(seed: int = 0, n_requests: int = 30_000, rate_hz: float = 500.0,
                     n_viewers: int = 64):
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps)
    viewers = rng.integers(0, n_viewers, size=n_requests)
    pos = rig_positions()
    lo = np.min(pos, axis=0) - 0.5
    hi = np.max(pos, axis=0) + 0.5
    vpos = rng.uniform(lo, hi, size=(n_viewers, 3))
    vpos[:, 2] = rng.uniform(-0.5, 0.5, size=n_viewers)
    yaw = np.radians(rng.uniform(-10, 10, size=n_viewers))
    pitch = np.radians(rng.uniform(-10, 10, size=n_viewers))
    res = rng.integers(0, len(RESOLUTIONS), size=n_requests)
    reqs = []
    for i in range(n_requests):
        v = int(viewers[i])
        cy_, sy_ = math.cos(yaw[v]), math.sin(yaw[v])
        cp, sp = math.cos(pitch[v]), math.sin(pitch[v])
        Ry = np.array([[cy_, 0, -sy_], [0, 1, 0], [sy_, 0, cy_]])
        Rx = np.array([[1, 0, 0], [0, cp, -sp], [0, sp, cp]])
        W, H = RESOLUTIONS[int(res[i])]
        reqs.append(Request(float(arrivals[i]), v, make_camera(Rx @ Ry, vpos[v], W, H)))
    return reqs


def random_images(seed: int, n_views: int, width: int, height: int, lo=0.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return [rng.uniform(lo, hi, size=(3, height, width)).astype(np.float32) for _ in range(n_views)]


def tiny_scene(seed: int, n: int, width: int, height: int, sh_degree: int = 0, log_scale_mu=-2.5,
               log_scale_sd=0.3, spread=0.6):
    """A small scene in front of a single camera at (0,0,4) (used for checks with brute force)."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-spread, spread, size=(3, n)).astype(np.float32)
    log_scale = rng.normal(log_scale_mu, log_scale_sd, size=(3, n)).astype(np.float32)
    quat = _quats(rng, n)
    logit = rng.normal(0.5, 1.0, size=n).astype(np.float32)
    sh = _colour_coeffs(rng, n, sh_degree, 0.2)
    cam = make_camera(np.diag([1.0, -1.0, -1.0]), (0.0, 0.0, 4.0), width, height)
    dl = rng.normal(0.0, 1.0, size=(3, height, width)).astype(np.float32)
    return Scene(mean, quat, log_scale, logit, sh, sh_degree), [cam], [dl]


def opaque_scene(seed: int, n: int = 240, width: int = 64, height: int = 48, n_opaque: int = 12,
                 sh_degree: int = 1):
    """tiny_scene's Gaussians (log-scales N(-2.2, 0.3)) behind n_opaque nearly opaque ones (logits
    N(8, 0.5), opacity about 0.9997) at depth 2.5 in front of the camera at (0, 0, 4): centres on
    a 4-wide grid of 16-pixel cells jittered by U[-4, 4] pixels, footprint standard deviation
    U[8, 12] pixels (log-scales perturbed by N(0, 0.2) per axis), random orientation.  Near the
    opaque centres alpha reaches the 0.99 clamp.
    Draw order: the tiny scene, then jitter, footprint, log-scale noise, quaternions, logits,
    colour coefficients."""
    scene, cams, dls = tiny_scene(seed, n, width, height, sh_degree=sh_degree, log_scale_mu=-2.2)
    rng = np.random.default_rng(seed + 1000)
    cam = cams[0]
    f = focal_from_fov(width)
    z = 2.5  # camera depth (the camera sits at z = 4 looking along -z)
    cells = [(i, j) for j in range(max(1, height // 16)) for i in range(4)][:n_opaque]
    m = len(cells)
    u = np.array([8.0 + 16.0 * i for i, _ in cells]) + rng.uniform(-4.0, 4.0, size=m)
    v = np.array([8.0 + 16.0 * j for _, j in cells]) + rng.uniform(-4.0, 4.0, size=m)
    mean = np.stack([(u - cam.cx) * z / f, -(v - cam.cy) * z / f, np.full(m, 4.0 - z)])
    sd = rng.uniform(8.0, 12.0, size=m) * z / f
    log_scale = np.log(sd)[None, :] + rng.normal(0.0, 0.2, size=(3, m))
    quat = _quats(rng, m)
    logit = rng.normal(8.0, 0.5, size=m)
    sh = _colour_coeffs(rng, m, sh_degree, 0.2)
    cat = lambda a, b: np.concatenate([a, b.astype(np.float32)], axis=-1)
    out = Scene(cat(scene.mean, mean), cat(scene.quat, quat), cat(scene.log_scale, log_scale),
                cat(scene.logit, logit), cat(scene.sh, sh), sh_degree)
    return out, cams, dls


def yawed_camera(campos, yaw_deg: float, pitch_deg: float, width: int, height: int) -> Camera:
    """Camera at campos looking along +z turned by yaw (about the camera's y axis) then pitch
    (about its x axis)."""
    a, b = math.radians(yaw_deg), math.radians(pitch_deg)
    ry = np.array([[math.cos(a), 0.0, -math.sin(a)], [0.0, 1.0, 0.0], [math.sin(a), 0.0, math.cos(a)]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(b), math.sin(b)], [0.0, -math.sin(b), math.cos(b)]])
    return make_camera(rx @ ry, campos, width, height)


def off_frustum_scene(seed: int, n: int, width: int, height: int, n_views: int = 1, sh_degree: int = 3,
                      frac_outside: float = 0.7):
    """Gaussians placed beside the field of view with footprints large enough to reach the image,
    seen by n_views cameras on a short horizontal line, turned by yaw and pitch U[-8, 8] degrees
    (view 0 looks straight along +z).

    In view 0's image plane a Gaussian's centre sits at (a_x W/2, a_y H/2) pixels from the image
    centre, at depth U[2, 6].  A fraction frac_outside lies off the image, half to the left or
    right (|a_x| in U[1.3, 1.75], a_y in U[-1, 1]) and half above or below (|a_y| in U[1.3, 1.75],
    a_x in U[-1, 1]); the rest lies on the image (|a_x|, |a_y| < 1).  Scales give a footprint
    standard deviation of U[0.15, 0.35] x W/2 pixels at the Gaussian's depth (log-scales perturbed
    by N(0, 0.3) per axis), so about three standard deviations reach back into the image.
    Draw order: views' yaw and pitch, class, offsets, depth, scale factor, log-scale noise, then
    quaternions, opacity logits, colour coefficients, upstream gradients N(0, 1)."""
    rng = np.random.default_rng(seed)
    turns = rng.uniform(-8.0, 8.0, size=(n_views, 2))
    turns[0] = 0.0
    cams = [yawed_camera((0.15 * v, 0.0, 0.0), turns[v, 0], turns[v, 1], width, height) for v in range(n_views)]
    cls = rng.uniform(0.0, 1.0, size=n)
    off = rng.uniform(1.3, 1.75, size=n) * rng.choice([-1.0, 1.0], size=n)
    inner = rng.uniform(-1.0, 1.0, size=(2, n))
    ax = np.where(cls < frac_outside / 2, off, inner[0])
    ay = np.where((cls >= frac_outside / 2) & (cls < frac_outside), off, inner[1])
    z = rng.uniform(2.0, 6.0, size=n)
    f = focal_from_fov(width)
    xc = np.stack([ax * (width / 2.0) / f * z, ay * (height / 2.0) / f * z, z])
    c0 = cams[0]
    mean = (c0.R.astype(np.float64).T @ (xc - c0.t.astype(np.float64)[:, None])).astype(np.float32)
    sd_px = rng.uniform(0.15, 0.35, size=n) * (width / 2.0)
    log_scale = (np.log(sd_px * z / f)[None, :] + rng.normal(0.0, 0.3, size=(3, n))).astype(np.float32)
    quat = _quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    sh = _colour_coeffs(rng, n, sh_degree, 0.2)
    dls = [rng.normal(0.0, 1.0, size=(3, height, width)).astype(np.float32) for _ in cams]
    return Scene(mean, quat, log_scale, logit, sh, sh_degree), cams, dls


@dataclass
class HashFieldParams:
    """Parameters of one hash-encoded deformation field (float32): per-level grid resolutions,
    F features per table row, 2^log2_table rows per level, an MLP of one hidden layer."""
    res: list
    features: int
    log2_table: int
    hidden: int
    aabb_min: np.ndarray
    aabb_max: np.ndarray
    table: np.ndarray  # (L, T, F)
    w1: np.ndarray     # (hidden, L*F)
    b1: np.ndarray     # (hidden,)
    w2: np.ndarray     # (7, hidden)
    b2: np.ndarray     # (7,)


def geometric_res(n_min: int, n_max: int, levels: int) -> list:
    """Level resolutions N_min..N_max in a geometric progression, floored (top level exact)."""
    if levels == 1:
        return [int(n_min)]
    return [int(math.floor(n_min * (n_max / n_min) ** (l / (levels - 1)) + 1e-9)) for l in range(levels)]


def hash_field_params(seed: int, levels: int = 16, features: int = 4, log2_table: int = 16,
                      hidden: int = 64, n_min: int = 16, n_max: int = 2048, aabb=(-1.5, 1.5),
                      table_scale: float = 0.5, w2_scale: float = 0.1) -> HashFieldParams:
    """Random field parameters; draws table, w1, b1, w2, b2 in that order.  Defaults: the dynamic
    group's field of the N3DV setting (T = 2^16, F = 4; App. B)."""
    rng = np.random.default_rng(seed)
    lf = levels * features
    table = rng.uniform(-table_scale, table_scale, size=(levels, 1 << log2_table, features)).astype(np.float32)
    w1 = (rng.normal(0.0, 1.0, size=(hidden, lf)) * math.sqrt(2.0 / lf)).astype(np.float32)
    b1 = rng.normal(0.0, 0.1, size=hidden).astype(np.float32)
    w2 = (rng.normal(0.0, 1.0, size=(7, hidden)) * w2_scale).astype(np.float32)
    b2 = rng.normal(0.0, 0.01, size=7).astype(np.float32)
    lo = np.full(3, aabb[0], np.float32)
    hi = np.full(3, aabb[1], np.float32)
    return HashFieldParams(geometric_res(n_min, n_max, levels), features, log2_table, hidden, lo, hi,
                           table, w1, b1, w2, b2)


def field_queries(seed: int, n: int, m: int, spread: float = 1.2):
    """Positions (3, n) in a box of half-width `spread`, m distinct query indices (sorted), and
    upstream gradients d_dpos (3, m), d_drot (4, m)."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-spread, spread, size=(3, n)).astype(np.float32)
    idx = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
    d_dpos = rng.normal(0.0, 1.0, size=(3, m)).astype(np.float32)
    d_drot = rng.normal(0.0, 1.0, size=(4, m)).astype(np.float32)
    return mean, idx, d_dpos, d_drot


def inheritance_logits(seed: int, n_var: int, frac_masked: float = 0.3):
    """Learnable inheritance values m of G^var: about frac_masked of them negative (masked out),
    a few exactly zero (the rounding tie of Quant(sigmoid(m)) at 1/2)."""
    rng = np.random.default_rng(seed)
    m = np.abs(rng.normal(0.0, 1.5, size=n_var)) + 1e-3
    neg = rng.random(n_var) < frac_masked
    m[neg] = -m[neg]
    m[rng.random(n_var) < 0.02] = 0.0
    return m.astype(np.float32)


def identity_setup(seed: int, n: int, n_objects: int = 8, channels: int = 16, noise: float = 0.15):
    """Identity features of Gaussian Grouping for n Gaussians: each belongs to one of n_objects
    objects (uniform), its feature is the object's unit code plus noise; a linear classifier
    (cls_w (K, C), cls_b (K,)) that maps the codes to their objects.  Returns
    (feat (C, n) float32, object of each Gaussian (n,), cls_w, cls_b)."""
    rng = np.random.default_rng(seed)
    codes = rng.normal(size=(n_objects, channels))
    codes /= np.linalg.norm(codes, axis=1, keepdims=True)
    obj = rng.integers(0, n_objects, size=n)
    feat = (codes[obj].T + noise * rng.normal(size=(channels, n))).astype(np.float32)
    cls_w = (4.0 * codes).astype(np.float32)
    cls_b = rng.normal(0.0, 0.05, size=n_objects).astype(np.float32)
    return feat, obj.astype(np.int32), cls_w, cls_b


def flow_maps(seed: int, cams, frac: float = 0.05):
    """Per-view optical-flow magnitudes (H, W): mostly small, large in a few random discs."""
    rng = np.random.default_rng(seed)
    out = []
    for c in cams:
        f = np.abs(rng.normal(0.0, 0.2, size=(c.height, c.width)))
        yy, xx = np.mgrid[0:c.height, 0:c.width]
        for _ in range(3):
            cx, cy = rng.uniform(0, c.width), rng.uniform(0, c.height)
            r = np.sqrt(frac * c.width * c.height / np.pi)
            f[(xx - cx) ** 2 + (yy - cy) ** 2 < r * r] += 3.0
        out.append(f.astype(np.float32))
    return out

"""Python binding of libdass over torch device tensors.

PyTorch provides device memory and streams only: every step of the hot path runs in the
library's HIP kernels, reached through the C ABI of include/dass.h.  There is no CPU
fallback -- a missing or unloadable library raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _ffi as F


class DassError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{F.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def n_sh(deg: int) -> int:
    return (deg + 1) * (deg + 1)


@dataclass
class GaussianBuffers:
    """Structure-of-arrays parameter planes with `capacity` columns (rows [0,n) live)."""
    mean: torch.Tensor       # (3, cap)
    quat: torch.Tensor       # (4, cap)
    log_scale: torch.Tensor  # (3, cap)
    logit: torch.Tensor      # (cap,)
    sh: torch.Tensor         # (3K, cap)
    n: int
    n_base: int
    sh_degree: int

    @property
    def capacity(self) -> int:
        return int(self.mean.shape[1])

    @staticmethod
    def allocate(capacity: int, sh_degree: int, device="cuda") -> "GaussianBuffers":
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=device)
        return GaussianBuffers(z(3, capacity), z(4, capacity), z(3, capacity), z(capacity),
                               z(3 * n_sh(sh_degree), capacity), 0, 0, sh_degree)

    @staticmethod
    def from_arrays(mean, quat, log_scale, logit, sh, sh_degree: int, capacity: Optional[int] = None,
                    n_base: Optional[int] = None, device="cuda") -> "GaussianBuffers":
        n = int(np.asarray(mean).shape[1])
        cap = capacity if capacity is not None else n
        g = GaussianBuffers.allocate(cap, sh_degree, device)
        for dst, src in ((g.mean, mean), (g.quat, quat), (g.log_scale, log_scale), (g.sh, sh)):
            dst[:, :n] = torch.as_tensor(np.asarray(src, np.float32), device=device)
        g.logit[:n] = torch.as_tensor(np.asarray(logit, np.float32), device=device)
        g.n = n
        g.n_base = n if n_base is None else n_base
        return g

    def planes(self):
        return (self.mean, self.quat, self.log_scale, self.logit, self.sh)

    def struct(self) -> F.Gaussians:
        return F.Gaussians(self.n, self.capacity, self.n_base, self.sh_degree, _ptr(self.mean), _ptr(self.quat),
                           _ptr(self.log_scale), _ptr(self.logit), _ptr(self.sh))

    def zeros_like(self) -> "GaussianBuffers":
        g = GaussianBuffers.allocate(self.capacity, self.sh_degree, self.mean.device)
        g.n, g.n_base = self.n, self.n_base
        return g

    def clone(self) -> "GaussianBuffers":
        return GaussianBuffers(self.mean.clone(), self.quat.clone(), self.log_scale.clone(), self.logit.clone(),
                               self.sh.clone(), self.n, self.n_base, self.sh_degree)


def carve_zeroed(specs, device="cuda"):
    """One zeroed device buffer holding contiguous tensors of the given (shape, dtype) specs
    (float32 or int32, each starting on a 256-byte boundary), so that per-step accumulators are
    cleared by a single fill of the buffer.  Returns (buffer, [tensors])."""
    sizes = [int(np.prod(shape)) for shape, _ in specs]
    offs, o = [], 0
    for n in sizes:
        offs.append(o)
        o += (n + 63) // 64 * 64
    buf = torch.zeros(max(o, 1), dtype=torch.float32, device=device)
    out = []
    for (shape, dt), off, n in zip(specs, offs, sizes):
        t = buf[off:off + n]
        if dt == torch.int32:
            t = t.view(torch.int32)
        out.append(t.view(*shape))
    return buf, out


def zeroed_grads(g: "GaussianBuffers", extra=()):
    """Gradient planes shaped like g plus the extra (shape, dtype) tensors, carved from one buffer:
    (buffer, GaussianBuffers of gradients, [extra tensors])."""
    cap, P = g.capacity, g.sh.shape[0]
    specs = [((3, cap), torch.float32), ((4, cap), torch.float32), ((3, cap), torch.float32),
             ((cap,), torch.float32), ((P, cap), torch.float32), *extra]
    buf, t = carve_zeroed(specs, g.mean.device)
    return buf, GaussianBuffers(*t[:5], g.n, g.n_base, g.sh_degree), t[5:]


def grads_struct(g: Optional[GaussianBuffers]) -> F.Grads:
    if g is None:
        return F.Grads()
    return F.Grads(_ptr(g.mean), _ptr(g.quat), _ptr(g.log_scale), _ptr(g.logit), _ptr(g.sh))


def camera_struct(cam) -> F.Camera:
    c = F.Camera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(-1)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).reshape(-1)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.campos[:] = [float(x) for x in np.asarray(cam.campos, np.float32).reshape(-1)]
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def cameras_array(cams):
    arr = (F.Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


@dataclass
class RenderOut:
    rgb: torch.Tensor        # (3, H, W)
    t_final: torch.Tensor    # (H, W)
    n_contrib: torch.Tensor  # (H, W) int32

    @staticmethod
    def allocate(cam, device="cuda") -> "RenderOut":
        H, W = int(cam.height), int(cam.width)
        return RenderOut(torch.empty(3, H, W, device=device), torch.empty(H, W, device=device),
                         torch.empty(H, W, dtype=torch.int32, device=device))

    def struct(self) -> F.Image:
        return F.Image(_ptr(self.rgb), _ptr(self.t_final), _ptr(self.n_contrib))


def keys_needed_estimate(n_gaussians: int, n_views: int, tiles_per_gaussian: float = 16.0) -> int:
    return int(n_gaussians * n_views * tiles_per_gaussian)


def geometric_res(n_min: int, n_max: int, levels: int) -> list:
    """Level resolutions from n_min to n_max in a geometric progression, floored (top level exact)."""
    if levels == 1:
        return [int(n_min)]
    return [int(np.floor(n_min * (n_max / n_min) ** (l / (levels - 1)) + 1e-9)) for l in range(levels)]


@dataclass
class HashField:
    """Device parameters of one hash-encoded deformation field (dass_hash_field)."""
    res: list
    features: int
    log2_table: int
    hidden: int
    aabb_min: tuple
    aabb_max: tuple
    table: torch.Tensor  # (L, T, F)
    w1: torch.Tensor     # (hidden, L*F)
    b1: torch.Tensor     # (hidden,)
    w2: torch.Tensor     # (7, hidden)
    b2: torch.Tensor     # (7,)

    @property
    def levels(self) -> int:
        return len(self.res)

    def arrays(self):
        return (self.table, self.w1, self.b1, self.w2, self.b2)

    def zeros_like(self) -> "HashField":
        return HashField(list(self.res), self.features, self.log2_table, self.hidden, self.aabb_min, self.aabb_max,
                         *[torch.zeros_like(t) for t in self.arrays()])

    def struct(self) -> F.HashField:
        L = self.levels
        r = (list(self.res) + [0] * F.HASH_MAX_LEVELS)[:F.HASH_MAX_LEVELS]  # levels > 16: refused by the library
        res = (C.c_int32 * F.HASH_MAX_LEVELS)(*r)
        return F.HashField(L, int(self.features), int(self.log2_table), int(self.hidden), res,
                           (C.c_float * 3)(*self.aabb_min), (C.c_float * 3)(*self.aabb_max),
                           *[_ptr(t) for t in self.arrays()])

    @staticmethod
    def from_numpy(p, device) -> "HashField":
        """From host arrays (an object with res, features, log2_table, hidden, aabb_min, aabb_max,
        table, w1, b1, w2, b2)."""
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        return HashField(list(p.res), int(p.features), int(p.log2_table), int(p.hidden),
                         tuple(float(x) for x in p.aabb_min), tuple(float(x) for x in p.aabb_max),
                         t(p.table), t(p.w1), t(p.b1), t(p.w2), t(p.b2))

    @staticmethod
    def init(res, features, log2_table, hidden, aabb_min, aabb_max, device, seed=0, table_scale=1e-4):
        """A fresh field: table entries uniform in +-table_scale, a He-normal first layer, zero
        biases and a zero output layer (the identity shift)."""
        g = torch.Generator(device="cpu").manual_seed(int(seed))
        L, lf = len(res), len(res) * features
        table = (torch.rand(L, 1 << log2_table, features, generator=g) * 2 - 1) * table_scale
        w1 = torch.randn(hidden, lf, generator=g) * float(np.sqrt(2.0 / lf))
        return HashField(list(res), int(features), int(log2_table), int(hidden), tuple(map(float, aabb_min)),
                         tuple(map(float, aabb_max)), table.to(device), w1.to(device),
                         torch.zeros(hidden, device=device), torch.zeros(7, hidden, device=device),
                         torch.zeros(7, device=device))


class Context:
    """One libdass context (device workspace + state of the last render_fwd)."""

    def __init__(self, max_gaussians: int, max_views: int, max_keys: int, max_tiles: int, device: int = 0):
        self._lib = F.lib()
        self.device = device
        self._h = C.c_void_p()
        lim = F.Limits(max_gaussians, max_views, max_keys, max_tiles)
        st = self._lib.dass_create(C.byref(self._h), device, C.byref(lim))
        if st != F.DASS_OK:
            raise DassError(st, "dass_create failed")
        self.limits = lim
        self.generation = 0  # bumped by every call that replaces the state kept for render_bwd
        # tile size of render_fwd / render_bwd: (tw, th) with edges 16, 32 or 64, optionally with
        # a third entry, the sub-tile edge of the blend (16, or 8 for one pixel per lane)
        self.tile = (16, 16)
        # list entries the blend stages in LDS at a time (64, 128 or 256); only speed depends on it
        self.batch = 128

    def close(self):
        if self._h:
            self._lib.dass_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _opts_for(tile, flags: int = 0, batch: int = 128) -> F.Opts:
        if len(tile) > 2 and int(tile[2]) == 8:
            flags |= F.FLAG_SUBTILE8
        return F.Opts(int(tile[0]), int(tile[1]), int(batch), flags)

    def _opts(self, flags: int = 0) -> F.Opts:
        return self._opts_for(self.tile, flags, self.batch)

    def _check(self, st: int):
        if st != F.DASS_OK:
            msg = self._lib.dass_last_error(self._h)
            raise DassError(st, msg.decode() if msg else "")

    # ---- context ---------------------------------------------------------------------------
    def reserve(self, max_gaussians=0, max_views=1, max_keys=0, max_tiles=0):
        self._check(self._lib.dass_reserve(self._h, C.byref(F.Limits(max_gaussians, max_views, max_keys,
                                                                        max_tiles))))

    def sync(self, stream=None):
        self._check(self._lib.dass_sync(self._h, _stream(stream)))

    # ---- hot path --------------------------------------------------------------------------
    def render_fwd(self, g: GaussianBuffers, cams: Sequence, bg=(0.0, 0.0, 0.0), out=None, stream=None,
                   count_pairs: bool = False):
        out = out if out is not None else [RenderOut.allocate(c, g.mean.device) for c in cams]
        imgs = (F.Image * len(cams))(*[o.struct() for o in out])
        bgf = (C.c_float * 3)(*[float(x) for x in bg])
        gs = g.struct()
        opts = self._opts(F.FLAG_COUNT_PAIRS if count_pairs else 0)
        self.generation += 1
        self._check(self._lib.render_fwd(self._h, C.byref(gs), cameras_array(cams), len(cams), bgf, imgs,
                                         C.byref(opts), _stream(stream)))
        return out

    def render_bwd(self, g: GaussianBuffers, cams: Sequence, bg, fwd_out, dl_drgb, grads: GaussianBuffers,
                   gradnorm: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None, stream=None):
        imgs = (F.Image * len(cams))(*[o.struct() for o in fwd_out])
        dls = (C.c_void_p * len(cams))(*[_ptr(d) for d in dl_drgb])
        bgf = (C.c_float * 3)(*[float(x) for x in bg])
        gs = g.struct()
        gr = grads_struct(grads)
        opts = self._opts()
        self._check(self._lib.render_bwd(self._h, C.byref(gs), cameras_array(cams), len(cams), bgf, imgs, dls,
                                         C.byref(gr), _ptr(gradnorm), _ptr(count), C.byref(opts), _stream(stream)))

    # order of preference: 16x16 sub-tiles first, smaller key bins first (less work per list when
    # times are close); then 8x8 sub-tiles (one pixel per lane), which pay off on small images
    TILE_CANDIDATES = ((16, 16), (32, 16), (16, 32), (32, 32), (64, 32), (32, 64), (64, 64),
                       (16, 16, 8), (32, 16, 8), (32, 32, 8), (64, 64, 8))

    def autotune_tile(self, g: GaussianBuffers, cams: Sequence, bg, out, dl_drgb, grads: GaussianBuffers,
                      candidates=TILE_CANDIDATES, reps: int = 3, stream=None, apply: bool = True,
                      batches=(128,)) -> dict:
        """Times render_fwd + render_bwd of this workload at each candidate tile size and blend
        batch (native autotuner; synchronises) and, if `apply`, makes its choice this context's
        tile size and batch: the first candidate, in the given order (tiles, then batches), within
        1% of the fastest.  Returns {(tw, th[, 8]): ms} for a single batch, else
        {((tw, th[, 8]), batch): ms}; None where a candidate does not fit the budgets.  `grads`
        is scratch."""
        imgs = (F.Image * len(cams))(*[o.struct() for o in out])
        dls = (C.c_void_p * len(cams))(*[_ptr(d) for d in dl_drgb])
        bgf = (C.c_float * 3)(*[float(x) for x in bg])
        gs = g.struct()
        gr = grads_struct(grads)
        pairs = [(tuple(c), int(b)) for c in candidates for b in batches]
        cand = (F.Opts * len(pairs))(*[self._opts_for(c, 0, b) for c, b in pairs])
        best = C.c_int32(-1)
        ms = (C.c_float * len(pairs))()
        self.generation += 1
        self._check(self._lib.dass_autotune_tile(self._h, C.byref(gs), cameras_array(cams), len(cams), bgf, imgs, dls,
                                                 C.byref(gr), cand, len(pairs), int(reps), C.byref(best), ms,
                                                 _stream(stream)))
        if apply:
            self.tile = tuple(int(x) for x in pairs[best.value][0])
            self.batch = pairs[best.value][1]
        res = {p: (float(ms[i]) if ms[i] >= 0 else None) for i, p in enumerate(pairs)}
        return {p[0]: v for p, v in res.items()} if len(batches) == 1 else res

    def shift_fwd(self, g: GaussianBuffers, out: GaussianBuffers, dyn_idx: torch.Tensor, dpos: torch.Tensor,
                  drot: torch.Tensor, stream=None):
        gs, os_ = g.struct(), out.struct()
        self._check(self._lib.shift_apply(self._h, F.DASS_FWD, _ptr(dyn_idx), int(dyn_idx.numel()), _ptr(dpos),
                                          _ptr(drot), C.byref(gs), C.byref(os_), None, None, None, _stream(stream)))

    def shift_adjoint(self, g: GaussianBuffers, dyn_idx: torch.Tensor, drot: torch.Tensor, d_out: GaussianBuffers,
                      d_dpos: torch.Tensor, d_drot: torch.Tensor, stream=None):
        gs = g.struct()
        gr = grads_struct(d_out)
        self._check(self._lib.shift_apply(self._h, F.DASS_ADJOINT, _ptr(dyn_idx), int(dyn_idx.numel()), None,
                                          _ptr(drot), C.byref(gs), None, C.byref(gr), _ptr(d_dpos), _ptr(d_drot),
                                          _stream(stream)))

    @staticmethod
    def _cols(t: torch.Tensor, col: int, m: int):
        """Pointer to column `col` of a contiguous (rows, ld) float32 tensor holding m columns from there."""
        if t.dtype != torch.float32 or t.dim() != 2:
            raise ValueError("offset buffers are (rows, ld) float32 tensors")
        if col < 0 or col + m > t.shape[1]:
            raise ValueError(f"columns [{col}, {col + m}) outside a buffer of {t.shape[1]}")
        p = _ptr(t)
        return C.c_void_p(p.value + 4 * col) if p is not None else None

    def hash_field_fwd(self, field: "HashField", mean: torch.Tensor, n: int, idx: Optional[torch.Tensor],
                       m: int, dpos: torch.Tensor, drot: torch.Tensor, col: int = 0, stream=None):
        """Offsets of the field at rows idx (or rows [0, m)) of mean (3, stride): columns
        [col, col + m) of dpos (3, ld) and drot (4, ld)."""
        fs = field.struct()
        self._check(self._lib.dass_hash_field_fwd(self._h, C.byref(fs), _ptr(mean), int(mean.shape[1]), int(n),
                                                  _ptr(idx), int(m), self._cols(dpos, col, m),
                                                  self._cols(drot, col, m), int(dpos.shape[1]), _stream(stream)))

    def hash_field_bwd(self, field: "HashField", mean: torch.Tensor, n: int, idx: Optional[torch.Tensor], m: int,
                       d_dpos: torch.Tensor, d_drot: torch.Tensor, grads: "HashField", col: int = 0, stream=None):
        """Accumulates the field's parameter gradients into the arrays of `grads` (a HashField of
        the same shapes) from columns [col, col + m) of d_dpos (3, ld), d_drot (4, ld)."""
        fs = field.struct()
        gs = F.HashFieldGrads(*[_ptr(t) for t in grads.arrays()])
        self._check(self._lib.dass_hash_field_bwd(self._h, C.byref(fs), _ptr(mean), int(mean.shape[1]), int(n),
                                                  _ptr(idx), int(m), self._cols(d_dpos, col, m),
                                                  self._cols(d_drot, col, m), int(d_dpos.shape[1]), C.byref(gs),
                                                  _stream(stream)))

    # ---- selective inheritance and pruning of G^var ----------------------------------------
    def inherit_apply(self, g: GaussianBuffers, m: torch.Tensor, logit_eff: torch.Tensor,
                      log_scale_eff: torch.Tensor, stream=None):
        """Planes to render with under the inheritance mask of m (one value per G^var row)."""
        gs = g.struct()
        self._check(self._lib.dass_inherit_apply(self._h, C.byref(gs), _ptr(m), _ptr(logit_eff), _ptr(log_scale_eff),
                                                 _stream(stream)))

    def inherit_adjoint(self, g: GaussianBuffers, m: torch.Tensor, d_logit_eff: torch.Tensor,
                        d_log_scale_eff: torch.Tensor, lam: float, dm: torch.Tensor,
                        loss: Optional[torch.Tensor] = None, stream=None):
        gs = g.struct()
        self._check(self._lib.dass_inherit_adjoint(self._h, C.byref(gs), _ptr(m), _ptr(d_logit_eff),
                                                   _ptr(d_log_scale_eff), float(lam), _ptr(dm), _ptr(loss),
                                                   _stream(stream)))

    def compact_var(self, g: GaussianBuffers, m: Optional[torch.Tensor], min_opacity: float, n_kept: torch.Tensor,
                    stream=None):
        """Removes G^var rows in place (masked by m and/or below min_opacity); the kept count lands in
        n_kept (device int32): the caller reads it and sets g.n = g.n_base + kept."""
        gs = g.struct()
        self._check(self._lib.dass_compact_var(self._h, C.byref(gs), _ptr(m), float(min_opacity), _ptr(n_kept),
                                               _stream(stream)))

    # ---- identity features and the dynamics mask -----------------------------------------
    def render_features(self, g: GaussianBuffers, cams, features: torch.Tensor, out=None, stream=None):
        """Identity-feature images (C, H, W) per view of the last render_fwd (same g and cams):
        features is (C, capacity)."""
        C_ = int(features.shape[0])
        if out is None:
            out = [torch.empty(C_, c.height, c.width, device=features.device) for c in cams]
        gs = g.struct()
        O = (C.c_void_p * len(cams))(*[_ptr(o) for o in out])
        opts = self._opts()
        self._check(self._lib.dass_render_features(self._h, C.byref(gs), cameras_array(cams), len(cams),
                                                   _ptr(features), C_, O, C.byref(opts), _stream(stream)))
        return out

    def dynamic_mask(self, cams, feat_imgs, flows, gamma_op: float, cls_w: torch.Tensor, cls_b: torch.Tensor,
                     features: torch.Tensor, n: int, dyn_idx: torch.Tensor, n_dyn: torch.Tensor,
                     dyn_objects: Optional[torch.Tensor] = None, stream=None):
        """Dynamic Gaussians (Sec. 3.3) into dyn_idx (int32, >= n entries); their count lands in
        n_dyn (device int32).  features (C, stride); cls_w (K, C), cls_b (K,)."""
        V = len(cams)
        Fi = (C.c_void_p * V)(*[_ptr(f) for f in feat_imgs])
        Fl = (C.c_void_p * V)(*[_ptr(f) for f in flows])
        self._check(self._lib.dass_dynamic_mask(self._h, cameras_array(cams), V, Fi, Fl, float(gamma_op), _ptr(cls_w),
                                                _ptr(cls_b), int(cls_w.shape[0]), int(cls_w.shape[1]), _ptr(features),
                                                int(features.shape[1]), int(n), _ptr(dyn_idx), _ptr(n_dyn),
                                                _ptr(dyn_objects), _stream(stream)))

    @staticmethod
    def _adam_groups(groups):
        arr = (F.AdamGroup * len(groups))()
        for i, (p, g, m, v, lr) in enumerate(groups):
            arr[i] = F.AdamGroup(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(p.numel()), float(lr))
        return arr

    def adam_step(self, groups, beta1=0.9, beta2=0.999, eps=1e-15, step=1, stream=None, d_step=None):
        """groups: sequence of (param, grad, m, v, lr) with equal-length contiguous float32 tensors.
        With d_step (device int32 tensor) the step count lives on the device and is incremented."""
        arr = self._adam_groups(groups)
        if d_step is not None:
            self._check(self._lib.adam_step_device_count(self._h, arr, len(groups), beta1, beta2, eps, _ptr(d_step),
                                                         _stream(stream)))
        else:
            self._check(self._lib.adam_step(self._h, arr, len(groups), beta1, beta2, eps, int(step),
                                            _stream(stream)))

    def render_fwd_l1(self, g: GaussianBuffers, cams: Sequence, bg, targets, dl_out, err_out=None,
                      loss: Optional[torch.Tensor] = None, out=None, keep_rgb: bool = True, stream=None):
        """render_fwd fused with l1_loss_grad: the blend's epilogue writes dl_out (and err_out,
        and adds the loss into `loss`) as l1_loss_grad would on the rendered images.  With
        keep_rgb False the images themselves are not written (out[v].rgb is left as it was)."""
        out = out if out is not None else [RenderOut.allocate(c, g.mean.device) for c in cams]
        V = len(cams)
        imgs = (F.Image * V)(*[F.Image(_ptr(o.rgb) if keep_rgb else None, _ptr(o.t_final), _ptr(o.n_contrib))
                               for o in out])
        bgf = (C.c_float * 3)(*[float(x) for x in bg])
        T = (C.c_void_p * V)(*[_ptr(t) for t in targets])
        D = (C.c_void_p * V)(*[_ptr(d) for d in dl_out])
        E = (C.c_void_p * V)(*[_ptr(e) for e in err_out]) if err_out is not None else None
        gs = g.struct()
        opts = self._opts()
        self.generation += 1
        self._check(self._lib.dass_render_fwd_l1(self._h, C.byref(gs), cameras_array(cams), V, bgf, imgs, T, D, E,
                                                 _ptr(loss), C.byref(opts), _stream(stream)))
        return out

    def l1_loss_grad(self, cams, renders, targets, dl_out, err_out=None, loss: Optional[torch.Tensor] = None,
                     stream=None):
        V = len(cams)
        R = (C.c_void_p * V)(*[_ptr(r) for r in renders])
        T = (C.c_void_p * V)(*[_ptr(t) for t in targets])
        D = (C.c_void_p * V)(*[_ptr(d) for d in dl_out])
        E = (C.c_void_p * V)(*[_ptr(e) for e in err_out]) if err_out is not None else None
        self._check(self._lib.dass_l1_loss_grad(self._h, cameras_array(cams), V, R, T, D, E, _ptr(loss),
                                                _stream(stream)))

    def fidelity_loss_grad(self, cams, renders, targets, lam: float, dl_out, err_out=None,
                           loss: Optional[torch.Tensor] = None, scratch=None, stream=None):
        """Eq. (3) fidelity loss (1 - lam) L1 + lam D-SSIM: writes dl_out (and err_out, adds the
        loss into `loss`).  scratch: per view a float32 tensor of at least 9 H W elements (made
        here if None; pass preallocated ones in a captured or allocation-free loop)."""
        V = len(cams)
        if scratch is None and lam > 0.0:
            scratch = [torch.empty(9 * c.height * c.width, device=dl_out[i].device) for i, c in enumerate(cams)]
        for i, c in enumerate(cams):
            if scratch is not None and scratch[i].numel() < 9 * c.height * c.width:
                raise ValueError(f"scratch[{i}] holds {scratch[i].numel()} floats, needs {9 * c.height * c.width}")
        R = (C.c_void_p * V)(*[_ptr(r) for r in renders])
        T = (C.c_void_p * V)(*[_ptr(t) for t in targets])
        D = (C.c_void_p * V)(*[_ptr(d) for d in dl_out])
        E = (C.c_void_p * V)(*[_ptr(e) for e in err_out]) if err_out is not None else None
        S = (C.c_void_p * V)(*[_ptr(x) for x in scratch]) if scratch is not None else None
        self._check(self._lib.dass_fidelity_loss_grad(self._h, cameras_array(cams), V, R, T, float(lam), D, E,
                                                      _ptr(loss), S, _stream(stream)))

    def fidelity_loss_grad_noalloc(self, cams, renders, targets, lam: float, dl_out, err_out=None,
                                   loss: Optional[torch.Tensor] = None, stream=None):
        """fidelity_loss_grad with the D-SSIM maps in the library's static per-GPU scratch (no
        allocation anywhere in the call); the views' pixels must fit NOALLOC_MAX_PIXELS."""
        V = len(cams)
        R = (C.c_void_p * V)(*[_ptr(r) for r in renders])
        T = (C.c_void_p * V)(*[_ptr(t) for t in targets])
        D = (C.c_void_p * V)(*[_ptr(d) for d in dl_out])
        E = (C.c_void_p * V)(*[_ptr(e) for e in err_out]) if err_out is not None else None
        self._check(self._lib.dass_fidelity_loss_grad_noalloc(self._h, cameras_array(cams), V, R, T, float(lam), D,
                                                              E, _ptr(loss), _stream(stream)))

    def densify_append(self, g: GaussianBuffers, err_maps, cams, gradnorm, count, gamma_err, tau_pos, tau_err,
                       k_max, seed, n_appended: torch.Tensor, stream=None):
        """Appends children in rows [g.n, g.n + K); K lands in n_appended (device int32); the caller
        reads it and advances g.n."""
        gs = g.struct()
        self.generation += 1
        E = (C.c_void_p * len(cams))(*[_ptr(e) for e in err_maps])
        self._check(self._lib.densify_append(self._h, C.byref(gs), E, cameras_array(cams), len(cams), _ptr(gradnorm),
                                             _ptr(count), float(gamma_err), float(tau_pos), float(tau_err),
                                             int(k_max), int(seed), _ptr(n_appended), _stream(stream)))

    # ---- stage timers ----------------------------------------------------------------------
    def profile_begin(self, max_records: int = 256):
        self._check(self._lib.dass_profile_begin(self._h, int(max_records)))

    def profile_end(self) -> dict:
        ms = (C.c_double * len(F.STAGES))()
        rec = (C.c_int32 * len(F.STAGES))()
        self._check(self._lib.dass_profile_end(self._h, ms, rec))
        return {name: (ms[i], rec[i]) for i, name in enumerate(F.STAGES)}

    # ---- debug -----------------------------------------------------------------------------
    def pair_counts(self):
        ev, bl = C.c_uint64(), C.c_uint64()
        self._check(self._lib.dass_debug_pair_counts(self._h, C.byref(ev), C.byref(bl)))
        return ev.value, bl.value

    def debug_keys(self, view: int, max_keys: int, n_tiles: int, device="cuda"):
        keys = torch.empty(max(max_keys, 1), dtype=torch.int64, device=device)
        vals = torch.empty(max(max_keys, 1), dtype=torch.int32, device=device)
        ranges = torch.empty(n_tiles, 2, dtype=torch.int64, device=device)
        cnt = C.c_int64()
        self._check(self._lib.dass_debug_keys(self._h, view, _ptr(keys), _ptr(vals), max_keys, _ptr(ranges),
                                              C.byref(cnt)))
        c = cnt.value
        return (keys[:c].cpu().numpy().view(np.uint64), vals[:c].cpu().numpy().view(np.uint32),
                ranges.cpu().numpy())

    def debug_projection(self, g: GaussianBuffers, cam):
        out = torch.empty(max(g.n, 1), 16, dtype=torch.float64, device=g.mean.device)
        gs = g.struct()
        opts = self._opts()
        self._check(self._lib.dass_debug_projection(self._h, C.byref(gs), C.byref(camera_struct(cam)),
                                                    C.byref(opts), _ptr(out)))
        return out[:g.n].cpu().numpy()

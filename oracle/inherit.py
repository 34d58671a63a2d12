"""Oracle of selective inheritance (Sec. 3.2 with the straight-through estimator of App. B) and of
the low-opacity pruning of G^var (Sec. 3.4) -- TEST INFRASTRUCTURE, part of the CPU oracle (same
import rules as the package).

Selective inheritance gives each Gaussian of G^var (rows [n_base, n)) a learnable value m.  The
binary mask M = Quant(sigmoid(m)) multiplies the activated opacity and scale used for rendering:
o_r = M o, s_r = M s.  Readings:
  * Quant rounds to the nearer of 0 and 1 with 1/2 going to 1, so M = 1 exactly when m >= 0
    (sigmoid is increasing and sigmoid(0) = 1/2); the decision is taken on m itself;
  * in the renderer's parametrisation (o = sigmoid(logit), s = exp(log_scale)) a masked Gaussian
    has logit = log_scale = -inf (o_r = s_r = 0) and an unmasked one keeps its parameters;
  * the straight-through estimator: the forward uses M, the backward treats it as sigmoid(m), so
    dL/dm = (dL/dM) sigmoid'(m), with dL/dM = <dL/do_r, o> + <dL/ds_r, s> for the Gaussian; the
    mask loss lambda_inher sum sigmoid(m) adds lambda_inher sigmoid'(m);
  * a masked Gaussian is not drawn (its alpha 0 is below the 1/255 skip), so its fidelity terms
    are zero; for an unmasked one, from the renderer's parameter gradients,
    dL/dM = g_logit / (1 - o) + sum_d g_log_scale[d];
  * after the stage the masked rows are removed (order of the kept rows preserved);
  * pruning keeps a G^var row when its opacity is at least min_opacity, i.e. when
    logit >= log(min_opacity / (1 - min_opacity)).
Everything in float64.
"""
from __future__ import annotations

import numpy as np


def sigmoid(x):
    x = np.asarray(x, np.float64)
    return 1.0 / (1.0 + np.exp(-x))


def quant_mask(m) -> np.ndarray:
    """M = Quant(sigmoid(m)) as booleans: m >= 0."""
    return np.asarray(m, np.float64) >= 0.0


def inherit_planes(logit, log_scale, n_base, m):
    """Rendered (effective) opacity logits (n,) and log-scales (3, n) of Eq. for o_r and s_r."""
    lg = np.array(logit, np.float64, copy=True)
    ls = np.array(log_scale, np.float64, copy=True)
    off = ~quant_mask(m)
    idx = n_base + np.nonzero(off)[0]
    lg[idx] = -np.inf
    ls[:, idx] = -np.inf
    return lg, ls


def inherit_grad(logit, n_base, m, g_logit_eff, g_log_scale_eff, lam):
    """dL/dm (n_var,) for the fidelity gradients of the effective planes (g_logit_eff (n,),
    g_log_scale_eff (3, n)) plus the mask loss; also returns the mask-loss value
    lam sum sigmoid(m)."""
    m = np.asarray(m, np.float64)
    nv = m.size
    rows = slice(n_base, n_base + nv)
    M = quant_mask(m)
    o = sigmoid(np.asarray(logit, np.float64)[rows])
    d_M = np.where(M, np.asarray(g_logit_eff, np.float64)[rows] / (1.0 - o)
                   + np.asarray(g_log_scale_eff, np.float64)[:, rows].sum(axis=0), 0.0)
    sp = sigmoid(m) * (1.0 - sigmoid(m))
    return d_M * sp + lam * sp, float(lam * sigmoid(m).sum())


def keep_rows(logit, n_base, m=None, min_opacity=0.0) -> np.ndarray:
    """Which G^var rows survive: the inheritance mask (if m is given) and the opacity floor (if
    min_opacity > 0)."""
    lg = np.asarray(logit, np.float64)[n_base:]
    keep = np.ones(lg.size, bool)
    if m is not None:
        keep &= quant_mask(m)
    if min_opacity > 0.0:
        keep &= lg >= np.log(min_opacity / (1.0 - min_opacity))
    return keep


def compact(planes: dict, n_base: int, keep) -> dict:
    """Planes (each (P, n) or (n,)) with the G^var rows not kept removed, order preserved."""
    keep = np.asarray(keep, bool)
    cols = np.concatenate([np.arange(n_base), n_base + np.nonzero(keep)[0]])
    return {k: np.asarray(v)[..., cols].copy() for k, v in planes.items()}

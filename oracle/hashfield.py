"""Oracle of the hash-encoded deformation fields H_dyn / H_st (Sec. 3.3, App. B) -- TEST
INFRASTRUCTURE, part of the CPU oracle (same import rules as the package).

A field maps a Gaussian's position to its shift offsets: a multi-resolution hash encoding of the
normalised position (the I-NGP encoding the paper cites) followed by a small MLP.  Readings (the
paper gives only T_Hash and F_Hash per group):
  * position p = clamp((mu - aabb_min) / (aabb_max - aabb_min), 0, 1) per axis;
  * level l of L has grid resolution N_l (the caller's list; the encoding's geometric progression
    N_l = floor(N_min b^l) is one choice); x = p N_l; cell c0 = min(floor(x), N_l - 1);
    frac = x - c0; the 8 corners c0 + d, d in {0,1}^3, weighted by prod(d ? frac : 1 - frac);
  * a corner's entry: dense index c_x + (N_l + 1)(c_y + (N_l + 1) c_z) when (N_l + 1)^3 <= T,
    else the spatial hash (c_x * 1 xor c_y * 2654435761 xor c_z * 805459861) mod T in 32-bit
    unsigned arithmetic; F features per entry, one table of T entries per level;
  * MLP: h = relu(W1 enc + b1), out = W2 h + b2 with out in R^7; dpos = out[0:3], drot =
    (1, 0, 0, 0) + out[3:7] (so a zero output layer is the identity shift).
Everything in float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PRIMES = (1, 2654435761, 805459861)


@dataclass
class Field:
    res: list            # N_l per level (L entries)
    features: int
    log2_table: int
    aabb_min: np.ndarray  # (3,)
    aabb_max: np.ndarray  # (3,)
    table: np.ndarray     # (L, T, F)
    w1: np.ndarray        # (H, L*F)
    b1: np.ndarray        # (H,)
    w2: np.ndarray        # (7, H)
    b2: np.ndarray        # (7,)


def corner_index(f: Field, l: int, c) -> np.ndarray:
    """Table row of integer corner coordinates c (..., 3) at level l."""
    n = f.res[l]
    T = 1 << f.log2_table
    c = np.asarray(c, np.int64)
    if (n + 1) ** 3 <= T:
        return c[..., 0] + (n + 1) * (c[..., 1] + (n + 1) * c[..., 2])
    h = np.zeros(c.shape[:-1], np.uint64)
    for d in range(3):
        h ^= (c[..., d].astype(np.uint64) * np.uint64(PRIMES[d])) & np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def normalised(f: Field, mean) -> np.ndarray:
    """(3, m) positions -> (m, 3) in [0, 1]^3."""
    mu = np.asarray(mean, np.float64).T
    p = (mu - f.aabb_min) / (f.aabb_max - f.aabb_min)
    return np.clip(p, 0.0, 1.0)


def corners(f: Field, l: int, p):
    """Rows (m, 8) and trilinear weights (m, 8) of the 8 corners around each position."""
    n = f.res[l]
    x = p * n
    c0 = np.minimum(np.floor(x), n - 1).astype(np.int64)
    fr = x - c0
    rows, wts = [], []
    for k in range(8):
        d = np.array([(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1])
        rows.append(corner_index(f, l, c0 + d))
        wts.append(np.prod(np.where(d == 1, fr, 1.0 - fr), axis=-1))
    return np.stack(rows, -1), np.stack(wts, -1)


def encode(f: Field, p) -> np.ndarray:
    """(m, 3) -> (m, L*F) features."""
    m = p.shape[0]
    enc = np.zeros((m, len(f.res) * f.features))
    for l in range(len(f.res)):
        rows, wts = corners(f, l, p)
        for k in range(8):
            enc[:, l * f.features:(l + 1) * f.features] += wts[:, k, None] * f.table[l][rows[:, k]]
    return enc


def field_fwd(f: Field, mean):
    """Shift offsets of the Gaussians at `mean` (3, m): dpos (3, m), drot (4, m)."""
    enc = encode(f, normalised(f, mean))
    h = np.maximum(enc @ f.w1.T + f.b1, 0.0)
    out = h @ f.w2.T + f.b2
    drot = out[:, 3:7].T.copy()
    drot[0] += 1.0
    return out[:, 0:3].T.copy(), drot


def field_bwd(f: Field, mean, d_dpos, d_drot):
    """Gradients of <d_dpos, dpos> + <d_drot, drot> with respect to the field's parameters:
    dict(table, w1, b1, w2, b2) shaped like the field's arrays."""
    p = normalised(f, mean)
    enc = encode(f, p)
    pre = enc @ f.w1.T + f.b1
    h = np.maximum(pre, 0.0)
    d_out = np.concatenate([np.asarray(d_dpos, np.float64).T, np.asarray(d_drot, np.float64).T], axis=1)
    g = {"w2": d_out.T @ h, "b2": d_out.sum(0)}
    d_pre = (d_out @ f.w2) * (pre > 0.0)
    g["w1"] = d_pre.T @ enc
    g["b1"] = d_pre.sum(0)
    d_enc = d_pre @ f.w1
    table = np.zeros_like(f.table)
    for l in range(len(f.res)):
        rows, wts = corners(f, l, p)
        for k in range(8):
            np.add.at(table[l], rows[:, k], wts[:, k, None] * d_enc[:, l * f.features:(l + 1) * f.features])
    g["table"] = table
    return g


def from_params(p) -> Field:
    """Field in float64 from seeded float32 parameters (synth.HashFieldParams)."""
    f64 = lambda a: np.asarray(a, np.float64)
    return Field(list(p.res), p.features, p.log2_table, f64(p.aabb_min), f64(p.aabb_max), f64(p.table),
                 f64(p.w1), f64(p.b1), f64(p.w2), f64(p.b2))

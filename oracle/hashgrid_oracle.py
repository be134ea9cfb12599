"""Plain float64 oracle of the hash-grid DDF, the paper's fast field.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and imports nothing from it.

What is computed (Sec. III-D):

* The ray origin x is encoded with a multiresolution hash grid (the encoding
  the paper cites as Mueller et al. 2022): L levels with resolutions
  N_l = floor(N_min b^l), each a table of F features per vertex.  Level l
  scales the point, normalised to the unit cube of the object box, by N_l; the
  8 vertices of the cell containing it are looked up and their features are
  interpolated trilinearly.  A level whose (N_l + 1)^3 vertices fit the table
  size T indexes them densely (v0 + v1 (N_l + 1) + v2 (N_l + 1)^2); a finer
  level hashes them, h(v) = (v0 pi_0 XOR v1 pi_1 XOR v2 pi_2) mod T with the
  published primes pi = (1, 2654435761, 805459861), in 32-bit unsigned
  arithmetic.
* The direction d is encoded with four sinusoidal bands,
  [d, sin(pi 2^k d), cos(pi 2^k d)] for k < 4 (the same block form as the
  sinusoidal field).
* A ReLU MLP of two hidden layers of width 64 reads [position code, direction
  code] and two linear heads give t = softplus(z_t) and xi = sigmoid(z_xi).
* The paper's sizes: 16 levels, 2 features, 2^19 entries per level, N_min = 16,
  b = 1.5 over the object box: about 13M table parameters and an MLP of about
  8k, a 52 MB field.

Readings where the paper is silent (each also listed in the design notes):
* The box is [-1.5, 1.5]^3; a point outside is clamped to it.
* Level l: s = p N_l with p in [0, 1]^3; the cell's lower vertex is
  c = min(floor(s), N_l - 1) per axis (so p = 1 lies in the last cell), the
  weights w = s - c.
* The cell is an integer decision taken from floating point, so for parity with
  a float32 kernel the oracle can form p and s the way that kernel does
  (coords="fp32": p = fl(fl(x + h) fl(0.5 / h)) clamped, s = fl(p N), each
  operation rounded to float32); the interpolation from s on stays exact.  At
  the finest levels (N ~ 7000) float32 grid coordinates are off by up to ~1e-3
  cell, so this matters.  coords="exact" (the default) uses float64 throughout.
* The table is laid out level after level, F floats per entry; level l holds
  min(T, (N_l + 1)^3) entries.  The MLP parameters follow the table: W1 [64 x D],
  b1, W2 [64 x 64], b2, heads [2 x 64], [2], with D = 2 L + 3 (1 + 2 bands).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ddf_oracle as O

PRIMES = (1, 2654435761, 805459861)


# ----------------------------------------------------------------------------
# Layout
# ----------------------------------------------------------------------------

def resolutions(desc):
    """N_l = floor(N_min b^l) for every level."""
    return [int(math.floor(desc.base_res * desc.growth ** l)) for l in range(desc.n_levels)]


def levels(desc):
    """[(N_l, entries_l, dense_l, offset_l)] with offsets counted in entries."""
    T = 1 << desc.log2_table
    out, off = [], 0
    for N in resolutions(desc):
        full = (N + 1) ** 3
        dense = full <= T
        e = full if dense else T
        out.append((N, e, dense, off))
        off += e
    return out


def table_entries(desc):
    return sum(e for _, e, _, _ in levels(desc))


def n_dir_features(desc):
    return 3 * (1 + 2 * desc.dir_bands)


def mlp_shapes(desc):
    fan_in = desc.n_feat * desc.n_levels + n_dir_features(desc)
    shapes = []
    for _ in range(desc.n_hidden):
        shapes.append((desc.width, fan_in))
        fan_in = desc.width
    shapes.append((desc.n_out, desc.width))
    return shapes


def param_count(desc):
    return table_entries(desc) * desc.n_feat + sum(o * i + o for o, i in mlp_shapes(desc))


def split(desc, params):
    """(table [E, F] float64, [(W, b)] float64)."""
    p = np.asarray(params, dtype=np.float64)
    E = table_entries(desc)
    table = p[:E * desc.n_feat].reshape(E, desc.n_feat)
    off = E * desc.n_feat
    mlp = []
    for o, i in mlp_shapes(desc):
        W = p[off:off + o * i].reshape(o, i); off += o * i
        b = p[off:off + o]; off += o
        mlp.append((W, b))
    assert off == p.size
    return table, mlp


# ----------------------------------------------------------------------------
# Encoding
# ----------------------------------------------------------------------------

def unit_coords(desc, x, coords="exact"):
    """Points [N, 3] in the object box -> [0, 1]^3 (clamped)."""
    if coords == "fp32":
        h = np.float32(desc.box_half)
        inv = np.float32(0.5) / h
        p = (np.asarray(x, dtype=np.float32) + h) * inv
        return np.clip(p, np.float32(0), np.float32(1))
    lo = -desc.box_half
    return np.clip((np.asarray(x, dtype=np.float64) - lo) / (2 * desc.box_half), 0.0, 1.0)


def vertex_index(N, dense, T, v):
    """Table index of integer vertices v [..., 3] of a level (int64 arithmetic, uint32 hash)."""
    v = np.asarray(v, dtype=np.int64)
    if dense:
        return v[..., 0] + v[..., 1] * (N + 1) + v[..., 2] * (N + 1) ** 2
    h = np.zeros(v.shape[:-1], dtype=np.int64)
    for a in range(3):
        h ^= (v[..., a] * PRIMES[a]) & 0xFFFFFFFF
    return h % T


def corners(desc, x, coords="exact"):
    """Per level: (indices [N, 8] into the whole table, weights [N, 8]) of the trilinear lookup."""
    p = unit_coords(desc, x, coords)
    T = 1 << desc.log2_table
    out = []
    for N, e, dense, off in levels(desc):
        s = (p * np.float32(N)).astype(np.float64) if coords == "fp32" else p * N
        c = np.minimum(np.floor(s), N - 1)
        w = s - c
        idx = np.empty((len(p), 8), dtype=np.int64)
        wt = np.empty((len(p), 8))
        for k in range(8):
            dl = np.array([(k >> a) & 1 for a in range(3)])
            idx[:, k] = off + vertex_index(N, dense, T, c.astype(np.int64) + dl)
            wt[:, k] = np.prod(np.where(dl[None] == 1, w, 1.0 - w), axis=1)
        out.append((idx, wt))
    return out


def encode_position(desc, table, x, coords="exact"):
    """[N, L F] interpolated features, level-major."""
    feats = [np.einsum('nk,nkf->nf', wt, table[idx]) for idx, wt in corners(desc, x, coords)]
    return np.concatenate(feats, axis=1)


def encode(desc, params, rays, coords="exact"):
    """The MLP input [N, D] of rays [6, N]: position code then direction code."""
    r = np.asarray(rays, dtype=np.float64)
    table, _ = split(desc, params)
    pos = encode_position(desc, table, np.asarray(rays)[0:3].T, coords)
    return np.concatenate([pos, O.encode(r[3:6].T, desc.dir_bands)], axis=1)


# ----------------------------------------------------------------------------
# Field, loss, gradient
# ----------------------------------------------------------------------------

def mlp_forward(mlp, g):
    hs = [g]
    h = g
    for W, b in mlp[:-1]:
        h = np.maximum(h @ W.T + b, 0.0)
        hs.append(h)
    Wh, bh = mlp[-1]
    return hs, h @ Wh.T + bh


def hash_query(desc, params, rays, coords="exact"):
    """(t, xi, z_t, z_xi) per ray [6, N]."""
    _, mlp = split(desc, params)
    _, z = mlp_forward(mlp, encode(desc, params, rays, coords))
    return O.softplus(z[:, 0]), O.sigmoid(z[:, 1]), z[:, 0], z[:, 1]


def backward(desc, params, rays, dz, coords="exact"):
    """Gradient of sum(dz * z) with respect to every parameter (flat, float64)."""
    table, mlp = split(desc, params)
    r = np.asarray(rays, dtype=np.float64)
    g = encode(desc, params, rays, coords)
    hs, _ = mlp_forward(mlp, g)
    grads = []
    delta = np.asarray(dz, dtype=np.float64)
    for li in range(len(mlp) - 1, -1, -1):
        W, _ = mlp[li]
        grads.append((delta.T @ hs[li], delta.sum(axis=0)))
        delta = delta @ W
        if li > 0:
            delta = delta * (hs[li] > 0)
    grads.reverse()
    # delta is now dL/dg; the position part scatters to the table with the lookup weights
    gtab = np.zeros_like(table)
    F = desc.n_feat
    for l, (idx, wt) in enumerate(corners(desc, np.asarray(rays)[0:3].T, coords)):
        dfeat = delta[:, l * F:(l + 1) * F]
        for k in range(8):
            np.add.at(gtab, idx[:, k], wt[:, k, None] * dfeat)
    return np.concatenate([gtab.ravel()] + [np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def loss_and_grad(desc, params, rays, t_gt, hit, coords="exact"):
    """Distillation loss (the same terms as the sinusoidal field) and its gradient."""
    _, _, zt, zx = hash_query(desc, params, rays, coords)
    terms, dzt, dzx = O.loss_terms(zt, zx, t_gt, hit)
    return terms, backward(desc, params, rays, np.stack([dzt, dzx], axis=1), coords)

"""Plain float64 oracle of the training-ray sampler (the batches the field is distilled on).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP path and imports nothing
from it.

What is computed (Sec. III-B: the field learns from rays that start on the surface and
point in every direction, for the secondary visibility shadows and AO need, and from rays
of the views it is rendered from; the batches of Sec. III-D):

* A surface ray: a primitive k chosen with probability proportional to its surface area,
  a point p = c_k + R_k (a_k * s) with s uniform on the unit sphere, the outward normal
  n = R_k (s / a_k) normalised; origin p + offset n; direction uniform on the sphere.
* A free ray: an origin uniform in the box [-h, h]^3, direction uniform on the sphere.
* A candidate point inside another primitive (a surface point) or inside any primitive (a
  free origin) is rejected and the next candidate taken; after `tries` rejections the last
  candidate is kept.
* Mixed batches (mode 2) put surface rays at even and free rays at odd positions.

Readings where the paper is silent (each also listed in the design notes):
* Free rays stand in for camera rays (the scene has no cameras of its own).
* The surface area of an ellipsoid is Knud Thomsen's approximation
  4 pi ((a^p b^p + a^p c^p + b^p c^p) / 3)^(1/p), p = 1.6075 (exact for spheres, within
  about 1.1 % otherwise); the point density on a primitive is uniform in s, not in area.
* Uniforms are inputs, u [3 tries + 2, n]: rows 3j .. 3j + 2 drive candidate j (primitive
  choice and sphere point for a surface ray, the three coordinates for a free ray), the last
  two the direction.  The primitive is the first index whose cumulative weight exceeds u.
  A sphere point from (u1, u2): z = 1 - 2 u1, phi = 2 pi u2.
* "Inside" is strictly inside: |R^T (x - c) / a|^2 < 1.
"""
from __future__ import annotations

import math

import numpy as np

THOMSEN_P = 1.6075


def ellipsoid_area(axes):
    """Approximate surface areas of ellipsoids with semi-axes axes [P, 3]."""
    a = np.asarray(axes, dtype=np.float64) ** THOMSEN_P
    m = (a[:, 0] * a[:, 1] + a[:, 0] * a[:, 2] + a[:, 1] * a[:, 2]) / 3.0
    return 4.0 * math.pi * m ** (1.0 / THOMSEN_P)


def area_cdf(scene):
    w = ellipsoid_area(scene.axes)
    c = np.cumsum(w)
    return c / c[-1]


def sphere_point(u1, u2):
    z = 1.0 - 2.0 * np.asarray(u1, dtype=np.float64)
    phi = 2.0 * math.pi * np.asarray(u2, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=-1)


def implicit(scene, x):
    """|R^T (x - c) / a|^2 - 1 per point and primitive, [N, P]."""
    c = np.asarray(scene.centers, dtype=np.float64)
    a = np.asarray(scene.axes, dtype=np.float64)
    R = np.asarray(scene.rot, dtype=np.float64)
    q = np.einsum('pji,npj->npi', R, np.asarray(x, dtype=np.float64)[:, None, :] - c[None]) / a[None]
    return np.einsum('npi,npi->np', q, q) - 1.0


def sample_rays(scene, u, mode, box_half, offset, tries):
    """(rays [n, 6] float64, chosen try [n], margin [n]).  margin is the smallest |implicit|
    over every inside test the ray's accepted-or-last candidate and its rejected
    predecessors went through (how close a float32 test comes to deciding otherwise), and
    the distance of each primitive draw from a cumulative-weight boundary."""
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[1]
    assert u.shape[0] == 3 * tries + 2
    c = np.asarray(scene.centers, dtype=np.float64)
    a = np.asarray(scene.axes, dtype=np.float64)
    R = np.asarray(scene.rot, dtype=np.float64)
    cdf = area_cdf(scene)
    P = len(c)
    idx = np.arange(n)
    surf = np.zeros(n, dtype=bool) if mode == 1 else (np.ones(n, dtype=bool) if mode == 0 else
                                                      (idx % 2 == 0) & (idx < 2 * (n // 2)))
    origin = np.zeros((n, 3))
    chosen = np.full(n, tries - 1)
    margin = np.full(n, np.inf)
    done = np.zeros(n, dtype=bool)
    for j in range(tries):
        # surface candidates
        k = np.minimum(np.searchsorted(cdf, u[3 * j], side='right'), P - 1)
        s = sphere_point(u[3 * j + 1], u[3 * j + 2])
        p = c[k] + np.einsum('nij,nj->ni', R[k], a[k] * s)
        nr = np.einsum('nij,nj->ni', R[k], s / a[k])
        nr /= np.linalg.norm(nr, axis=1, keepdims=True)
        # free candidates
        x = -box_half + 2.0 * box_half * u[3 * j:3 * j + 3].T
        cand = np.where(surf[:, None], p + offset * nr, x)
        F = implicit(scene, np.where(surf[:, None], p, x))
        own = np.zeros((n, P), dtype=bool)
        own[np.arange(n), k] = True
        F_test = np.where(surf[:, None] & own, np.inf, F)
        inside = (F_test < 0).any(axis=1)
        live = ~done
        m = np.abs(F_test).min(axis=1)
        mk = np.min(np.abs(cdf[None, :] - u[3 * j][:, None]), axis=1)
        margin[live] = np.minimum(margin[live], np.where(surf[live], np.minimum(m[live], mk[live]), m[live]))
        take = live & (~inside | (j == tries - 1))
        origin[take] = cand[take]
        chosen[take & ~inside] = j
        done |= take
    d = sphere_point(u[3 * tries], u[3 * tries + 1])
    return np.concatenate([origin, d], axis=1), chosen, margin

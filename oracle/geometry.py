"""Exact ray casting and signed distances on analytic scenes (float64).

TEST INFRASTRUCTURE.  This is the oracle's ground truth, a slow and plain
reference.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the HIP product path never does.

The paper supervises its field with exact distances from ray casting a
ground-truth surface (Sec. III-B, the upper-bound supervision source).  Here
the surface is a union of spheres and ellipsoids, so the first hit has a
closed form: for the primitive {c + R (a * u) : |u| <= 1} the ray x + t d is
mapped into the primitive's unit-sphere frame, q = R^T (x - c) / a and
e = R^T d / a, and the first hit solves |q + t e|^2 = 1, a quadratic
A t^2 + 2 B t + C = 0 with A = e.e, B = q.e, C = q.q - 1.

Conventions (readings where the paper is silent):
* The first hit is the smallest root strictly greater than 0 over all
  primitives; a tangent ray (zero discriminant) hits; an origin inside a
  primitive hits at that primitive's exit root.
* A miss has t = +inf and hit = False.
* The signed distance of the union is the minimum over primitives of an
  exact (sphere) or lower-bound (ellipsoid) distance:
  sphere |p - c| - r; ellipsoid (|R^T (p - c) / a| - 1) * min(a).
"""
from __future__ import annotations

import numpy as np


def _prim_arrays(scene):
    c = np.asarray(scene.centers, dtype=np.float64)
    a = np.asarray(scene.axes, dtype=np.float64)
    R = np.asarray(scene.rot, dtype=np.float64)
    return c, a, R


def intersect(scene, origins, dirs, chunk=2048):
    """First hit along each ray.

    origins, dirs: [N, 3] (promoted to float64; dirs need not be unit length,
    t is then measured in units of |d|).  Returns (t [N] float64 with inf on a
    miss, hit [N] bool, prim [N] int64 with -1 on a miss)."""
    o = np.asarray(origins, dtype=np.float64)
    d = np.asarray(dirs, dtype=np.float64)
    c, a, R = _prim_arrays(scene)
    n = len(o)
    t_best = np.full(n, np.inf)
    prim = np.full(n, -1, dtype=np.int64)
    for s in range(0, n, chunk):
        oo = o[s:s + chunk]; dd = d[s:s + chunk]
        # local frame: rows are rays, middle axis primitives
        q = np.einsum('pji,npj->npi', R, oo[:, None, :] - c[None]) / a[None]
        e = np.einsum('pji,nj->npi', R, dd) / a[None]
        A = np.einsum('npi,npi->np', e, e)
        B = np.einsum('npi,npi->np', q, e)
        C = np.einsum('npi,npi->np', q, q) - 1.0
        disc = B * B - A * C
        ok = disc >= 0.0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        # numerically stable pair of roots: k = -(B + sign(B) sqrt(disc))
        sgn = np.where(B >= 0.0, 1.0, -1.0)
        k = -(B + sgn * sq)
        with np.errstate(divide='ignore', invalid='ignore'):
            r1 = k / A
            r2 = np.where(k != 0.0, C / k, -B / A)
        lo = np.minimum(r1, r2)
        hi = np.maximum(r1, r2)
        t = np.where(lo > 0.0, lo, np.where(hi > 0.0, hi, np.inf))
        t = np.where(ok, t, np.inf)
        j = np.argmin(t, axis=1)
        tb = t[np.arange(len(t)), j]
        t_best[s:s + chunk] = tb
        prim[s:s + chunk] = np.where(np.isfinite(tb), j, -1)
    return t_best, np.isfinite(t_best), prim


def intersect_soa(scene, rays):
    """intersect() on a float32 [6, N] SoA ray array (promoted exactly)."""
    r = np.asarray(rays, dtype=np.float64)
    return intersect(scene, r[0:3].T, r[3:6].T)


def implicit(scene, p):
    """Per-primitive implicit value |R^T (p - c) / a|^2 - 1, [N, P] (zero on the surface)."""
    c, a, R = _prim_arrays(scene)
    p = np.asarray(p, dtype=np.float64)
    q = np.einsum('pji,npj->npi', R, p[:, None, :] - c[None]) / a[None]
    return np.einsum('npi,npi->np', q, q) - 1.0


def sdf(scene, p, chunk=4096):
    """Signed distance bound of the union at points p [N, 3] (float64)."""
    c, a, R = _prim_arrays(scene)
    p = np.asarray(p, dtype=np.float64)
    out = np.empty(len(p))
    amin = a.min(axis=1)
    for s in range(0, len(p), chunk):
        q = np.einsum('pji,npj->npi', R, p[s:s + chunk, None, :] - c[None]) / a[None]
        out[s:s + chunk] = np.min((np.sqrt(np.einsum('npi,npi->np', q, q)) - 1.0) * amin[None], axis=1)
    return out


def sphere_trace(sdf_fn, origins, dirs, max_steps=128, hit_eps=1e-4, t_max=6.0):
    """Sphere tracing (the paper's SDF baseline, Sec. IV-D / Table IV).

    Starting at t = 0, each step evaluates s = sdf(x + t d); |s| < hit_eps is a
    hit (t kept), otherwise t <- t + s; t > t_max is a miss.  A ray that has
    neither hit nor left after max_steps evaluations is a miss that did not
    converge.  Returns (t, hit, steps, converged) with steps = number of SDF
    evaluations the ray used.  sdf_fn maps [M, 3] float64 points to [M]."""
    o = np.asarray(origins, dtype=np.float64)
    d = np.asarray(dirs, dtype=np.float64)
    n = len(o)
    t = np.zeros(n)
    hit = np.zeros(n, dtype=bool)
    done = np.zeros(n, dtype=bool)
    steps = np.zeros(n, dtype=np.int64)
    for _ in range(max_steps):
        act = np.nonzero(~done)[0]
        if act.size == 0:
            break
        s = sdf_fn(o[act] + t[act, None] * d[act])
        steps[act] += 1
        h = np.abs(s) < hit_eps
        hit[act[h]] = True
        done[act[h]] = True
        mv = act[~h]
        t[mv] = t[mv] + s[~h]
        gone = mv[t[mv] > t_max]
        done[gone] = True
    return t, hit, steps, done

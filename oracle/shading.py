"""Plain float64 oracle of the DDF's shading consumers: shadow and ambient occlusion maps.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP path and imports nothing
from it.

What is computed (Sec. III-C, the queries a renderer sends; Sec. IV-F, shadows and
ambient occlusion compared with a reference ray tracer, Table VI):

* Primary visibility comes from the exact geometry (a pinhole camera and the analytic
  scene): only the secondary-ray oracle differs between a DDF render and the reference,
  as in the paper's comparison.  Each pixel keeps its first hit point p and the outward
  unit normal n there.
* Shadow: the point is lifted along its normal, o = p + offset n, and one ray goes from o
  toward the point light; the pixel is in shadow when that ray hits something closer
  than the light.
* Ambient occlusion: K rays from o over the hemisphere around n; the pixel's value is the
  mean of their hit flags (within ao_radius).
* The field answers (t, xi); a ray counts as hitting when xi > 0.5.  The reference
  answers with the exact first hit (xi = 1 on a hit, 0 on a miss).
* One bounce of global illumination (Sec. I: a bounce query asks what a surface point sees
  in some direction): the pixel's K hemisphere rays are cosine-weighted, so for a diffuse
  surface each carries the same weight, and the bounce term is the mean over them of the
  radiance each ray sees: the surface radiance at its hit point o + t d when it hits, the sky
  when it misses.
* Error measures over the pixels with a primary hit: PSNR = 10 log10(1 / MSE) of maps in
  [0, 1], and the mean absolute error of the AO map.

Readings where the paper is silent (each also listed in the design notes):
* Camera: pinhole, square pixels sampled at their centres, row 0 at the top;
  s_x = (2 (i + 0.5) / W - 1) tan(fov_y / 2) W / H, s_y = (1 - 2 (j + 0.5) / H) tan(fov_y / 2),
  direction normalise(f + s_x r + s_y u) with f the view direction, r = normalise(f x up)
  and u = r x f.
* AO directions are cosine-weighted (Malley's method: a uniform point of the unit disk,
  r = sqrt(u1), phi = 2 pi u2, lifted to the hemisphere) in the orthonormal basis of
  Duff et al. (2017) around n; the uniforms are inputs.
* Hit threshold xi > 0.5; shadow when t < |light - o|; AO counts hits with t < ao_radius
  (infinite: every hit).
* Background pixels (no primary hit) get shadow 0 and AO 0 and are left out of the
  error measures.
* The scene's outgoing surface radiance is given as values at the vertices of a res^3 grid
  over the object box [-h, h]^3 (a stand-in for the appearance a renderer would read at the
  hit point; the paper's renderer reads the Gaussians there), interpolated trilinearly, a
  point outside the box clamped to it; the sky seen by a missing ray of direction d is
  sky_lo + (sky_hi - sky_lo) (d_y + 1) / 2.  Background pixels get a bounce term of 0.
"""
from __future__ import annotations

import numpy as np

from oracle import geometry as G


def camera_rays(eye, target, up, fov_y, width, height):
    """(origins [P, 3], unit directions [P, 3]) of the W x H pixel centres, row-major."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = np.tan(fov_y / 2)
    i = np.arange(width)
    j = np.arange(height)
    sx = (2 * (i + 0.5) / width - 1) * th * width / height
    sy = (1 - 2 * (j + 0.5) / height) * th
    d = f[None, None] + sx[None, :, None] * r[None, None] + sy[:, None, None] * u[None, None]
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.repeat(eye[None], len(d), axis=0), d


def normals(scene, prim, points):
    """Outward unit normal of primitive prim[k] at points[k] (on its surface): the gradient
    of |R^T (x - c) / a|^2, proportional to R (q / a) with q = R^T (x - c) / a."""
    c = np.asarray(scene.centers, dtype=np.float64)[prim]
    a = np.asarray(scene.axes, dtype=np.float64)[prim]
    R = np.asarray(scene.rot, dtype=np.float64)[prim]
    q = np.einsum('kji,kj->ki', R, points - c) / a
    n = np.einsum('kij,kj->ki', R, q / a)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def gbuffer(scene, eye, target, up, fov_y, width, height):
    """(points [P, 3], normals [P, 3], hit [P], margin [P]) of the primary rays.  margin is
    the smallest |disc| / A^2 over all primitives: the squared half-chord (in the
    primitive's unit-sphere frame) of the closest-to-tangent crossing, 0 for a tangent ray.
    Pixels with a small margin are numerically ambiguous (a float32 cast may decide them
    either way)."""
    o, d = camera_rays(eye, target, up, fov_y, width, height)
    t, hit, prim = G.intersect(scene, o, d)
    p = np.zeros_like(o)
    n = np.zeros_like(o)
    p[hit] = o[hit] + t[hit, None] * d[hit]
    n[hit] = normals(scene, prim[hit], p[hit])
    return p, n, hit, _margin(scene, o, d)


def _margin(scene, o, d):
    c = np.asarray(scene.centers, dtype=np.float64)
    a = np.asarray(scene.axes, dtype=np.float64)
    R = np.asarray(scene.rot, dtype=np.float64)
    q = np.einsum('pji,npj->npi', R, o[:, None, :] - c[None]) / a[None]
    e = np.einsum('pji,nj->npi', R, d) / a[None]
    A = np.einsum('npi,npi->np', e, e)
    B = np.einsum('npi,npi->np', q, e)
    C = np.einsum('npi,npi->np', q, q) - 1.0
    return (np.abs(B * B - A * C) / (A * A)).min(axis=1)


def basis(n):
    """Orthonormal (t, b) with t x b = n (Duff et al. 2017, branchless)."""
    sign = np.where(n[:, 2] >= 0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = np.stack([1 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]], axis=1)
    bb = np.stack([b, sign + n[:, 1] ** 2 * a, -n[:, 1]], axis=1)
    return t, bb


def secondary_rays(points, nrm, light, n_ao, u, offset):
    """Rays [P (1 + K), 6] (origin, unit direction), pixel-major: the shadow ray, then the K
    AO rays from uniforms u [2, P K].  Background pixels are passed as given (any point and
    unit normal); their rays are never read back."""
    p = np.asarray(points, dtype=np.float64)
    n = np.asarray(nrm, dtype=np.float64)
    P = len(p)
    o = p + offset * n
    ds = np.asarray(light, dtype=np.float64)[None] - o
    ds /= np.linalg.norm(ds, axis=1, keepdims=True)
    u = np.asarray(u, dtype=np.float64).reshape(2, P, n_ao)
    r = np.sqrt(u[0])
    phi = 2 * np.pi * u[1]
    lx, ly, lz = r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1 - u[0]))
    t, b = basis(n)
    da = lx[..., None] * t[:, None] + ly[..., None] * b[:, None] + lz[..., None] * n[:, None]
    da /= np.linalg.norm(da, axis=2, keepdims=True)
    d = np.concatenate([ds[:, None], da], axis=1)
    oo = np.repeat(o[:, None], 1 + n_ao, axis=1)
    return np.concatenate([oo, d], axis=2).reshape(P * (1 + n_ao), 6)


def shade(t, hitflag, points, nrm, hit, light, n_ao, offset, ao_radius=np.inf):
    """(shadow [P], ao [P]) from the answers to the secondary rays: t [P (1 + K)] and a
    boolean hit flag per ray (xi > 0.5 for the field, the exact hit for the reference)."""
    P = len(points)
    t = np.asarray(t, dtype=np.float64).reshape(P, 1 + n_ao)
    f = np.asarray(hitflag, dtype=bool).reshape(P, 1 + n_ao)
    o = np.asarray(points, dtype=np.float64) + offset * np.asarray(nrm, dtype=np.float64)
    dist = np.linalg.norm(np.asarray(light, dtype=np.float64)[None] - o, axis=1)
    shadow = (f[:, 0] & (t[:, 0] < dist)).astype(np.float64)
    ao = (f[:, 1:] & (t[:, 1:] < ao_radius)).mean(axis=1) if n_ao > 0 else np.zeros(P)
    hit = np.asarray(hit, dtype=bool)
    return np.where(hit, shadow, 0.0), np.where(hit, ao, 0.0)


def reference(scene, points, nrm, hit, light, n_ao, u, offset, ao_radius=np.inf):
    """The reference maps: the same secondary rays answered by exact ray casting."""
    rays = secondary_rays(points, nrm, light, n_ao, u, offset)
    t, h, _ = G.intersect(scene, rays[:, 0:3], rays[:, 3:6])
    return shade(t, h, points, nrm, hit, light, n_ao, offset, ao_radius)


def psnr(a, b, mask):
    """10 log10(1 / MSE) over the masked pixels (maps in [0, 1]); inf when equal."""
    m = np.asarray(mask, dtype=bool)
    mse = float(np.mean((np.asarray(a, dtype=np.float64)[m] - np.asarray(b, dtype=np.float64)[m]) ** 2))
    return np.inf if mse == 0 else 10 * np.log10(1.0 / mse)


def mae(a, b, mask):
    m = np.asarray(mask, dtype=bool)
    return float(np.mean(np.abs(np.asarray(a, dtype=np.float64)[m] - np.asarray(b, dtype=np.float64)[m])))


def surface_radiance(q, radiance, box_half):
    """Trilinear interpolation of the vertex grid radiance [res, res, res] (indexed [z, y, x])
    at points q [N, 3] of the box [-box_half, box_half]^3 (clamped to it)."""
    R = np.asarray(radiance, dtype=np.float64)
    res = R.shape[0]
    p = np.clip((np.asarray(q, dtype=np.float64) + box_half) / (2 * box_half), 0.0, 1.0)
    s = p * (res - 1)
    c = np.minimum(np.floor(s), res - 2).astype(np.int64)
    w = s - c
    out = np.zeros(len(p))
    for k in range(8):
        dx, dy, dz = k & 1, (k >> 1) & 1, (k >> 2) & 1
        wt = (w[:, 0] if dx else 1 - w[:, 0]) * (w[:, 1] if dy else 1 - w[:, 1]) * (w[:, 2] if dz else 1 - w[:, 2])
        out += wt * R[c[:, 2] + dz, c[:, 1] + dy, c[:, 0] + dx]
    return out


def sky(d, sky_lo, sky_hi):
    """Radiance seen by a ray of unit direction d [N, 3] that hits nothing."""
    return sky_lo + (sky_hi - sky_lo) * (np.asarray(d, dtype=np.float64)[:, 1] + 1.0) / 2.0


def bounce(t, hitflag, rays, hit, n_ao, radiance, box_half, sky_lo, sky_hi):
    """The one-bounce term [P]: per pixel, the mean over its K hemisphere rays (rays
    [P (1 + K), 6], pixel-major, the shadow ray first and skipped) of the radiance each ray
    sees, surface_radiance(o + t d) on a hit, sky(d) on a miss; 0 for background pixels."""
    hit = np.asarray(hit, dtype=bool)
    P = len(hit)
    if n_ao == 0:
        return np.zeros(P)
    r = np.asarray(rays, dtype=np.float64).reshape(P, 1 + n_ao, 6)[:, 1:].reshape(-1, 6)
    tt = np.asarray(t, dtype=np.float64).reshape(P, 1 + n_ao)[:, 1:].reshape(-1)
    f = np.asarray(hitflag, dtype=bool).reshape(P, 1 + n_ao)[:, 1:].reshape(-1)
    q = r[:, 0:3] + np.where(f, tt, 0.0)[:, None] * r[:, 3:6]
    L = np.where(f, surface_radiance(q, radiance, box_half), sky(r[:, 3:6], sky_lo, sky_hi))
    return np.where(hit, L.reshape(P, n_ao).mean(axis=1), 0.0)


def reference_bounce(scene, rays, hit, n_ao, radiance, box_half, sky_lo, sky_hi):
    """The reference one-bounce map: the same rays answered by exact ray casting."""
    r = np.asarray(rays, dtype=np.float64)
    t, h, _ = G.intersect(scene, r[:, 0:3], r[:, 3:6])
    return bounce(t, h, r, hit, n_ao, radiance, box_half, sky_lo, sky_hi)

"""Pins of the training-ray sampler oracle: the ellipsoid area against numerical
integration, area-proportional primitive choice, points on the surface with outward normals,
uniform directions (Archimedes: z uniform on [-1, 1]), rejection of points inside other
primitives, free origins in the box and outside every primitive, the mixed-batch layout."""
import math

import numpy as np
from scipy import integrate

from oracle import sampling as SM
from paper_2606_00817_amd import inputs as I


def _exact_area(a, b, c):
    """Surface area of the ellipsoid by integrating |dX/dth x dX/dph| over the sphere chart."""
    def f(th, ph):
        st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
        xt = np.array([a * ct * cp, b * ct * sp, -c * st])
        xp = np.array([-a * st * sp, b * st * cp, 0.0])
        return np.linalg.norm(np.cross(xt, xp))
    v, _ = integrate.dblquad(f, 0, 2 * math.pi, 0, math.pi, epsabs=1e-10, epsrel=1e-10)
    return v


def test_ellipsoid_area():
    assert math.isclose(SM.ellipsoid_area([[0.7, 0.7, 0.7]])[0], 4 * math.pi * 0.49, rel_tol=1e-12)
    for ax in ([1.0, 0.5, 0.25], [2.0, 1.0, 1.0], [0.3, 0.3, 0.05], [1.45, 0.02, 1.45]):
        assert abs(SM.ellipsoid_area([ax])[0] / _exact_area(*ax) - 1) < 0.0115


def _two_spheres(r1=1.0, r2=2.0, gap=5.0):
    return I.Scene(np.array([[-gap, 0.0, 0.0], [gap, 0.0, 0.0]]), np.array([[r1] * 3, [r2] * 3]),
                   np.repeat(np.eye(3)[None], 2, axis=0))


def test_area_proportional_choice_and_surface_points():
    sc = _two_spheres()
    n = 20000
    u = I.uniforms(5, n, 3)
    rays, _, _ = SM.sample_rays(sc, u, 0, 10.0, 0.0, 1)
    o = rays[:, 0:3]
    big = o[:, 0] > 0
    assert abs(big.mean() - 0.8) < 5 * math.sqrt(0.16 / n)
    # on the chosen sphere; z of the point uniform on [-r, r]
    r = np.where(big, 2.0, 1.0)
    cx = np.where(big, 5.0, -5.0)
    rel = (o - np.stack([cx, np.zeros(n), np.zeros(n)], 1)) / r[:, None]
    assert np.allclose(np.linalg.norm(rel, axis=1), 1.0)
    assert abs(rel[:, 2].mean()) < 5 * math.sqrt(1 / 3 / n) and abs((rel[:, 2] ** 2).mean() - 1 / 3) < 0.01


def test_normals_and_offset():
    sc = I.scene_ellipsoids(5, 12)
    n = 2000
    u = I.uniforms(5, n, 4)
    off = 1e-3
    r0, _, _ = SM.sample_rays(sc, u, 0, 1.5, 0.0, 1)
    r1, _, _ = SM.sample_rays(sc, u, 0, 1.5, off, 1)
    step = r1[:, 0:3] - r0[:, 0:3]
    assert np.allclose(np.linalg.norm(step, axis=1), off)
    # the step is along the outward normal: moving along it leaves the primitive
    F0 = SM.implicit(sc, r0[:, 0:3]).min(axis=1)
    F1 = SM.implicit(sc, r0[:, 0:3] + 10 * step).min(axis=1)
    on = np.abs(F0) < 1e-9
    assert on.mean() > 0.5 and (F1[on] > 0).all()


def test_uniform_directions():
    n = 50000
    u = I.uniforms(5, n, 5)
    rays, _, _ = SM.sample_rays(_two_spheres(), u, 1, 10.0, 0.0, 1)
    d = rays[:, 3:6]
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    assert np.abs(d.mean(axis=0)).max() < 5 * math.sqrt(1 / 3 / n)
    assert np.abs((d ** 2).mean(axis=0) - 1 / 3).max() < 0.01


def test_rejection_of_points_inside_other_primitives():
    sc = I.Scene(np.array([[0.0, 0.0, 0.0], [0.6, 0.0, 0.0]]), np.array([[1.0] * 3, [0.5] * 3]),
                 np.repeat(np.eye(3)[None], 2, axis=0))
    n = 5000
    T = 8
    u = I.uniforms(3 * T + 2, n, 6)
    rays, chosen, _ = SM.sample_rays(sc, u, 0, 2.0, 0.0, T)
    F = SM.implicit(sc, rays[:, 0:3])
    # every point is on one sphere and not strictly inside the other (8 tries leave ~0.5^8)
    on_a = np.abs(F[:, 0]) < 1e-9
    assert ((on_a & (F[:, 1] >= 0)) | (~on_a & (F[:, 0] >= 0))).mean() > 0.99
    # the part of the small sphere inside the big one is never kept when a later try exists
    assert (F[chosen < T - 1].min(axis=1) > -1e-9).all()


def test_free_origins_and_mixed_layout():
    sc = I.scene_ground(10, 7)
    n = 6001
    T = 4
    u = I.uniforms(3 * T + 2, n, 8)
    rays, chosen, _ = SM.sample_rays(sc, u, 2, 1.5, 1e-3, T)
    o = rays[:, 0:3]
    F = SM.implicit(sc, o)
    free = np.arange(n) % 2 == 1
    free[-1] = True                                  # odd n: the last ray is free
    assert (np.abs(o) <= 1.5).all()
    kept = chosen < T - 1
    assert (F[free & kept] >= 0).all()
    # surface origins sit offset off a surface: within 1e-3 of it, outside every primitive
    sd = np.sqrt(np.maximum(F[~free] + 1, 0)).min(axis=1)
    assert (F[~free & kept].min(axis=1) > 0).all() and np.median(sd) < 1.1

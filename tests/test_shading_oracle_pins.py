"""Pins of the shading oracle (shadow and AO maps, Sec. III-C and IV-F) to closed forms of
simple scenes: camera geometry, hit points and normals, the shadow disk a sphere casts on a
plane, the cosine-weighted occlusion (r / h)^2 a sphere causes above a plane point, no
self-occlusion on a convex object, an occluder behind the light, and the error measures."""
import math

import numpy as np

from oracle import geometry as G
from oracle import shading as S
from paper_2606_00817_amd import inputs as I


def _plane_and_sphere(h, r):
    """A (practically flat) ground slab with its top face at y = 0 and a sphere at (0, h, 0)."""
    return I.Scene(np.array([[0.0, -0.01, 0.0], [0.0, h, 0.0]]),
                   np.array([[60.0, 0.01, 60.0], [r, r, r]]),
                   np.repeat(np.eye(3)[None], 2, axis=0))


def test_camera_geometry():
    fov = math.radians(50.0)
    W, H = 9, 7
    o, d = S.camera_rays((0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fov, W, H)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    d = d.reshape(H, W, 3)
    # the centre pixel looks at the target
    assert np.allclose(d[H // 2, W // 2], [0.0, 0.0, -1.0])
    # the centre column's top and bottom pixel centres are (1 - 1/H) of the half-angle's tangent
    # away from the axis, on either side
    ang = math.acos(float(np.dot(d[0, W // 2], d[H - 1, W // 2])))
    assert abs(ang - 2 * math.atan((1 - 1 / H) * math.tan(fov / 2))) < 1e-12
    # row 0 is the top (+y), column W - 1 the right (+x when looking down -z with y up)
    assert d[0, W // 2, 1] > 0 and d[H // 2, W - 1, 0] > 0
    # square pixels: neighbouring centres are equally far apart horizontally and vertically
    assert abs(d[H // 2, W // 2 + 1, 0] / d[H // 2, W // 2 + 1, 2] + d[H // 2 + 1, W // 2, 1] / d[H // 2 + 1, W // 2, 2]) < 1e-12


def test_gbuffer_sphere_head_on():
    """A sphere of radius r at distance D: the centre pixel hits at D - r with normal -f, and
    the pixels that hit fill the projected disk of angular radius asin(r / D)."""
    D, r = 4.0, 0.8
    sc = I.Scene(np.zeros((1, 3)), np.full((1, 3), r), np.eye(3)[None])
    W = H = 201
    fov = math.radians(40.0)
    p, n, hit, margin = S.gbuffer(sc, (0.0, 0.0, D), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fov, W, H)
    c = (H // 2) * W + W // 2
    assert hit[c] and np.allclose(p[c], [0.0, 0.0, r]) and np.allclose(n[c], [0.0, 0.0, 1.0])
    rho = math.tan(math.asin(r / D)) / math.tan(fov / 2)         # disk radius in half-heights
    expect = math.pi * rho ** 2 / 4 * W * H                       # pixels inside it
    assert abs(hit.sum() - expect) < 2 * math.pi * rho * W / 2 * 1.5   # within the boundary ring
    # hit points lie on the sphere, normals are radial; the margin is small only on the rim
    assert np.allclose(np.linalg.norm(p[hit], axis=1), r)
    assert np.allclose(n[hit], p[hit] / r)
    assert margin[c] > 0.5


def test_normals_are_implicit_gradients():
    """Ellipsoid normals against a central-difference gradient of the implicit function."""
    sc = I.scene_ellipsoids(6, 77)
    rng = np.random.default_rng(3)
    o = rng.uniform(-1, 1, (400, 3)) * 2.5
    d = -o + rng.normal(0, 0.3, o.shape)
    t, hit, prim = G.intersect(sc, o, d)
    pts = o[hit] + t[hit, None] * d[hit]
    n = S.normals(sc, prim[hit], pts)
    h = 1e-6
    g = np.zeros_like(pts)
    for a in range(3):
        e = np.zeros(3); e[a] = h
        for k, pk in enumerate(prim[hit]):
            one = I.Scene(sc.centers[pk:pk + 1], sc.axes[pk:pk + 1], sc.rot[pk:pk + 1])
            g[k, a] = (G.implicit(one, pts[k:k + 1] + e)[0, 0] - G.implicit(one, pts[k:k + 1] - e)[0, 0]) / (2 * h)
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    assert np.abs(n - g).max() < 1e-5
    # outward: the normal points away from the primitive's centre side
    assert (np.einsum('ki,ki->k', n, pts - sc.centers[prim[hit]]) > 0).all()


def test_shadow_disk_of_a_sphere():
    """Ground points whose segment to the light passes within r of the sphere's centre are in
    shadow (point-to-line distance, computed independently), the others lit."""
    h, r, Ly = 1.0, 0.3, 3.0
    sc = _plane_and_sphere(h, r)
    light = (0.0, Ly, 0.0)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.0, 0.8, 400)
    phi = rng.uniform(0, 2 * math.pi, 400)
    p = np.stack([rho * np.cos(phi), np.zeros(400), rho * np.sin(phi)], 1)
    nrm = np.tile([0.0, 1.0, 0.0], (400, 1))
    off = 1e-4
    o = p + off * nrm
    L = np.asarray(light)[None] - o
    cvec = np.array([0.0, h, 0.0])[None] - o
    dist = np.linalg.norm(np.cross(cvec, L), axis=1) / np.linalg.norm(L, axis=1)
    keep = np.abs(dist - r) > 1e-6
    sh, _ = S.reference(sc, p, nrm, np.ones(400, bool), light, 0, np.zeros((2, 0)), off)
    assert np.array_equal(sh[keep] == 1.0, dist[keep] < r)
    assert 0.1 < sh.mean() < 0.9


def test_ao_of_a_sphere_above_a_plane_point():
    """Cosine-weighted occlusion of a sphere of radius r whose centre is at height h straight
    above the point: the cap of half-angle asin(r / h) around the normal blocks sin^2 = (r / h)^2."""
    h, r = 1.0, 0.35
    sc = _plane_and_sphere(h, r)
    K = 200000
    u = I.uniforms(2, K, 91).astype(np.float64)
    off = 1e-9
    _, ao = S.reference(sc, np.zeros((1, 3)), np.array([[0.0, 1.0, 0.0]]), np.ones(1, bool), (5.0, 5.0, 5.0), K,
                        u, off)
    p = (r / (h - off)) ** 2
    assert abs(ao[0] - p) < 5 * math.sqrt(p * (1 - p) / K)


def test_no_self_occlusion_on_a_convex_object():
    sc = I.Scene(np.zeros((1, 3)), np.array([[0.5, 0.3, 0.2]]), I._random_rotations(np.random.default_rng(1), 1))
    p, nrm = I.surface_points(sc, 300, 8)
    u = I.uniforms(2, 300 * 8, 9)
    sh, ao = S.reference(sc, p, nrm, np.ones(300, bool), (0.0, 3.0, 0.0), 8, u, 1e-4)
    assert ao.max() == 0.0
    # the lit side sees the light, the far side is shadowed by the object itself (away from
    # the terminator, where the lifted origin decides)
    L = np.array([[0.0, 3.0, 0.0]]) - p
    c = np.einsum('ki,ki->k', nrm, L / np.linalg.norm(L, axis=1, keepdims=True))
    assert (sh[c > 0.05] == 0).all() and (sh[c < -0.05] == 1).all()


def test_occluder_beyond_the_light_casts_no_shadow():
    h, r = 3.0, 0.3
    sc = _plane_and_sphere(h, r)
    p = np.zeros((1, 3)); nrm = np.array([[0.0, 1.0, 0.0]])
    sh_below, _ = S.reference(sc, p, nrm, np.ones(1, bool), (0.0, 2.0, 0.0), 0, np.zeros((2, 0)), 1e-4)
    sh_above, _ = S.reference(sc, p, nrm, np.ones(1, bool), (0.0, 4.0, 0.0), 0, np.zeros((2, 0)), 1e-4)
    assert sh_below[0] == 0.0 and sh_above[0] == 1.0
    # a background pixel gets nothing whatever its rays say
    sh, ao = S.shade(np.zeros(3), np.ones(3, bool), p, nrm, np.zeros(1, bool), (0.0, 4.0, 0.0), 2, 1e-4)
    assert sh[0] == 0.0 and ao[0] == 0.0


def test_error_measures():
    a = np.array([0.0, 1.0, 0.5, 0.25])
    b = np.array([0.0, 0.0, 0.5, 0.75])
    m = np.array([True, True, True, False])
    assert math.isclose(S.psnr(a, b, m), 10 * math.log10(3.0))   # MSE 1/3
    assert S.psnr(a, a, m) == np.inf
    assert math.isclose(S.mae(a, b, m), 1 / 3)


def test_secondary_rays_layout():
    """Shadow ray first, aimed at the light; AO rays unit, in the normal's hemisphere, their
    cosine with the normal equal to sqrt(1 - u1)."""
    sc = I.scene_ground(8, 5)
    p, nrm = I.surface_points(sc, 50, 6)
    K = 4
    u = I.uniforms(2, 50 * K, 7).astype(np.float64)
    rays = S.secondary_rays(p, nrm, I.SHADE_LIGHT, K, u, 1e-3).reshape(50, 1 + K, 6)
    o = p + 1e-3 * nrm
    assert np.allclose(rays[:, :, 0:3], o[:, None])
    to_light = np.asarray(I.SHADE_LIGHT)[None] - o
    assert np.allclose(rays[:, 0, 3:6], to_light / np.linalg.norm(to_light, axis=1, keepdims=True))
    ca = np.einsum('pki,pi->pk', rays[:, 1:, 3:6], nrm)
    assert np.allclose(ca, np.sqrt(1 - u[0].reshape(50, K)))
    assert np.allclose(np.linalg.norm(rays[:, :, 3:6], axis=2), 1.0)


# ---- the one-bounce term

def _linear_grid(res, coef):
    """Vertex grid of the linear radiance a + b x + c y + d z over the box ([z][y][x])."""
    g = np.linspace(-I.BOX_HALF, I.BOX_HALF, res)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return coef[0] + coef[1] * x + coef[2] * y + coef[3] * z


def test_surface_radiance_reproduces_a_linear_field_and_clamps():
    """Trilinear interpolation is exact for a linear field; a point outside the box reads the
    value on the box face nearest to it (the clamp)."""
    coef = (0.5, 0.1, -0.05, 0.02)
    R = _linear_grid(7, coef)
    rng = np.random.default_rng(3)
    q = rng.uniform(-I.BOX_HALF, I.BOX_HALF, (500, 3))
    ref = coef[0] + q @ np.array(coef[1:])
    np.testing.assert_allclose(S.surface_radiance(q, R, I.BOX_HALF), ref, atol=1e-13)
    out = np.array([[2.5, 0.3, -0.2], [-9.0, -9.0, 9.0]])
    cl = np.clip(out, -I.BOX_HALF, I.BOX_HALF)
    np.testing.assert_allclose(S.surface_radiance(out, R, I.BOX_HALF), coef[0] + cl @ np.array(coef[1:]), atol=1e-13)


def test_bounce_sees_the_hit_point_or_the_sky():
    """A pixel whose two hemisphere rays are cast exactly: one hits a sphere head on at a known
    point (radiance of the linear field there), one escapes straight up (the zenith sky)."""
    coef = (0.4, 0.1, 0.2, -0.3)
    R = _linear_grid(5, coef)
    sc = I.Scene(np.array([[0.0, 0.0, 0.5]]), np.array([[0.25, 0.25, 0.25]]), np.eye(3)[None])
    # pixel-major rays of one pixel: a shadow ray (skipped), then the two hemisphere rays
    rays = np.array([[0, 0, -1.0, 0, 1, 0],        # shadow ray (ignored by the bounce term)
                     [0, 0, -1.0, 0, 0, 1],        # hits the sphere at (0, 0, 0.25)
                     [0, 0, -1.0, 0, 1, 0]])       # misses: zenith
    lo, hi = 0.2, 1.0
    gi = S.reference_bounce(sc, rays, np.ones(1, bool), 2, R, I.BOX_HALF, lo, hi)
    expect = 0.5 * ((coef[0] + coef[3] * 0.25) + hi)
    assert abs(gi[0] - expect) < 1e-12
    # a background pixel gets 0; with no hemisphere rays the term is 0
    assert S.reference_bounce(sc, rays, np.zeros(1, bool), 2, R, I.BOX_HALF, lo, hi)[0] == 0.0
    assert S.bounce(np.zeros(1), np.zeros(1, bool), rays[:1], np.ones(1, bool), 0, R, I.BOX_HALF, lo, hi)[0] == 0.0


def test_bounce_under_an_open_sky():
    """A horizontal point with nothing above it: the cosine-weighted mean of the sky gradient is
    lo + (hi - lo) (E[d_y] + 1) / 2 with E[d_y] = 2/3 over the cosine-weighted hemisphere, so
    the bounce term is lo + (5/6) (hi - lo); the oracle's own secondary rays (Malley) get there
    within Monte Carlo error."""
    K = 200000
    u = I.uniforms(2, K, 92).astype(np.float64)
    sc = I.Scene(np.array([[0.0, -5.0, 0.0]]), np.array([[0.1, 0.1, 0.1]]), np.eye(3)[None])   # below: never hit
    rays = S.secondary_rays(np.zeros((1, 3)), np.array([[0.0, 1.0, 0.0]]), (0.0, 3.0, 0.0), K, u, 1e-3)
    lo, hi = 0.2, 1.0
    gi = S.reference_bounce(sc, rays, np.ones(1, bool), K, np.zeros((2, 2, 2)), I.BOX_HALF, lo, hi)
    # d_y = sqrt(1 - u1) under Malley's method: variance of (hi - lo) d_y / 2 over the hemisphere
    sd = (hi - lo) / 2 * math.sqrt(1 / 2 - 4 / 9)
    assert abs(gi[0] - (lo + 5 / 6 * (hi - lo))) < 5 * sd / math.sqrt(K)


def test_bounce_constant_radiance_and_full_occlusion():
    """A point at the centre of a closed sphere sees the surface in every direction: with a
    constant radiance c the bounce term is exactly c."""
    sc = I.Scene(np.zeros((1, 3)), np.array([[1.2, 1.2, 1.2]]), np.eye(3)[None])
    K = 64
    u = I.uniforms(2, K, 93).astype(np.float64)
    rays = S.secondary_rays(np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), (0.0, 0.5, 0.0), K, u, 0.0)
    gi = S.reference_bounce(sc, rays, np.ones(1, bool), K, np.full((3, 3, 3), 0.37), I.BOX_HALF, 0.0, 1.0)
    assert abs(gi[0] - 0.37) < 1e-12

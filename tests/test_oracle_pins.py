"""Pins of the float64 oracle against facts that do not come from the oracle itself.

Each test checks one part of the oracle against a closed form, an invariant,
a special case that reduces to something known, a library routine, or brute
force on a tiny input, chosen so that a plausible slip (a dropped term, a
swapped sin/cos, a wrong sign or index, a transposed operand) fails."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import ddf_oracle as O
from oracle import geometry as G
from paper_2606_00817_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- encoding

def test_encode_dyadic_closed_form():
    # sin(pi 2^k v) and cos(pi 2^k v) at dyadic v are exact table values.
    v = np.array([[0.25, 0.5, 1.5, -0.5, 0.0, 1.0]])
    g = O.encode(v, 4)
    assert g.shape == (1, 6 * 9)
    r2 = math.sqrt(0.5)
    # rows: block (identity, then sin k=0, cos k=0, sin k=1, ...), columns: the 6 coordinates
    expect = np.array([
        [0.25, 0.5, 1.5, -0.5, 0.0, 1.0],       # v
        [r2, 1.0, -1.0, -1.0, 0.0, 0.0],         # sin(pi v)
        [r2, 0.0, 0.0, 0.0, 1.0, -1.0],          # cos(pi v)
        [1.0, 0.0, 0.0, 0.0, 0.0, 0.0],          # sin(2 pi v)
        [0.0, -1.0, -1.0, -1.0, 1.0, 1.0],       # cos(2 pi v)
        [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],          # sin(4 pi v)
        [-1.0, 1.0, 1.0, 1.0, 1.0, 1.0],         # cos(4 pi v)
        [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],          # sin(8 pi v)
        [1.0, 1.0, 1.0, 1.0, 1.0, 1.0],          # cos(8 pi v)
    ]).ravel()
    np.testing.assert_allclose(g[0], expect, atol=1e-12)


def test_encode_periodicity_and_width():
    rng = np.random.default_rng(0)
    v = rng.uniform(-1.5, 1.5, (50, 3))
    g0 = O.encode(v, 10)
    g1 = O.encode(v + 2.0, 10)          # every band has period dividing 2
    assert g0.shape == (50, 63)
    np.testing.assert_allclose(g0[:, 3:], g1[:, 3:], atol=1e-9)
    np.testing.assert_allclose(g1[:, :3] - g0[:, :3], 2.0, atol=1e-12)
    # sin^2 + cos^2 = 1 band by band
    for k in range(10):
        s = g0[:, 3 + 6 * k:6 + 6 * k]; c = g0[:, 6 + 6 * k:9 + 6 * k]
        np.testing.assert_allclose(s * s + c * c, 1.0, atol=1e-12)


# ---------------------------------------------------------------- heads

def test_heads_special_values():
    assert O.softplus(0.0) == pytest.approx(math.log(2.0), abs=1e-15)
    assert O.sigmoid(0.0) == 0.5
    assert O.softplus(50.0) == pytest.approx(50.0 + math.exp(-50.0), rel=1e-15)
    assert O.softplus(-50.0) == pytest.approx(math.exp(-50.0), rel=1e-12)
    assert O.sigmoid(-800.0) >= 0.0 and O.sigmoid(800.0) == 1.0
    z = np.linspace(-20, 20, 101)
    np.testing.assert_allclose(O.sigmoid(z) + O.sigmoid(-z), 1.0, atol=1e-15)
    # softplus' = sigmoid (central difference)
    h = 1e-5
    np.testing.assert_allclose((O.softplus(z + h) - O.softplus(z - h)) / (2 * h), O.sigmoid(z), atol=1e-9)


# ---------------------------------------------------------------- MLP forward

def _brute_forward(desc, params, ray):
    """Pure-Python loops over a single ray (independent of numpy matmul)."""
    v = [float(x) for x in ray]
    feats = list(v)
    for k in range(desc.n_freq):
        feats += [math.sin(math.pi * (2 ** k) * x) for x in v]
        feats += [math.cos(math.pi * (2 ** k) * x) for x in v]
    p = [float(x) for x in params]
    off = 0
    h = feats
    for layer in range(desc.n_hidden + 1):
        n_in = len(h)
        n_out = desc.width if layer < desc.n_hidden else desc.n_out
        W = p[off:off + n_out * n_in]; off += n_out * n_in
        b = p[off:off + n_out]; off += n_out
        a = []
        for o in range(n_out):
            acc = b[o]
            for i in range(n_in):
                acc += W[o * n_in + i] * h[i]
            a.append(acc)
        h = [max(x, 0.0) for x in a] if layer < desc.n_hidden else a
    assert off == len(p)
    return h


def test_mlp_forward_matches_brute_force():
    desc = I.NetDesc(6, 2, 3, 8, 2)
    params = I.test_params(desc, 3, bias_std=0.3)
    rays = I.free_rays(I.scene_spheres(4, 1), 5, 9)
    t, xi, zt, zx = O.ddf_query(desc, params, rays)
    for j in range(5):
        z = _brute_forward(desc, params, rays[:, j])
        assert zt[j] == pytest.approx(z[0], abs=1e-12)
        assert zx[j] == pytest.approx(z[1], abs=1e-12)
        assert t[j] == pytest.approx(math.log1p(math.exp(z[0])), abs=1e-12)
        assert xi[j] == pytest.approx(1.0 / (1.0 + math.exp(-z[1])), abs=1e-12)


def test_mlp_special_case_abs_and_identity():
    # One hidden layer: h0 = relu(x0), h1 = relu(-x0); heads z_t = h0 + h1 = |x0|, z_xi = h0 - h1 = x0.
    desc = I.NetDesc(6, 1, 1, 4, 2)
    D = desc.n_feat
    W1 = np.zeros((4, D)); W1[0, 0] = 1.0; W1[1, 0] = -1.0
    Wh = np.zeros((2, 4)); Wh[0, 0] = Wh[0, 1] = 1.0; Wh[1, 0] = 1.0; Wh[1, 1] = -1.0
    params = np.concatenate([W1.ravel(), np.zeros(4), Wh.ravel(), np.zeros(2)]).astype(np.float32)
    rays = I.free_rays(I.scene_spheres(2, 0), 64, 1)
    t, xi, zt, zx = O.ddf_query(desc, params, rays)
    x0 = rays[0].astype(np.float64)
    np.testing.assert_allclose(zt, np.abs(x0), atol=1e-15)
    np.testing.assert_allclose(zx, x0, atol=1e-15)
    np.testing.assert_allclose(t, np.log1p(np.exp(np.abs(x0))), rtol=1e-14)


# ---------------------------------------------------------------- geometry

def _one(center, axes, rot=None):
    return I.Scene(np.array([center], float), np.array([axes], float),
                   np.array([np.eye(3) if rot is None else rot], float))


def test_intersect_closed_forms():
    unit = _one([0, 0, 0], [1, 1, 1])
    cases = [((0, 0, -5), (0, 0, 1), 4.0),       # head-on
             ((1, 0, -5), (0, 0, 1), 5.0),       # tangent: touches at (1, 0, 0)
             ((0, 0, 0), (0, 0, 1), 1.0),        # inside: exit root
             ((0, 0, 0.5), (0, 0, -1), 1.5),     # inside, pointing back
             ((0, 0, -5), (0, 0, 2), 2.0)]       # non-unit direction: t in units of |d|
    for o, d, t in cases:
        tt, hit, prim = G.intersect(unit, [o], [d])
        assert hit[0] and prim[0] == 0 and tt[0] == pytest.approx(t, abs=1e-12)
    tt, hit, prim = G.intersect(unit, [(0, 0, -5), (1.0001, 0, -5)], [(0, 0, -1), (0, 0, 1)])
    assert not hit.any() and np.all(np.isinf(tt)) and np.all(prim == -1)
    ell = _one([0, 0, 0], [0.5, 1.0, 2.0])
    tt, hit, _ = G.intersect(ell, [(0, 0, -5), (-5, 0, 0), (0, 7, 0)], [(0, 0, 1), (1, 0, 0), (0, -1, 0)])
    np.testing.assert_allclose(tt, [3.0, 4.5, 6.0], atol=1e-12)
    # two spheres along the ray: the nearer one wins
    two = I.Scene(np.array([[0, 0, 0], [0, 0, 3.0]]), np.array([[1, 1, 1], [0.5, 0.5, 0.5]]),
                  np.repeat(np.eye(3)[None], 2, 0))
    tt, hit, prim = G.intersect(two, [(0, 0, 5)], [(0, 0, -1)])
    assert prim[0] == 1 and tt[0] == pytest.approx(1.5, abs=1e-12)


def test_intersect_invariants():
    sc = I.scene_mixed(64, 5)
    rays = I.free_rays(sc, 3000, 6)
    o = rays[0:3].T.astype(np.float64); d = rays[3:6].T.astype(np.float64)
    t, hit, prim = G.intersect(sc, o, d)
    assert hit.mean() > 0.2 and (~hit).mean() > 0.05
    assert np.all(t[hit] > 0)
    # the hit point lies on the hit primitive's surface
    pts = o[hit] + t[hit, None] * d[hit]
    imp = G.implicit(sc, pts)[np.arange(hit.sum()), prim[hit]]
    assert np.max(np.abs(imp)) < 1e-9
    # re-parameterisation along d: t(x + s d) = t(x) - s for 0 <= s < t
    s = 0.5 * np.where(hit, t, 1.0)
    t2, hit2, prim2 = G.intersect(sc, o + s[:, None] * d, d)
    np.testing.assert_array_equal(hit2, hit)
    np.testing.assert_allclose(t2[hit], t[hit] - s[hit], atol=1e-9)
    # rigid-motion invariance
    R = I._random_rotations(np.random.default_rng(1), 1)[0]
    tr = np.array([0.3, -0.2, 0.1])
    moved = I.Scene(sc.centers @ R.T + tr, sc.axes, np.einsum('ij,pjk->pik', R, sc.rot))
    t3, hit3, _ = G.intersect(moved, o @ R.T + tr, d @ R.T)
    np.testing.assert_array_equal(hit3, hit)
    np.testing.assert_allclose(t3[hit], t[hit], atol=1e-9)


def test_intersect_matches_brute_force_march():
    sc = I.scene_mixed(6, 11)
    rays = I.free_rays(sc, 60, 12)
    o = rays[0:3].T.astype(np.float64); d = rays[3:6].T.astype(np.float64)
    t, hit, _ = G.intersect(sc, o, d)
    step = 1e-4
    ts = np.arange(0.0, 6.0, step)
    for j in range(len(o)):
        pts = o[j] + ts[:, None] * d[j]
        inside = (G.implicit(sc, pts) < 0).any(axis=1)
        k = np.argmax(inside)
        if inside[k]:
            assert hit[j] and abs(ts[k] - t[j]) <= 1.5 * step
        else:
            assert not hit[j] or t[j] > 6.0 - step


def test_sdf_bound_and_sign():
    sc = I.scene_mixed(8, 3)
    rng = np.random.default_rng(4)
    p = rng.uniform(-1.5, 1.5, (400, 3))
    s = G.sdf(sc, p)
    inside = (G.implicit(sc, p) < 0).any(axis=1)
    assert np.all((s < 0) == inside)
    # lower bound of the true distance: no surface point is closer than s
    u = I._unit_sphere_dirs(rng, 4000)
    surf = np.concatenate([sc.centers[k] + (sc.rot[k] @ (sc.axes[k] * u).T).T for k in range(sc.n)])
    dist = np.min(np.linalg.norm(p[:, None] - surf[None], axis=2), axis=1)
    out = ~inside
    assert np.all(s[out] <= dist[out] + 1e-12)
    # exact for a lone sphere
    sp = _one([0.1, 0.2, 0.3], [0.4, 0.4, 0.4])
    q = rng.uniform(-1, 1, (50, 3))
    np.testing.assert_allclose(G.sdf(sp, q), np.linalg.norm(q - [0.1, 0.2, 0.3], axis=1) - 0.4, atol=1e-14)


def test_sphere_trace_analytic_sdf():
    sp = _one([0, 0, 0], [1, 1, 1])
    fn = lambda p: G.sdf(sp, p)
    t, hit, steps, done = G.sphere_trace(fn, [(0, 0, -5), (3, 0, -5)], [(0, 0, 1), (0, 0, 1)])
    assert hit[0] and t[0] == pytest.approx(4.0, abs=1e-12) and steps[0] == 2
    assert not hit[1] and done[1]
    # exact SDF of a union of spheres: a declared hit is within hit_eps of the surface, and
    # away from grazing incidence t matches the closed-form first hit
    sc = I.scene_spheres(32, 7)
    rays = I.shadow_rays(sc, 400, 8)
    o = rays[0:3].T.astype(np.float64); d = rays[3:6].T.astype(np.float64)
    t, hit, steps, done = G.sphere_trace(lambda p: G.sdf(sc, p), o, d, max_steps=4000, t_max=6.0)
    assert np.all(done)
    tg, hg, prim = G.intersect(sc, o, d)
    p = o + t[:, None] * d
    assert np.all(np.abs(G.sdf(sc, p[hit])) < 1e-4)
    nrm = np.zeros_like(o)
    nrm[hg] = (o[hg] + tg[hg, None] * d[hg]) - sc.centers[prim[hg]]
    nrm[hg] /= np.linalg.norm(nrm[hg], axis=1, keepdims=True)
    cosi = np.abs(np.sum(nrm * d, axis=1))
    clear = hg & (cosi > 0.2)
    assert clear.sum() > 20 and np.all(hit[clear])
    np.testing.assert_allclose(t[clear], tg[clear], atol=1e-4 / 0.2 + 1e-9)
    # a ray the closed form says misses can only be declared a hit if it grazes within hit_eps
    false_hit = hit & ~hg
    assert np.all(np.abs(G.sdf(sc, p[false_hit])) < 1e-4)


# ---------------------------------------------------------------- quantisation

def test_bf16_matches_torch_cast():
    x = np.random.default_rng(0).standard_normal(200000).astype(np.float32) * np.float32(7.0)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1e-40, 3.4e38, -3.4e38])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.round_bf16(x), ref)


def test_e4m3_codes_cast_and_saturation():
    assert len(O.E4M3_VALUES) == 127 and O.E4M3_VALUES[-1] == 448.0 and O.E4M3_VALUES[1] == 2.0 ** -9
    # every code is a fixed point; torch agrees on every code
    np.testing.assert_array_equal(O.round_e4m3(O.E4M3_VALUES), O.E4M3_VALUES)
    t = torch.arange(0, 127, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(t, O.E4M3_VALUES)
    x = np.random.default_rng(1).uniform(-440, 440, 100000).astype(np.float32)
    x = np.concatenate([x, np.random.default_rng(2).standard_normal(100000).astype(np.float32) * 0.01])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.round_e4m3(x), ref)
    # midpoints round to the even code
    mids = 0.5 * (O.E4M3_VALUES[1:] + O.E4M3_VALUES[:-1])
    r = O.round_e4m3(mids)
    idx = np.searchsorted(O.E4M3_VALUES, r)
    assert np.all(O.E4M3_CODES[idx] % 2 == 0)
    np.testing.assert_array_equal(O.round_e4m3([500.0, -1e9, 448.0]), [448.0, -448.0, 448.0])


def test_pow2_scale():
    assert O.pow2_scale(448.0) == 1.0
    assert O.pow2_scale(448.5) == 2.0
    assert O.pow2_scale(1.0) == 2.0 ** -8
    assert O.pow2_scale(1.75) == 2.0 ** -8 and O.pow2_scale(1.7500001) == 2.0 ** -7
    assert O.pow2_scale(0.0) == 1.0


def _gain_chain_net():
    """A 5-layer net whose per-layer maxima are known in closed form.

    Layer 1 reads the identity feature x0 with gain 240 (neuron 0) or 120 (neuron 1);
    layer l >= 2 reads neuron 0 of layer l - 1 with gain g_l (neuron 0) or g_l / 2
    (neuron 1); every other weight and every bias is 0.  For a calibration batch whose
    largest x0 is 1.25 the maxima are exact binary numbers:
      max h_1 = 300, max h_2 = 3000, max h_3 = 3000 / 4096, max h_4 = 46.875, max h_5 = 187.5
    and the largest |W_l| (l >= 2) are 10, 2^-12, 64, 4."""
    desc = I.NetDesc(6, 1, 5, 4, 2)
    gains = [240.0, 10.0, 2.0 ** -12, 64.0, 4.0]
    parts = []
    for li, g in enumerate(gains):
        W = np.zeros((4, desc.n_feat if li == 0 else 4))
        W[0, 0] = g
        W[1, 0] = g / 2
        parts += [W.ravel(), np.zeros(4)]
    parts += [np.ones(8), np.zeros(2)]
    return desc, np.concatenate(parts).astype(np.float32)


def test_fp8_scales_closed_form():
    """The per-layer FP8 scales of the reduced-precision query (Sec. III-C; per-layer
    power-of-two scales): the input scale of hidden layer l >= 2 comes from max h_(l-1)
    over the calibration batch, the weight scale from max |W_l|, each the smallest power of
    two s with max / s <= 448.  A layer shifted by one (h_2..h_n instead of h_1..h_(n-1)),
    a max over one ray instead of the batch, or a signed instead of an absolute weight
    maximum gives another list."""
    desc, params = _gain_chain_net()
    x0 = np.array([0.5, -1.0, 0.0, 1.25, 0.75, -3.0])     # largest positive x0 in the middle
    rays = np.zeros((6, x0.size), dtype=np.float32)
    rays[0] = x0
    rays[5] = 1.0
    # max h_(l-1) = 300, 3000, 0.732421875, 46.875 -> 1, 8, 2^-9, 2^-3
    assert O.act_scales_fp8(desc, params, rays) == [1.0, 8.0, 2.0 ** -9, 2.0 ** -3]
    # max |W_l| = 10, 2^-12, 64, 4 -> 2^-5, 2^-20, 2^-2, 2^-6
    assert O.weight_scales_fp8(desc, params) == [2.0 ** -5, 2.0 ** -20, 2.0 ** -2, 2.0 ** -6]
    neg = params.copy()
    lay = desc.offsets()
    w_off = lay[2][0]
    neg[w_off] = -neg[w_off]          # W_3[0, 0] = -2^-12: the largest magnitude is unchanged
    assert O.weight_scales_fp8(desc, neg)[1] == 2.0 ** -20
    # each scale puts the layer's largest value inside e4m3's range and no power of two
    # smaller does
    hs, _ = O.mlp_forward(desc, params, O.encode(O.rays_to_inputs(rays), desc.n_freq))
    for h, s in zip(hs[:-1], O.act_scales_fp8(desc, params, rays)):
        assert h.max() / s <= 448.0 < h.max() / (s / 2)


def _brute_emulated(desc, params, ray, precision, act_scales):
    """Element-by-element emulation with torch's own casts (independent of the oracle's rounding)."""
    def bf(x):
        return float(torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).double())

    def f8(x):
        x = max(-448.0, min(448.0, x))
        return float(torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.float8_e4m3fn).double())

    v = [float(x) for x in ray]
    feats = list(v)
    for k in range(desc.n_freq):
        feats += [math.sin(math.pi * (2 ** k) * x) for x in v]
        feats += [math.cos(math.pi * (2 ** k) * x) for x in v]
    L = O.layers(desc, params)
    W1, b1 = L[0]
    hi = [bf(x) for x in feats]
    lo = [bf(x - y) for x, y in zip(feats, hi)]
    h = [max(0.0, b1[o] + sum(bf(W1[o, i]) * (hi[i] + lo[i]) for i in range(len(feats))))
         for o in range(desc.width)]
    for li, (W, b) in enumerate(L[1:-1]):
        if precision == 'bf16':
            h = [max(0.0, b[o] + sum(bf(W[o, i]) * bf(h[i]) for i in range(len(h)))) for o in range(desc.width)]
        else:
            sw = 2.0 ** math.ceil(math.log2(np.max(np.abs(W)) / 448.0)); sa = act_scales[li]
            h = [max(0.0, b[o] + sa * sw * sum(f8(W[o, i] / sw) * f8(h[i] / sa) for i in range(len(h))))
                 for o in range(desc.width)]
    Wh, bh = L[-1]
    return [bh[o] + sum(Wh[o, i] * h[i] for i in range(len(h))) for o in range(desc.n_out)]


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_emulated_forward_matches_brute_force(precision):
    desc = I.NetDesc(6, 2, 3, 16, 2)
    params = I.test_params(desc, 5, bias_std=0.2)
    rays = I.free_rays(I.scene_spheres(4, 1), 4, 3)
    scales = O.act_scales_fp8(desc, params, I.free_rays(I.scene_spheres(4, 1), 64, 21))
    _, z = O.mlp_forward_emulated(desc, params, O.encode(O.rays_to_inputs(rays), desc.n_freq), precision, scales)
    for j in range(rays.shape[1]):
        ref = _brute_emulated(desc, params, rays[:, j], precision, scales)
        np.testing.assert_allclose(z[j], ref, atol=1e-9)
    # the emulation is a real perturbation, but a small one
    _, z64 = O.mlp_forward(desc, params, O.encode(O.rays_to_inputs(rays), desc.n_freq))
    d = np.abs(z - z64).max()
    assert 0 < d < (0.05 if precision == 'bf16' else 0.5)


# ---------------------------------------------------------------- loss, gradient, Adam

def test_loss_special_cases():
    z = np.array([0.0, 0.0, 0.0, 0.0])
    t = O.softplus(z)
    (tot, l1, bce), dzt, dzx = O.loss_terms(z, z, t, np.array([1, 1, 0, 0]))
    assert l1 == 0.0 and bce == pytest.approx(math.log(2.0), abs=1e-15)
    assert tot == pytest.approx(0.3 * math.log(2.0), abs=1e-15)
    np.testing.assert_allclose(dzx, 0.3 * np.array([-0.5, -0.5, 0.5, 0.5]) / 4, atol=1e-17)
    np.testing.assert_array_equal(dzt, 0.0)     # sign(0) = 0
    # a far miss of the distance is clamped and passes no gradient; misses carry no L1
    (tot, l1, bce), dzt, dzx = O.loss_terms(np.array([10.0, 10.0]), np.array([0.0, 0.0]),
                                            np.array([1.0, 50.0]), np.array([1, 0]))
    assert l1 == pytest.approx(3.0) and dzt[0] == 0.0 and dzt[1] == 0.0
    # no hits at all: the L1 term is 0
    (tot, l1, bce), dzt, dzx = O.loss_terms(np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3))
    assert l1 == 0.0 and np.all(dzt == 0)


def test_gradient_matches_central_differences():
    desc = I.NET_TINY
    params = I.test_params(desc, 1).astype(np.float64)
    sc = I.scene_ellipsoids(64, 3)
    rays = I.train_rays(sc, 24, 1000)
    t_gt, hit, _ = G.intersect_soa(sc, rays)
    (loss, _, _), grad = O.ddf_loss_and_grad(desc, params, rays, t_gt, hit)
    rng = np.random.default_rng(0)
    offs = desc.offsets()
    idx = []
    for w_off, b_off, o, i in offs:                # weights and biases of every layer
        idx += list(rng.integers(w_off, b_off, 12)) + list(rng.integers(b_off, b_off + o, 4))
    h = 1e-6
    for k in idx:
        pp = params.copy(); pp[k] += h
        pm = params.copy(); pm[k] -= h
        (lp, _, _), _ = O.ddf_loss_and_grad(desc, pp, rays, t_gt, hit)
        (lm, _, _), _ = O.ddf_loss_and_grad(desc, pm, rays, t_gt, hit)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, grad[k])


def test_adam_matches_torch():
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(50); grads = [rng.standard_normal(50) for _ in range(5)]
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for s, g in enumerate(grads, start=1):
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = O.adam_step(p, m, v, g, s, 3e-3)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-15)


def test_paper_constants_fixture():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        gold = json.load(f)
    assert O.BCE_WEIGHT == gold["hit_ce_weight"]["value"]
    assert O.lr_schedule(0) == pytest.approx(gold["lr_initial"]["value"])
    assert O.lr_schedule(gold["train_steps"]["value"]) == pytest.approx(
        gold["lr_initial"]["value"] * gold["lr_final_fraction"]["value"])
    assert O.lr_schedule(15000) == pytest.approx(0.5 * (3e-3 + 1.5e-4))
    # the full-size net is close to the paper's field-size budget
    mb = I.NET_FULL.param_count() * 4 / 1e6
    assert abs(mb - gold["field_size_mb"]["value"]) < 6.0


def test_emulated_bf16_backward_matches_brute_force():
    """The bf16-rounding backward against element-by-element loops using torch's casts."""
    def bf(x):
        return float(torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).double())

    desc = I.NetDesc(6, 1, 3, 6, 2)
    params = I.test_params(desc, 8, bias_std=0.2)
    rays = I.free_rays(I.scene_spheres(4, 1), 3, 5)
    g = O.encode(O.rays_to_inputs(rays), desc.n_freq)
    dz = np.random.default_rng(3).standard_normal((3, 2))
    got = O.mlp_backward_emulated_bf16(desc, params, g, dz)
    L = O.layers(desc, params)
    n_l = len(L)
    acc = [(np.zeros_like(W), np.zeros_like(b)) for W, b in L]
    for r in range(3):
        # forward with the kernel's roundings
        feats = list(g[r])
        hi = [bf(x) for x in feats]
        lo = [bf(x - y) for x, y in zip(feats, hi)]
        W1, b1 = L[0]
        a = [b1[o] + sum(bf(W1[o, i]) * (hi[i] + lo[i]) for i in range(len(feats))) for o in range(desc.width)]
        hs = [[max(0.0, x) for x in a]]
        for W, b in L[1:-1]:
            a = [b[o] + sum(bf(W[o, i]) * bf(hs[-1][i]) for i in range(desc.width)) for o in range(desc.width)]
            hs.append([max(0.0, x) for x in a])
        ins = [[bf(x) for x in feats]] + [[bf(x) for x in h] for h in hs]
        Wh, _ = L[-1]
        for o in range(2):
            for j in range(desc.width):
                acc[-1][0][o, j] += dz[r, o] * ins[-1][j]
            acc[-1][1][o] += dz[r, o]
        d = [bf(sum(dz[r, o] * Wh[o, j] for o in range(2)) * (hs[-1][j] > 0)) for j in range(desc.width)]
        for l in range(n_l - 2, -1, -1):
            W, _ = L[l]
            for o in range(W.shape[0]):
                for i in range(W.shape[1]):
                    acc[l][0][o, i] += d[o] * ins[l][i]
                acc[l][1][o] += d[o]
            if l > 0:
                d = [bf(sum(d[o] * bf(W[o, i]) for o in range(W.shape[0])) * (hs[l - 1][i] > 0))
                     for i in range(W.shape[1])]
    ref = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in acc])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_sdf_loss_gradient_matches_central_differences():
    desc = I.NetDesc(3, 4, 3, 32, 1)
    params = I.test_params(desc, 2).astype(np.float64)
    sc = I.scene_mixed(8, 3)
    pts = I.sdf_train_points(sc, 40, 4).T.astype(np.float64)
    gt = G.sdf(sc, pts)
    loss, grad = O.sdf_loss_and_grad(desc, params, pts, gt)
    assert loss == pytest.approx(np.mean(np.abs(O.sdf_eval(desc, params, pts) - gt)), rel=1e-14)
    rng = np.random.default_rng(1)
    h = 1e-6
    for k in rng.choice(len(params), 60, replace=False):
        pp = params.copy(); pp[k] += h
        pm = params.copy(); pm[k] -= h
        fd = (O.sdf_loss_and_grad(desc, pp, pts, gt)[0] - O.sdf_loss_and_grad(desc, pm, pts, gt)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_shift_rays_targets_match_exact_casting():
    """Self-consistency points: the exact cast from a moved origin along its direction hits at
    the shifted target (to the float32 rounding of t); unselected slots are untouched; about
    frac of the slots move; frac = 0 and an all-miss batch change nothing."""
    sc = I.scene_ellipsoids(64, 3)
    n = 2000
    rays = I.train_rays(sc, n, 77)
    tg, hit, _ = G.intersect_soa(sc, rays)
    t32 = np.where(hit, tg, 0).astype(np.float32)
    u = np.random.default_rng(1).random((3, n)).astype(np.float32)
    ro, to, ho, src, sh = O.shift_rays(rays, t32, hit, u, 0.3)
    assert abs(sh.mean() - 0.3) < 0.04 and ho[sh].all()
    t2, h2, _ = G.intersect(sc, ro[0:3, sh].T, ro[3:6, sh].T)
    assert h2.all()
    assert np.abs(t2 - to[sh]).max() <= 4e-7 * max(1.0, t32.max())
    assert np.all(to[sh] > 0) and np.all(to[sh] <= t32[src[sh]])
    np.testing.assert_array_equal(ro[:, ~sh], rays[:, ~sh].astype(np.float64))
    np.testing.assert_array_equal(ro[3:6, sh], rays[3:6, src[sh]].astype(np.float64))
    assert hit[src[sh]].all()
    ro0, to0, _, _, sh0 = O.shift_rays(rays, t32, hit, u, 0.0)
    assert not sh0.any() and np.array_equal(ro0, rays.astype(np.float64))
    _, _, _, _, shm = O.shift_rays(rays, t32, np.zeros(n, np.uint8), u, 1.0)
    assert not shm.any()


def test_lifted_shadow_origins_sit_at_the_offset():
    """The trace leg lifts shadow-ray origins past each hit threshold: on a sphere-only scene
    (where the oracle's distance is exact) an origin lifted by `offset` along the outward
    normal lies `offset` from the union surface, unless another sphere is nearer; the
    fitting samples keep half their points uniform in the box and half near the surface."""
    sc = I.scene_spheres(16, 5)
    for off in (1e-3, 2e-3, 2e-2):
        r = I.shadow_rays(sc, 2000, 9, offset=off).astype(np.float64)
        s = G.sdf(sc, r[0:3].T)
        close = np.abs(s - off) < 1e-5
        assert close.mean() > 0.95, (off, close.mean())
        assert np.all(s[~close] < off)          # only a nearer sphere can make it differ
        d = r[3:6].T
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    p = I.sdf_fit_points(sc, 4000, 3).astype(np.float64)
    s = np.abs(G.sdf(sc, p.T))
    assert p.shape == (3, 4000)
    assert np.all(np.abs(p) <= I.BOX_HALF + 0.2)
    # [uniform | N(0, 0.05^2) band | uniform | N(0, 0.005^2) band], 1000 points each
    wide, tight = s[1000:2000], s[3000:4000]
    assert np.median(tight) < 0.01 < np.median(wide) < 0.1 < np.median(s[:1000])

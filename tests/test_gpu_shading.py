"""The shading consumers (Sec. III-C, IV-F) on the GPU through the C ABI, against the float64
oracle: the primary G-buffer, the secondary rays, the per-pixel shadow/AO reduction, the
reference maps by exact casting, and an end-to-end render with a trained hash-grid field."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as G
from oracle import shading as S
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda

pytestmark = pytest.mark.gpu

OFF = I.NORMAL_OFFSET


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _view(w, h):
    return I.View(width=w, height=h)


def _gbuf_np(p, n):
    return np.ascontiguousarray(np.concatenate([p, n], axis=1).T.astype(np.float32))


@pytest.mark.parametrize("w,h", [(97, 61), (1, 1), (64, 64)])
def test_gbuffer_matches_oracle(w, h):
    """Hit flags agree wherever the cast is not numerically ambiguous (a ray passing a
    primitive nearly tangent may hit or miss it in float32); points (to 1e-4) and normals (to
    2e-3) wherever the ray is not grazing, except normals at the curves where two surfaces
    meet (either primitive is a valid answer there)."""
    dev = cuda()
    sc = I.scene_ground(24, 5)
    v = _view(w, h)
    gb, hit = ddf.primary_gbuffer(v, _t(ddf.scene_prims(sc), dev))
    torch.cuda.synchronize()
    gb, hit = gb.cpu().numpy().astype(np.float64), hit.cpu().numpy().astype(bool)
    p, n, h64, margin = S.gbuffer(sc, v.eye, v.target, v.up, v.fov_y, v.width, v.height)
    clear = margin > 1e-4
    assert np.array_equal(hit[clear], h64[clear])
    # a root's float32 error grows like 1 / sqrt(disc): points are compared away from grazing
    both = hit & h64 & (margin > 1e-3)
    dp = np.abs(gb[0:3].T[both] - p[both]).max(axis=1) if both.any() else np.zeros(0)
    assert (dp <= 1e-4).all()
    dn = np.abs(gb[3:6].T[both] - n[both]).max(axis=1) if both.any() else np.zeros(0)
    bad = np.flatnonzero(both)[dn > 2e-3]
    if bad.size:
        F = np.abs(G.implicit(sc, p[bad]))
        assert ((F < 1e-3).sum(axis=1) >= 2).all(), "normal mismatch away from an intersection curve"
    assert (gb[:, ~hit] == 0).all()
    print(f"gbuffer {w}x{h}: hits {hit.sum()}, max |dp| {dp.max() if dp.size else 0:.2e}, "
          f"ambiguous {int((~clear).sum())}, normal ties {bad.size}")


@pytest.mark.parametrize("n_ao", [0, 1, 16])
def test_secondary_rays_match_oracle(n_ao):
    dev = cuda()
    sc = I.scene_ground(24, 5)
    P = 1500
    p, n = I.surface_points(sc, P, 41)
    hit = np.ones(P, dtype=np.uint8)
    hit[::7] = 0
    u = I.uniforms(2, P * n_ao, 42) if n_ao else np.zeros((2, 1), np.float32)
    gb = _gbuf_np(p, n)
    rays = ddf.secondary_rays(_t(gb, dev), _t(hit, dev), I.SHADE_LIGHT, n_ao, _t(u, dev), OFF)
    torch.cuda.synchronize()
    r = rays.cpu().numpy().astype(np.float64).T.reshape(P, 1 + n_ao, 6)
    ref = S.secondary_rays(gb[0:3].T.astype(np.float64), gb[3:6].T.astype(np.float64), I.SHADE_LIGHT, n_ao,
                           u[:, :P * n_ao].astype(np.float64), OFF).reshape(P, 1 + n_ao, 6)
    h = hit.astype(bool)
    assert np.abs(r[h, :, 0:3] - ref[h, :, 0:3]).max() <= 1e-6
    assert np.abs(r[h, :, 3:6] - ref[h, :, 3:6]).max() <= 2e-6
    # background pixels: finite unit dummy rays
    assert np.isfinite(r[~h]).all() and np.allclose(np.linalg.norm(r[~h, :, 3:6], axis=2), 1.0)


@pytest.mark.parametrize("answers", ["field", "exact"])
@pytest.mark.parametrize("ao_radius", [math.inf, 0.7])
def test_shade_matches_oracle(answers, ao_radius):
    """The reduction against the oracle's on the same answers, bit for bit (shadow 0/1, AO
    count / K rounded once); a shadow decision within 1e-5 of the light distance is left out
    (float32 vs float64 distance)."""
    dev = cuda()
    sc = I.scene_ground(24, 5)
    P, K = 3001, 8
    p, n = I.surface_points(sc, P, 43)
    hit = np.ones(P, dtype=np.uint8)
    hit[::5] = 0
    rng = np.random.default_rng(44)
    t = rng.uniform(0, 6, P * (1 + K)).astype(np.float32)
    xi = rng.uniform(0, 1, P * (1 + K)).astype(np.float32)
    xi[::11] = 0.5                                   # exactly at the threshold: not a hit
    rh = (rng.uniform(size=P * (1 + K)) < 0.4).astype(np.uint8)
    gb = _gbuf_np(p, n)
    kw = {"xi": _t(xi, dev)} if answers == "field" else {"ray_hit": _t(rh, dev)}
    sh, ao = ddf.shade(_t(t, dev), _t(gb, dev), _t(hit, dev), I.SHADE_LIGHT, K, OFF, ao_radius=ao_radius, **kw)
    torch.cuda.synchronize()
    flag = xi > 0.5 if answers == "field" else rh.astype(bool)
    p64, n64 = gb[0:3].T.astype(np.float64), gb[3:6].T.astype(np.float64)
    s64, a64 = S.shade(t, flag, p64, n64, hit.astype(bool), I.SHADE_LIGHT, K, OFF, ao_radius)
    o = p64 + OFF * n64
    dist = np.linalg.norm(np.asarray(I.SHADE_LIGHT)[None] - o, axis=1)
    clear = np.abs(t.reshape(P, 1 + K)[:, 0] - dist) > 1e-5
    assert np.array_equal(sh.cpu().numpy()[clear], s64[clear].astype(np.float32))
    assert np.array_equal(ao.cpu().numpy(), a64.astype(np.float32))


def test_shade_argument_errors():
    dev = cuda()
    P = 16
    gb = torch.zeros((6, P), device=dev)
    hit = torch.zeros(P, dtype=torch.uint8, device=dev)
    t = torch.zeros(P, device=dev)
    with pytest.raises(ddf.DDFError, match="exactly one"):
        ddf.shade(t, gb, hit, I.SHADE_LIGHT, 0, OFF)
    with pytest.raises(ddf.DDFError, match="degenerate camera"):
        ddf.primary_gbuffer(I.View(eye=(0.0, 1.0, 0.0), target=(0.0, 0.0, 0.0), width=4, height=4),
                            torch.zeros((1, 16), device=dev))


@pytest.mark.parametrize("answers", ["field", "exact"])
def test_bounce_matches_oracle(answers):
    """The one-bounce term against the oracle's on the same answers and rays: float32 hit
    points and trilinear weights, a sum of K terms in [0, 1] (observed ~1e-7)."""
    dev = cuda()
    P, K = 3001, 8
    rng = np.random.default_rng(50)
    hit = np.ones(P, dtype=np.uint8)
    hit[::7] = 0
    o = rng.uniform(-1.4, 1.4, (P * (1 + K), 3))
    d = rng.standard_normal((P * (1 + K), 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.ascontiguousarray(np.concatenate([o, d], axis=1).T.astype(np.float32))
    t = rng.uniform(0, 4, P * (1 + K)).astype(np.float32)
    xi = rng.uniform(0, 1, P * (1 + K)).astype(np.float32)
    xi[::13] = 0.5                                   # exactly at the threshold: a miss
    rh = (rng.uniform(size=P * (1 + K)) < 0.4).astype(np.uint8)
    R = I.radiance_grid(I.RADIANCE_RES, 49)
    kw = {"xi": _t(xi, dev)} if answers == "field" else {"ray_hit": _t(rh, dev)}
    gi = ddf.bounce(_t(t, dev), _t(rays, dev), _t(hit, dev), K, _t(R, dev), I.BOX_HALF, I.SKY, **kw)
    torch.cuda.synchronize()
    flag = xi > 0.5 if answers == "field" else rh.astype(bool)
    g64 = S.bounce(t, flag, rays.T.astype(np.float64), hit.astype(bool), K, R, I.BOX_HALF, *I.SKY)
    err = np.abs(gi.cpu().numpy().astype(np.float64) - g64)
    print(f"bounce ({answers}): max |d gi| {err.max():.2e}")
    assert err.max() <= 2e-6
    assert (gi.cpu().numpy()[hit == 0] == 0).all()


def test_bounce_argument_errors():
    dev = cuda()
    P, K = 4, 2
    t = torch.zeros(P * (1 + K), device=dev)
    rays = torch.zeros((6, P * (1 + K)), device=dev)
    hit = torch.ones(P, dtype=torch.uint8, device=dev)
    with pytest.raises(ddf.DDFError, match="exactly one"):
        ddf.bounce(t, rays, hit, K, torch.zeros((2, 2, 2), device=dev), I.BOX_HALF, I.SKY)
    with pytest.raises(ddf.DDFError, match="res"):
        ddf.bounce(t, rays, hit, K, torch.zeros((1, 1, 1), device=dev), I.BOX_HALF, I.SKY, xi=t)
    with pytest.raises(ddf.DDFError, match="box_half"):
        ddf.bounce(t, rays, hit, K, torch.zeros((2, 2, 2), device=dev), 0.0, I.SKY, xi=t)


def test_reference_maps_match_oracle():
    """The reference pipeline on the GPU (G-buffer, secondary rays, exact cast, reduction)
    against the oracle's: the maps differ only where float32 points move a ray across an
    occluder's silhouette (a few pixels)."""
    dev = cuda()
    sc = I.scene_ground(24, 5)
    v = _view(80, 64)
    K = 8
    prims = _t(ddf.scene_prims(sc), dev)
    gb, hit = ddf.primary_gbuffer(v, prims)
    P = v.width * v.height
    u = I.uniforms(2, P * K, 45)
    rays = ddf.secondary_rays(gb, hit, I.SHADE_LIGHT, K, _t(u, dev), OFF)
    tg, rh = ddf.cast_targets(prims, rays)
    sh, ao = ddf.shade(tg, gb, hit, I.SHADE_LIGHT, K, OFF, ray_hit=rh)
    torch.cuda.synchronize()
    p, n, h64, _ = S.gbuffer(sc, v.eye, v.target, v.up, v.fov_y, v.width, v.height)
    s64, a64 = S.reference(sc, p, n, h64, I.SHADE_LIGHT, K, u.astype(np.float64), OFF)
    m = hit.cpu().numpy().astype(bool) & h64
    ds = np.abs(sh.cpu().numpy() - s64)[m]
    da = np.abs(ao.cpu().numpy() - a64)[m]
    R = I.radiance_grid(I.RADIANCE_RES, 49)
    gi = ddf.bounce(tg, rays, hit, K, _t(R, dev), I.BOX_HALF, I.SKY, ray_hit=rh)
    torch.cuda.synchronize()
    rays64 = S.secondary_rays(p, n, I.SHADE_LIGHT, K, u.astype(np.float64), OFF)
    g64 = S.reference_bounce(sc, rays64, h64, K, R, I.BOX_HALF, *I.SKY)
    dg = np.abs(gi.cpu().numpy() - g64)[m]
    print(f"reference maps: shadow mismatches {int((ds > 0).sum())} / {m.sum()}, AO MAE {da.mean():.2e}, "
          f"bounce MAE {dg.mean():.2e}")
    assert (ds > 0).mean() < 0.01 and da.mean() < 0.01 and dg.mean() < 0.01


def test_trained_hash_field_shading():
    """End to end: the paper's hash-grid field distilled by its recipe (fresh GPU-sampled
    batches of 16,384 rays, 30 % self-consistency points, cosine schedule; 3,000 steps here)
    on one compound object above a ground slab, then the render's secondary rays answered by
    the field.  The field's maps equal the oracle's reduction of the field's own answers and
    track the reference maps (floors from a 3,000-step run with margin; the table gradient's
    float atomics make runs differ slightly)."""
    dev = cuda()
    sc = I.scene_object(8, 5)
    desc = I.HASH_PAPER
    prims = _t(ddf.scene_prims(sc), dev)
    import oracle.hashgrid_oracle as H
    from oracle import ddf_oracle as O
    p = _t(I.hash_params(desc, H.table_entries(desc), 46), dev)
    m = torch.zeros_like(p); vv = torch.zeros_like(p)
    B, T = 16384, 4
    ws = torch.empty(ddf.hash_train_workspace_bytes(desc, B), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(48)
    U = torch.empty((3 * T + 2, B), device=dev)
    cdf = ddf.prim_area_cdf(prims)
    steps = 3000
    for s in range(1, steps + 1):
        U.uniform_(generator=gen)
        rays = ddf.sample_rays(prims, U, mode=2, offset=OFF, cdf=cdf)
        t, h = ddf.cast_targets(prims, rays)
        t = torch.where(h > 0, t, torch.zeros_like(t))
        rs, ts, hs = ddf.shift_rays(rays, t, h, torch.rand((3, B), device=dev, generator=gen), 0.3)
        hp = ddf.TrainHParamsC(ddf.lr_cosine(s - 1, total=steps), 0.9, 0.999, 1e-8, O.BCE_WEIGHT, O.L1_CLAMP, s)
        ddf.hash_train_step(desc, p, m, vv, rs, ts, hs, hp, ws)
    v = _view(128, 128)
    K = 8
    gb, hit = ddf.primary_gbuffer(v, prims)
    P = v.width * v.height
    u = I.uniforms(2, P * K, 47)
    rays = ddf.secondary_rays(gb, hit, I.SHADE_LIGHT, K, _t(u, dev), OFF)
    tf, xf = ddf.hash_query(desc, p, rays)
    sh, ao = ddf.shade(tf, gb, hit, I.SHADE_LIGHT, K, OFF, xi=xf)
    tg, rh = ddf.cast_targets(prims, rays)
    shr, aor = ddf.shade(tg, gb, hit, I.SHADE_LIGHT, K, OFF, ray_hit=rh)
    torch.cuda.synchronize()
    hm = hit.cpu().numpy().astype(bool)
    g64 = gb.cpu().numpy().astype(np.float64)
    s64, a64 = S.shade(tf.cpu().numpy(), xf.cpu().numpy() > 0.5, g64[0:3].T, g64[3:6].T, hm, I.SHADE_LIGHT, K, OFF)
    o = g64[0:3].T + OFF * g64[3:6].T
    dist = np.linalg.norm(np.asarray(I.SHADE_LIGHT)[None] - o, axis=1)
    clear = np.abs(tf.cpu().numpy().reshape(P, 1 + K)[:, 0] - dist) > 1e-5
    assert np.array_equal(sh.cpu().numpy()[clear], s64[clear].astype(np.float32))
    assert np.array_equal(ao.cpu().numpy(), a64.astype(np.float32))
    ps = S.psnr(sh.cpu().numpy(), shr.cpu().numpy(), hm)
    pa = S.psnr(ao.cpu().numpy(), aor.cpu().numpy(), hm)
    ma = S.mae(ao.cpu().numpy(), aor.cpu().numpy(), hm)
    R = _t(I.radiance_grid(I.RADIANCE_RES, 49), dev)
    gf = ddf.bounce(tf, rays, hit, K, R, I.BOX_HALF, I.SKY, xi=xf)
    gr = ddf.bounce(tg, rays, hit, K, R, I.BOX_HALF, I.SKY, ray_hit=rh)
    torch.cuda.synchronize()
    g64 = S.bounce(tf.cpu().numpy(), xf.cpu().numpy() > 0.5, rays.cpu().numpy().T.astype(np.float64), hm, K,
                   R.cpu().numpy(), I.BOX_HALF, *I.SKY)
    assert np.abs(gf.cpu().numpy() - g64).max() <= 2e-6
    pg = S.psnr(gf.cpu().numpy(), gr.cpu().numpy(), hm)
    print(f"trained hash field ({steps} steps): shadow PSNR {ps:.2f} dB, AO PSNR {pa:.2f} dB, AO MAE {ma:.4f}, "
          f"bounce PSNR {pg:.2f} dB; shadowed {shr.cpu().numpy()[hm].mean():.3f}, mean AO "
          f"{aor.cpu().numpy()[hm].mean():.3f}")
    assert ps > 9.0 and pa > 18.0 and ma < 0.06 and pg > 18.0

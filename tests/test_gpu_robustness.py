"""Per-ray isolation of non-finite inputs (the C ABI's promise that a NaN in a ray only
affects that ray's outputs): rays are independent queries (Sec. III-C), so a workgroup
that shares its tile, its matrix products and its head reductions with a poisoned ray
must give every other ray exactly the answer it gives without it."""
import numpy as np
import pytest
import torch

from oracle import hashgrid_oracle as H
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda

pytestmark = pytest.mark.gpu


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _poison(rays):
    """(rays with NaN / inf planted in a few rays of different tiles, their indices)."""
    bad = np.array([0, 5, 63, 64, 130, rays.shape[1] - 1])
    r = rays.copy()
    r[0, bad[0]] = np.nan           # origin component
    r[4, bad[1]] = np.nan           # direction component
    r[:, bad[2]] = np.nan           # the whole ray
    r[2, bad[3]] = np.inf
    r[3, bad[4]] = -np.inf
    r[1, bad[5]] = np.nan           # the ragged tail's last ray
    return r, bad


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_dense_query_nan_stays_in_its_ray(prec):
    dev = cuda()
    desc = I.NetDesc(6, 10, 4, 512, 2)
    params = I.test_params(desc, 21)
    sc = I.scene_mixed(256, 2)
    rays = I.shadow_rays(sc, 128 * 3 + 45, 22)
    scales = None
    if prec == "fp8":
        packed32 = ddf.pack(desc, "fp32", _t(params, dev))
        scales = ddf.fp8_act_scales(desc, packed32, _t(I.free_rays(sc, 1024, 21), dev))
    packed = ddf.pack(desc, prec, _t(params, dev), act_scales=scales)
    poisoned, bad = _poison(rays)
    t0, x0 = ddf.query(desc, prec, packed, _t(rays, dev))
    t1, x1 = ddf.query(desc, prec, packed, _t(poisoned, dev))
    torch.cuda.synchronize()
    t0, x0, t1, x1 = (v.cpu().numpy() for v in (t0, x0, t1, x1))
    good = np.ones(rays.shape[1], dtype=bool)
    good[bad] = False
    assert np.isfinite(t0).all() and np.isfinite(x0).all()
    np.testing.assert_array_equal(t1[good], t0[good])
    np.testing.assert_array_equal(x1[good], x0[good])


def test_split_query_nan_stays_in_its_ray():
    dev = cuda()
    desc = I.NetDesc(6, 10, 4, 512, 2)
    params = I.test_params(desc, 23)
    rays = I.shadow_rays(I.scene_mixed(256, 2), 64 * 5 + 9, 24)
    packed = ddf.pack(desc, "bf16", _t(params, dev))
    poisoned, bad = _poison(rays)
    t0, x0 = ddf.query_split(desc, packed, _t(rays, dev))
    t1, x1 = ddf.query_split(desc, packed, _t(poisoned, dev))
    torch.cuda.synchronize()
    good = np.ones(rays.shape[1], dtype=bool)
    good[bad] = False
    np.testing.assert_array_equal(t1.cpu().numpy()[good], t0.cpu().numpy()[good])
    np.testing.assert_array_equal(x1.cpu().numpy()[good], x0.cpu().numpy()[good])


@pytest.mark.parametrize("fused", [False, True], ids=["two-pass", "fused"])
def test_hash_query_nan_stays_in_its_ray(fused):
    dev = cuda()
    desc = I.HASH_SMALL
    params = I.hash_params(desc, H.table_entries(desc), 25, table_std=0.3)
    rays = I.free_rays(I.scene_mixed(256, 2), 200, 26)
    poisoned, bad = _poison(rays)
    pd = _t(params, dev)
    t0, x0 = ddf.hash_query(desc, pd, _t(rays, dev), fused=fused)
    t1, x1 = ddf.hash_query(desc, pd, _t(poisoned, dev), fused=fused)
    torch.cuda.synchronize()
    good = np.ones(rays.shape[1], dtype=bool)
    good[bad] = False
    np.testing.assert_array_equal(t1.cpu().numpy()[good], t0.cpu().numpy()[good])
    np.testing.assert_array_equal(x1.cpu().numpy()[good], x0.cpu().numpy()[good])


def test_sphere_trace_nan_stays_in_its_ray():
    """Whatever a poisoned ray does (the ReLU maps a NaN pre-activation to 0, so its SDF may
    come out finite), every other ray's t, hit flag and step count are unchanged."""
    dev = cuda()
    desc = I.NetDesc(3, 10, 6, 256, 1)
    params = I.planted_box_sdf(desc, [0.3, 0.5, 0.7], 7)
    rng = np.random.default_rng(3)
    o = rng.uniform(-1.5, 1.5, (600, 3))
    o = o[np.max(np.abs(o) - [0.3, 0.5, 0.7], axis=1) > 0.05][:200]
    rays = I._soa(o, rng.uniform(-0.2, 0.2, (len(o), 3)) - o)
    poisoned, bad = _poison(rays)
    packed = ddf.pack(desc, "fp32", _t(params, dev))
    t0, h0, s0 = ddf.sphere_trace(desc, "fp32", packed, _t(rays, dev))
    t1, h1, s1 = ddf.sphere_trace(desc, "fp32", packed, _t(poisoned, dev))
    torch.cuda.synchronize()
    good = np.ones(rays.shape[1], dtype=bool)
    good[bad] = False
    for a, b in ((t0, t1), (h0, h1), (s0, s1)):
        np.testing.assert_array_equal(b.cpu().numpy()[good], a.cpu().numpy()[good])

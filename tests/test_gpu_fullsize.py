"""Full-size launches, checked on sampled outputs the oracle computes one by one.

The workloads: 2^20 shadow rays through the 12 x 1024 DDF (the benchmark's launch), the
ambient-occlusion batch of 512 x 512 surface points x 32 cosine rays (8,388,608 rays),
and 2^24 mixed shadow/AO/one-bounce rays through the 16 x 1024 DDF.  Every output is
checked against properties that hold at any size (finite, t >= 0, 0 <= xi <= 1); a
sample of 2,048 evenly spaced rays plus both sides of 64 seeded 128-ray tile boundaries
(the workgroup tiles are 32, 64 or 128 rays) and the last ray is compared with the float64
oracle (fp32: per-ray rounding-model tolerance; bf16: the emulated oracle; fp8: the
format's own error)."""
import numpy as np
import pytest
import torch

from oracle import ddf_oracle as O
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda, fp32_forward_sigma, U32

pytestmark = pytest.mark.gpu

SAMPLE = 2048


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _props(t, xi):
    assert torch.isfinite(t).all() and torch.isfinite(xi).all()
    assert (t >= 0).all() and (xi >= 0).all() and (xi <= 1).all()


def _sample(n):
    idx = np.linspace(0, n - 1, SAMPLE).astype(np.int64)
    tiles = np.random.default_rng(7).integers(1, n // 128, 64)
    edges = np.concatenate([tiles * 128 - 1, tiles * 128])   # the last ray of a tile, the first of the next
    return np.unique(np.concatenate([idx, edges, [n - 1]]))  # the ragged end of the last tile always


def _check_fp32_sample(desc, params, rays_s, t_s, xi_s):
    z, sig = fp32_forward_sigma(desc, params, rays_s)
    t64 = O.softplus(z[:, 0]); x64 = O.sigmoid(z[:, 1])
    assert np.all(np.abs(t_s - t64) <= 8 * sig[:, 0] + 8 * U32 * np.maximum(1, t64))
    assert np.all(np.abs(xi_s - x64) <= 2 * sig[:, 1] + 8 * U32)


def _query(desc, prec, params, rays, dev, scales=None):
    packed = ddf.pack(desc, prec, _t(params, dev), act_scales=scales)
    t, xi = ddf.query(desc, prec, packed, rays)
    torch.cuda.synchronize()
    _props(t, xi)
    return t, xi


def test_shadow_2p20_all_precisions():
    dev = cuda()
    desc = I.NET_FULL
    scene = I.scene_mixed(256, 2)
    rays_np = I.shadow_rays(scene, 1 << 20, 12)
    params = I.he_init(desc, 0)
    rays = _t(rays_np, dev)
    idx = _sample(rays_np.shape[1])
    rs = rays_np[:, idx]
    t, xi = _query(desc, "fp32", params, rays, dev)
    _check_fp32_sample(desc, params, rs, t.cpu().numpy()[idx].astype(np.float64),
                       xi.cpu().numpy()[idx].astype(np.float64))
    t, xi = _query(desc, "bf16", params, rays, dev)
    te, xe, _, _ = O.ddf_query_emulated(desc, params, rs, "bf16")
    d = np.abs(t.cpu().numpy()[idx] - te)
    assert d.mean() <= 1e-3 and d.max() <= 2e-2
    calib = I.free_rays(scene, 4096, 21)
    scales = O.act_scales_fp8(desc, params, calib)
    t, xi = _query(desc, "fp8", params, rays, dev, np.array(scales, dtype=np.float32))
    te, _, _, _ = O.ddf_query_emulated(desc, params, rs, "fp8", act_scales=scales)
    t64, _, _, _ = O.ddf_query(desc, params, rs)
    d = np.abs(t.cpu().numpy()[idx] - te)
    assert d.mean() <= 0.75 * np.abs(te - t64).mean()


def test_ao_8m_rays_bf16_fp8():
    dev = cuda()
    desc = I.NET_FULL
    scene = I.scene_mixed(256, 2)
    rays_np = I.ao_rays(scene, 512 * 512, 32, 13)
    assert rays_np.shape[1] == 8388608
    params = I.he_init(desc, 0)
    rays = _t(rays_np, dev)
    idx = _sample(rays_np.shape[1])
    rs = rays_np[:, idx]
    t64, x64, _, _ = O.ddf_query(desc, params, rs)
    t, xi = _query(desc, "bf16", params, rays, dev)
    te, _, _, _ = O.ddf_query_emulated(desc, params, rs, "bf16")
    d = np.abs(t.cpu().numpy()[idx] - te)
    assert d.mean() <= 1e-3 and np.abs(t.cpu().numpy()[idx] - t64).mean() <= 1e-2
    scales = O.act_scales_fp8(desc, params, I.free_rays(scene, 4096, 21))
    t, xi = _query(desc, "fp8", params, rays, dev, np.array(scales, dtype=np.float32))
    te, _, _, _ = O.ddf_query_emulated(desc, params, rs, "fp8", act_scales=scales)
    d = np.abs(t.cpu().numpy()[idx] - te)
    assert d.mean() <= 0.75 * np.abs(te - t64).mean()
    assert np.abs(t.cpu().numpy()[idx] - t64).mean() <= 5e-2


def test_mixed_16m_rays_16x1024():
    dev = cuda()
    desc = I.NET_LARGE
    scene = I.scene_mixed(256, 2)
    rays_np = I.mixed_rays(scene, 1 << 24, 15)
    params = I.he_init(desc, 0)
    rays = _t(rays_np, dev)
    idx = _sample(rays.shape[1])
    rs = rays_np[:, idx]
    t64, _, _, _ = O.ddf_query(desc, params, rs)
    scales = O.act_scales_fp8(desc, params, I.free_rays(scene, 4096, 21))
    t, xi = _query(desc, "fp8", params, rays, dev, np.array(scales, dtype=np.float32))
    te, _, _, _ = O.ddf_query_emulated(desc, params, rs, "fp8", act_scales=scales)
    d = np.abs(t.cpu().numpy()[idx] - te)
    assert d.mean() <= 0.75 * np.abs(te - t64).mean()
    t, xi = _query(desc, "bf16", params, rays, dev)
    te, _, _, _ = O.ddf_query_emulated(desc, params, rs, "bf16")
    assert np.abs(t.cpu().numpy()[idx] - te).mean() <= 1e-3


def test_train_step_262144_rays_16x1024_bf16_recompute4():
    """The large training configuration: batch 262,144 against 1,024 ellipsoids, 16 x 1024
    net, bf16, activation recomputation every 4 layers.  At full size: sampled logits against
    the emulated bf16 oracle; the loss against the oracle's loss of the kernel's own logits;
    the gradient additive over the two halves of the batch; Adam against the oracle's update
    from the kernel's gradient; a repeat of the step bit-identical."""
    dev = cuda()
    desc = I.NET_LARGE
    B, k = 1 << 18, 4
    sc = I.scene_ellipsoids(1024, 3)
    rays_np = I.train_rays(sc, B, 1300)
    rays = _t(rays_np, dev)
    tg, hit = ddf.cast_targets(_t(ddf.scene_prims(sc), dev), rays)
    params = I.he_init(desc, 0)
    P = desc.param_count()
    ws = torch.empty(ddf.train_workspace_bytes(desc, "bf16", B, k), dtype=torch.uint8, device=dev)
    assert ws.numel() < ddf.train_workspace_bytes(desc, "bf16", B, 0) * 0.6
    master0 = _t(params, dev)
    packed0 = ddf.pack(desc, "bf16", master0)

    zt, zx = ddf.forward_train(desc, "bf16", packed0, rays, ws, k)
    torch.cuda.synchronize()
    zt_h, zx_h = zt.cpu().numpy(), zx.cpu().numpy()
    assert np.isfinite(zt_h).all() and np.isfinite(zx_h).all()
    idx = _sample(B)
    _, _, zte, zxe = O.ddf_query_emulated(desc, params, rays_np[:, idx], "bf16")
    dz = np.abs(zt_h[idx] - zte)
    assert dz.mean() <= 2e-3 * max(1.0, np.abs(zte).mean()) and np.abs(zx_h[idx] - zxe).mean() <= 2e-3 * max(
        1.0, np.abs(zxe).mean())

    def step():
        master = master0.clone()
        m = torch.zeros_like(master); v = torch.zeros_like(master)
        packed = packed0.clone()
        grad = torch.empty(P, dtype=torch.float32, device=dev)
        hp = ddf.TrainHParamsC(3e-3, 0.9, 0.999, 1e-8, O.BCE_WEIGHT, O.L1_CLAMP, 1, k)
        loss, flag = ddf.train_step(desc, "bf16", master, m, v, packed, rays, tg, hit, hp, ws, grad_out=grad)
        torch.cuda.synchronize()
        assert int(flag.cpu()[0]) == 0
        return [x.cpu().numpy() for x in (loss, master, m, v, grad)]

    loss, master, m, v, grad = step()
    (tot, l1, bce), dzt64, dzx64 = O.loss_terms(zt_h.astype(np.float64), zx_h.astype(np.float64),
                                                tg.cpu().numpy().astype(np.float64), hit.cpu().numpy())
    np.testing.assert_allclose(loss[:3], [tot, l1, bce], rtol=1e-5)

    # additivity over the two halves, with the oracle's logit gradients as upstream gradients
    dzt_d = _t(dzt64.astype(np.float32), dev); dzx_d = _t(dzx64.astype(np.float32), dev)
    ddf.forward_train(desc, "bf16", packed0, rays, ws, k)
    g_full = ddf.backward(desc, "bf16", packed0, rays, dzt_d, dzx_d, ws, k)
    h = B // 2
    parts = []
    for sl in (slice(0, h), slice(h, B)):
        r = rays[:, sl].contiguous()
        ddf.forward_train(desc, "bf16", packed0, r, ws, k)
        parts.append(ddf.backward(desc, "bf16", packed0, r, dzt_d[sl].contiguous(), dzx_d[sl].contiguous(), ws, k))
    torch.cuda.synchronize()
    gf = g_full.cpu().numpy().astype(np.float64)
    gs = parts[0].cpu().numpy().astype(np.float64) + parts[1].cpu().numpy().astype(np.float64)
    for (w_off, b_off, o, i) in desc.offsets():
        sl = slice(w_off, b_off + o)
        assert np.linalg.norm(gf[sl] - gs[sl]) <= 1e-4 * np.linalg.norm(gf[sl])
    assert np.linalg.norm(grad - gf) <= 1e-4 * np.linalg.norm(gf)

    # Adam from the kernel's gradient
    p1, m1, v1 = O.adam_step(params.astype(np.float64), np.zeros(P), np.zeros(P), grad.astype(np.float64), 1, 3e-3)
    np.testing.assert_allclose(m, m1, rtol=1e-5, atol=1e-6 * np.abs(m1).max())
    np.testing.assert_allclose(v, v1, rtol=1e-4, atol=1e-6 * np.abs(v1).max())
    big = np.abs(grad) > 1e-6 * np.abs(grad).max()
    np.testing.assert_allclose(master[big], p1[big], rtol=0, atol=1e-6)

    again = step()
    for a, b in zip((loss, master, m, v, grad), again):
        np.testing.assert_array_equal(a, b)

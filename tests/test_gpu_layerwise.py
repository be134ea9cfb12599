"""One hidden layer at a time: the kernel's own layer input through the oracle's layer.

The query kernels expose the last hidden layer's float32 output (ddf_query_hidden).  Cutting
the 12 x 1024 network after layer l gives the kernel's h_l; the oracle's emulated layer l + 1
(the kernels' roundings, exact arithmetic: oracle.ddf_oracle.hidden_layer_emulated) applied to
that h_l must then reproduce the kernel's h_(l+1) within the rigorous float32 accumulation
bound of one layer,

    |h_k - h_ref| <= gamma_(K+2) (|x_q| |W_q|^T + |b|),   gamma_k = k u / (1 - k u),

for every ray and neuron (ReLU is 1-Lipschitz; x_q, W_q the operands after the format's
rounding).  This separates a mismatch inside one layer (operand rounding, scale, bias, ReLU)
from the cascade of rounding flips across layers, which the end-to-end tests see: a float32
accumulation difference that moves a value across a bf16 / e4m3 rounding boundary changes that
operand by a whole step, and the later layers carry it on.  The cascade is reported per layer as
the share of next-layer operands whose rounded value differs between the kernel's chain and
the exactly accumulated emulation.
"""
import numpy as np
import pytest
import torch

from oracle import ddf_oracle as O
from paper_2606_00817_amd import ddf
from paper_2606_00817_amd import inputs as I
from tests.helpers import cuda, gamma, U32

pytestmark = pytest.mark.gpu


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def cut_after(desc, params, l):
    """The first l hidden layers of `params` and its head: a network of n_hidden = l."""
    offs = desc.offsets()
    w_off, b_off, o, _ = offs[l - 1]
    hw, hb, ho, _ = offs[-1]
    d = I.NetDesc(desc.n_in, desc.n_freq, l, desc.width, desc.n_out)
    return d, np.concatenate([params[:b_off + o], params[hw:hb + ho]]).astype(np.float32)


def _operand(x, precision, s_a=None):
    """A layer input as the matrix cores read it (the format's rounding), in float64."""
    if precision == "bf16":
        return O.round_bf16(x)
    if precision == "fp8":
        return O.round_e4m3(np.asarray(x) / s_a) * s_a
    return np.asarray(x, dtype=np.float64)


def _weight_operand(W, precision, s_w=None):
    if precision == "bf16":
        return O.round_bf16(W)
    if precision == "fp8":
        return O.round_e4m3(W / s_w) * s_w
    return W


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_each_layer_within_accumulation_bound(precision):
    dev = cuda()
    desc = I.NET_FULL
    params = I.test_params(desc, 4)
    L = O.layers(desc, params)
    sc = I.scene_mixed(256, 2)
    rays = I.shadow_rays(sc, 128 * 3 + 37, 14)          # four 128-ray tiles, the last ragged
    scales = sw = None
    if precision == "fp8":
        calib = I.free_rays(sc, 4096, 21)
        scales = O.act_scales_fp8(desc, params, calib)
        sw = O.weight_scales_fp8(desc, params)
    g = O.encode(O.rays_to_inputs(rays), desc.n_freq)
    # the exactly accumulated emulation of the whole chain (for the cascade report)
    hs_emu, _ = (O.mlp_forward(desc, params, g) if precision == "fp32"
                 else O.mlp_forward_emulated(desc, params, g, precision, act_scales=scales))
    rays_d = _t(rays, dev)
    h_prev = None
    report = []
    for l in range(1, desc.n_hidden + 1):
        dl, pl = cut_after(desc, params, l)
        packed = ddf.pack(dl, precision, _t(pl, dev),
                          act_scales=None if scales is None else np.array(scales[:l - 1], dtype=np.float32))
        h = ddf.query_hidden(dl, precision, packed, rays_d).cpu().numpy().astype(np.float64)
        W, b = L[l - 1]
        if l == 1:
            # layer 1 reads the encoding: float32 sinpi / cospi (a few ulp), and in the reduced
            # precisions its bf16 hi + lo split (<= 2^-18 relative); weights bf16 there
            Wq = W if precision == "fp32" else O.round_bf16(W)
            ref = np.maximum(g @ Wq.T + b, 0.0)
            e_in = 4 * U32 * (np.abs(g) + 1.0) + (0.0 if precision == "fp32" else 2.0 ** -17 * np.abs(g))
            K = g.shape[1] * (1 if precision == "fp32" else 2)
            bound = e_in @ np.abs(Wq).T + gamma(K + 2) * (np.abs(g) * 1.01 @ np.abs(Wq).T + np.abs(b))
        else:
            s_a = scales[l - 2] if precision == "fp8" else None
            s_w = sw[l - 2] if precision == "fp8" else None
            ref = O.hidden_layer_emulated(W, b, h_prev, precision, s_a, s_w)
            xq = _operand(h_prev, precision, s_a)
            Wq = _weight_operand(W, precision, s_w)
            bound = gamma(W.shape[1] + 2) * (np.abs(xq) @ np.abs(Wq).T + np.abs(b))
        err = np.abs(h - ref)
        ratio = float((err / np.maximum(bound, 1e-300)).max())
        # cascade: next-layer operands that differ from the exactly accumulated chain (float32
        # operands are never rounded: the share is reported for the reduced precisions only)
        s_next = scales[min(l, desc.n_hidden - 1) - 1] if precision == "fp8" else None
        flips = (float((_operand(h, precision, s_next) != _operand(hs_emu[l - 1], precision, s_next)).mean())
                 if precision != "fp32" else float("nan"))
        report.append((l, ratio, flips))
        assert np.isfinite(h).all()
        assert np.all(err <= bound), (precision, l, ratio)
        h_prev = h
    print(f"\n{precision} 12x1024, one layer at a time (max error / bound, share of rounded operands "
          f"that differ from the exact chain):")
    for l, r, f in report:
        print(f"  layer {l:2d}: {r:.3f}  {f:.2e}")

"""Shared helpers of the test suite (tolerances, planted networks, device plumbing)."""
import math

import numpy as np
import pytest

from oracle import ddf_oracle as O
from paper_2606_00817_amd import inputs as I
from paper_2606_00817_amd.inputs import planted_box_sdf  # noqa: F401

U32 = 2.0 ** -24   # unit roundoff of float32


def gamma(k):
    """gamma_k = k u / (1 - k u): worst-case relative error of a k-term float32 dot product."""
    return k * U32 / (1.0 - k * U32)


def fp32_forward_bound(desc, params, rays):
    """Rigorous per-ray bound on |z_fp32 - z_exact| for any float32 evaluation order.

    The encoding is charged 4 ulp per feature (sinpi/cospi), every dot product of K
    terms gamma_(K+2) (products, sums and the bias), and ReLU is 1-Lipschitz:
      e_0 = 4u |gamma|,  e_l = |W_l| e_(l-1) + gamma_(K+2) (|W_l| |h_(l-1)| + |b_l|)."""
    L = O.layers(desc, params)
    g = O.encode(O.rays_to_inputs(rays), desc.n_freq)
    hs, z = O.mlp_forward(desc, params, g)
    ins = [g] + hs
    e = 4 * U32 * np.maximum(np.abs(g), 1.0)
    for li, (W, b) in enumerate(L):
        K = W.shape[1]
        aW = np.abs(W)
        e = e @ aW.T + gamma(K + 2) * (np.abs(ins[li]) @ aW.T + np.abs(b))
    return z, e      # z [N, n_out] exact logits, e [N, n_out] bounds


def box_sdf(p, half):
    return np.max(np.abs(p) - np.asarray(half), axis=1)


def fp32_forward_sigma(desc, params, rays):
    """First-order estimate of the float32 rounding error of the logits, per ray.

    Rounding errors are treated as independent with random signs (the usual
    first-order model).  A K-term dot product evaluated in float32 in any order
    carries variance about u^2 (K/2 + 1) sum_k (w_k h_k)^2 (each partial sum is
    rounded once, partial sums of random-sign terms grow like sqrt(i)), and an
    input error e propagates through W linearly and through ReLU only where the
    unit is active:
      s_0^2 = (2u gamma)^2
      s_l^2 = (W_l^2) (m_(l-1) s_(l-1)^2) + u^2 (K/2 + 1) (W_l^2)(h_(l-1)^2).
    Returns (z exact [N, n_out], sigma [N, n_out])."""
    L = O.layers(desc, params)
    g = O.encode(O.rays_to_inputs(rays), desc.n_freq)
    hs, z = O.mlp_forward(desc, params, g)
    ins = [g] + hs
    var = (2 * U32 * g) ** 2
    for li, (W, b) in enumerate(L):
        K = W.shape[1]
        W2 = W * W
        if li > 0:
            var = var * (ins[li] > 0)
        var = var @ W2.T + U32 ** 2 * (K / 2 + 1) * ((ins[li] ** 2) @ W2.T)
    return z, np.sqrt(var)


def kink_rays(desc, params, rays, k_sigma=8.0):
    """Rays with a hidden unit whose pre-activation lies within k sigma of 0.

    sigma is the first-order float32 rounding error of that pre-activation (the model
    of fp32_forward_sigma).  On such a ray float32 and float64 may disagree about the
    ReLU, which changes that ray's whole gradient row; parity tests give these rays
    no gradient on both sides."""
    L = O.layers(desc, params)
    g = O.encode(O.rays_to_inputs(rays), desc.n_freq)
    h = g
    var = (2 * U32 * g) ** 2
    bad = np.zeros(len(g), dtype=bool)
    for li, (W, b) in enumerate(L[:-1]):
        K = W.shape[1]
        W2 = W * W
        var = var @ W2.T + U32 ** 2 * (K / 2 + 1) * ((h ** 2) @ W2.T)
        a = h @ W.T + b
        bad |= np.any(np.abs(a) < k_sigma * np.sqrt(var) + 1e-30, axis=1)
        var = var * (a > 0)
        h = np.maximum(a, 0.0)
    return bad


def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def bf16_grad_fp32_accum(desc, params, gam, dz):
    """The bf16 training gradient with the kernels' rounding points (as
    oracle.ddf_oracle.mlp_backward_emulated_bf16) but every product summed in float32
    (numpy's float32 matmul, another valid summation order).  Its distance from the exactly
    accumulated emulation measures how far any float32-accumulating implementation may land
    from it: a float32 difference that moves a value across a bf16 rounding boundary flips a
    whole bf16 step, later layers carry it on, and a pre-activation near 0 flips its ReLU.
    Also returns the post-ReLU activations of the float32-summed forward."""
    f32 = np.float32

    def mm(a, b):
        return (np.asarray(a, dtype=f32) @ np.asarray(b, dtype=f32)).astype(np.float64)
    L = O.layers(desc, params)
    hi, lo = O.split_bf16(gam)
    W1, b1 = L[0]
    W1q = O.round_bf16(W1)
    h = np.maximum(mm(hi, W1q.T) + mm(lo, W1q.T) + b1, 0.0)
    hs = [h]
    for W, b in L[1:-1]:
        h = np.maximum(mm(O.round_bf16(h), O.round_bf16(W).T) + b, 0.0)
        hs.append(h)
    ins = [O.round_bf16(gam)] + [O.round_bf16(x) for x in hs]
    dz = np.asarray(dz, dtype=np.float64)
    grads = [None] * len(L)
    Wh, _ = L[-1]
    grads[-1] = (mm(dz.T, ins[-1]), dz.sum(axis=0))
    da = O.round_bf16(mm(dz, Wh) * (hs[-1] > 0.0))
    for l in range(len(L) - 2, -1, -1):
        W, _ = L[l]
        grads[l] = (mm(da.T, ins[l]), da.sum(axis=0))
        if l > 0:
            da = O.round_bf16(mm(da, O.round_bf16(W)) * (hs[l - 1] > 0.0))
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads]), hs

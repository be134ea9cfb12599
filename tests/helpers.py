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

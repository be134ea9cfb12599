"""Plain float64 oracle of the directed distance field (DDF) hot path.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It is written from the paper's
definitions, layer by layer, with numpy matmuls as the only library
primitive, and it shares no code with the HIP path.

What is computed (paper references by section / equation):

* The DDF maps a ray (origin x in R^3, unit direction d) to (t, xi): the
  distance to the first surface along d and the probability that the ray
  hits at all (Sec. III-A, Eq. 1).
* The field is the sinusoidal-encoding form with a dense ReLU network of the
  encoding comparison (Sec. IV-C, Table II): v = (x, d) is encoded as
  gamma(v) = [v, sin(pi 2^0 v), cos(pi 2^0 v), ..., sin(pi 2^(L-1) v), cos(pi 2^(L-1) v)]
  (each block holds all n_in coordinates), i.e. n_in (1 + 2L) features,
  followed by n_hidden Linear+ReLU layers (the first maps the features to the
  width) and a linear head.  The distance is t = softplus(z_t) and the
  visibility xi = sigmoid(z_xi).
* Distillation (Sec. III-B, III-D): an L1 term on distance, clamped at the box
  scale, over rays that hit, plus a cross-entropy term on the hit flag
  weighted 0.3; Adam; learning rate 3e-3 cosine-decayed to 5 %.
* Reduced-precision queries (Sec. III-C): emulated here exactly as the
  kernels round, so that a BF16 / FP8 kernel can be checked tightly.
* The SDF baseline evaluates the same kind of MLP (n_in = 3, one linear
  output) inside the sphere-tracing loop of geometry.sphere_trace.
"""
from __future__ import annotations

import math

import numpy as np

BCE_WEIGHT = 0.3     # weight of the hit cross-entropy (Sec. III-D)
L1_CLAMP = 3.0       # clamp of the L1 distance term: the edge of the [-1.5, 1.5]^3 box


# ----------------------------------------------------------------------------
# Network description (mirrors the flat parameter layout of the inputs module)
# ----------------------------------------------------------------------------

def layers(desc, params):
    """[(W [out, in], b [out])] in float64, hidden layers first, head last."""
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    fan_in = desc.n_in * (1 + 2 * desc.n_freq)
    shapes = [(desc.width, fan_in)] + [(desc.width, desc.width)] * (desc.n_hidden - 1) + \
             [(desc.n_out, desc.width)]
    for o, i in shapes:
        W = p[off:off + o * i].reshape(o, i); off += o * i
        b = p[off:off + o]; off += o
        out.append((W, b))
    assert off == p.size, "parameter vector does not match the net description"
    return out


# ----------------------------------------------------------------------------
# Encoding and forward pass
# ----------------------------------------------------------------------------

def sinpi(a):
    """sin(pi a) with the argument reduced exactly modulo 2 first."""
    return np.sin(np.pi * np.remainder(a, 2.0))


def cospi(a):
    """cos(pi a) with the argument reduced exactly modulo 2 first."""
    return np.cos(np.pi * np.remainder(a, 2.0))


def encode(v, n_freq):
    """Sinusoidal positional encoding gamma(v) of [N, n_in] inputs -> [N, n_in (1 + 2L)]."""
    v = np.asarray(v, dtype=np.float64)
    feats = [v]
    for k in range(n_freq):
        a = (2.0 ** k) * v
        feats.append(sinpi(a))
        feats.append(cospi(a))
    return np.concatenate(feats, axis=1)


def softplus(z):
    """log(1 + e^z) in the overflow-free form max(z, 0) + log1p(e^-|z|)."""
    z = np.asarray(z, dtype=np.float64)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def mlp_forward(desc, params, gamma):
    """Hidden activations h_1..h_n and head logits z [N, n_out] for encoded inputs."""
    L = layers(desc, params)
    h = np.asarray(gamma, dtype=np.float64)
    hs = []
    for W, b in L[:-1]:
        h = np.maximum(h @ W.T + b, 0.0)
        hs.append(h)
    Wh, bh = L[-1]
    return hs, h @ Wh.T + bh


def rays_to_inputs(rays):
    """[6, N] (or [3, N]) SoA float32 rays -> [N, n_in] float64 rows (exact promotion)."""
    return np.asarray(rays, dtype=np.float64).T


def ddf_query(desc, params, rays, chunk=8192):
    """The batched DDF query: (t, xi, z_t, z_xi) per ray, all float64."""
    v = rays_to_inputs(rays)
    zs = []
    for s in range(0, len(v), chunk):
        _, z = mlp_forward(desc, params, encode(v[s:s + chunk], desc.n_freq))
        zs.append(z)
    z = np.concatenate(zs) if zs else np.zeros((0, desc.n_out))
    return softplus(z[:, 0]), sigmoid(z[:, 1]), z[:, 0], z[:, 1]


def sdf_eval(desc, params, points, chunk=8192):
    """Signed distance predicted by an SDF MLP (n_in = 3, one linear output) at [M, 3] points."""
    p = np.asarray(points, dtype=np.float64)
    out = []
    for s in range(0, len(p), chunk):
        _, z = mlp_forward(desc, params, encode(p[s:s + chunk], desc.n_freq))
        out.append(z[:, 0])
    return np.concatenate(out) if out else np.zeros(0)


# ----------------------------------------------------------------------------
# Reduced-precision number formats (round to nearest, ties to even)
# ----------------------------------------------------------------------------

def round_bf16(x):
    """Nearest bfloat16 value (8 significant bits, float32 exponent range), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)                  # below 2^-126 the spacing stops shrinking
    scale = np.ldexp(1.0, 8 - e)             # integer grid of 8 significant bits
    r = np.rint(x * scale) / scale           # np.rint rounds half to even
    big = np.abs(r) > 3.3895313892515355e38  # above the largest finite bfloat16
    return np.where(np.isfinite(x), np.where(big, np.copysign(np.inf, x), r), x)


def _e4m3_table():
    """All non-negative finite OCP e4m3fn values, ascending, with their 7-bit codes."""
    vals, codes = [], []
    for code in range(0x7F):                  # 0x7F is NaN
        e = code >> 3
        m = code & 7
        v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
        vals.append(v); codes.append(code)
    return np.array(vals), np.array(codes)


E4M3_VALUES, E4M3_CODES = _e4m3_table()
E4M3_MAX = 448.0


def round_e4m3(x):
    """Nearest OCP e4m3fn value with saturation to +-448, ties to the even code."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.searchsorted(E4M3_VALUES, a, side='left')        # first value >= a
    hi = np.minimum(hi, len(E4M3_VALUES) - 1)
    lo = np.maximum(hi - 1, 0)
    vlo, vhi = E4M3_VALUES[lo], E4M3_VALUES[hi]
    dlo, dhi = a - vlo, vhi - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (E4M3_CODES[hi] % 2 == 0))
    r = np.where(a >= vhi, vhi, np.where(pick_hi, vhi, vlo))
    return np.where(np.isnan(x), np.nan, np.copysign(r, x))


def pow2_scale(amax, fmt_max=E4M3_MAX):
    """Smallest power of two s with amax / s <= fmt_max (1.0 for amax == 0)."""
    if not amax > 0:
        return 1.0
    return float(2.0 ** math.ceil(math.log2(amax / fmt_max)))


# ----------------------------------------------------------------------------
# Emulated reduced-precision forward (the kernels' rounding, exact arithmetic)
# ----------------------------------------------------------------------------

def split_bf16(x):
    """x ~ hi + lo with hi = bf16(x), lo = bf16(x - hi): about 16 significant bits."""
    hi = round_bf16(x)
    return hi, round_bf16(np.asarray(x, dtype=np.float64) - hi)


def weight_scales_fp8(desc, params):
    """Per hidden layer l >= 2 power-of-two weight scale s_W = 2^ceil(log2(amax|W_l| / 448))."""
    L = layers(desc, params)
    return [pow2_scale(float(np.max(np.abs(W)))) for W, _ in L[1:-1]]


def act_scales_fp8(desc, params, calib_rays):
    """Per hidden layer l >= 2 power-of-two input scale from the float64 forward on a calibration batch."""
    hs, _ = mlp_forward(desc, params, encode(rays_to_inputs(calib_rays), desc.n_freq))
    return [pow2_scale(float(np.max(h))) for h in hs[:-1]]


def hidden_layer_emulated(W, b, x, precision, s_a=None, s_w=None):
    """One hidden layer l >= 2 from its input x [N, width] with the kernels' roundings.

    'fp32': relu(x W^T + b), no rounding.  'bf16': relu(bf16(x) bf16(W)^T + b).
    'fp8': relu((e4m3(x / s_a) e4m3(W / s_w)^T) s_a s_w + b) with power-of-two scales.
    Products and sums exact (float64: every product of two bf16 or e4m3 values is exact,
    and a 1024-term sum of them loses nothing measurable against float32)."""
    x = np.asarray(x, dtype=np.float64)
    if precision == 'fp32':
        a = x @ W.T + b
    elif precision == 'bf16':
        a = round_bf16(x) @ round_bf16(W).T + b
    elif precision == 'fp8':
        a = (round_e4m3(x / s_a) @ round_e4m3(W / s_w).T) * (s_a * s_w) + b
    else:
        raise ValueError(precision)
    return np.maximum(a, 0.0)


def mlp_forward_emulated(desc, params, gamma, precision, act_scales=None):
    """Forward pass with the kernels' roundings, every other operation exact (float64).

    precision 'fp32': no rounding (the float64 forward).
    precision 'bf16': layer 1 takes gamma split as bf16 hi + lo with bf16
      weights; hidden layers take bf16 inputs and bf16 weights; every
      product is accumulated exactly; bias, ReLU and the heads are exact and
      the heads read the unrounded last hidden layer.
    precision 'fp8': layer 1 as for bf16; layer l >= 2 takes
      e4m3(h_{l-1} / s_A) and e4m3(W_l / s_W) with power-of-two scales and
      rescales the exact sum by s_A s_W."""
    L = layers(desc, params)
    g = np.asarray(gamma, dtype=np.float64)
    if precision == 'fp32':
        return mlp_forward(desc, params, g)
    hi, lo = split_bf16(g)
    W1, b1 = L[0]
    h = np.maximum((hi + lo) @ round_bf16(W1).T + b1, 0.0)
    hs = [h]
    sw = weight_scales_fp8(desc, params) if precision == 'fp8' else None
    for li, (W, b) in enumerate(L[1:-1]):
        if precision == 'fp8':
            h = hidden_layer_emulated(W, b, h, 'fp8', act_scales[li], sw[li])
        elif precision == 'bf16':
            h = hidden_layer_emulated(W, b, h, 'bf16')
        else:
            raise ValueError(precision)
        hs.append(h)
    Wh, bh = L[-1]
    return hs, h @ Wh.T + bh


def ddf_query_emulated(desc, params, rays, precision, act_scales=None, chunk=8192):
    v = rays_to_inputs(rays)
    zs = []
    for s in range(0, len(v), chunk):
        _, z = mlp_forward_emulated(desc, params, encode(v[s:s + chunk], desc.n_freq), precision,
                                    act_scales)
        zs.append(z)
    z = np.concatenate(zs) if zs else np.zeros((0, desc.n_out))
    return softplus(z[:, 0]), sigmoid(z[:, 1]), z[:, 0], z[:, 1]


# ----------------------------------------------------------------------------
# Distillation loss, backward pass, Adam
# ----------------------------------------------------------------------------

def loss_terms(z_t, z_xi, t_gt, hit, bce_weight=BCE_WEIGHT, clamp=L1_CLAMP):
    """(total, l1, bce) and per-ray logit gradients (dL/dz_t, dL/dz_xi).

    l1  = mean over hit rays of min(|softplus(z_t) - t_gt|, clamp)  (0 with no hits)
    bce = mean over all rays of -[y log sigmoid(z_xi) + (1 - y) log(1 - sigmoid(z_xi))]
    total = l1 + bce_weight * bce.
    The clamp passes gradient where |u| <= clamp (inclusive), the sign of 0 is 0."""
    z_t = np.asarray(z_t, dtype=np.float64); z_xi = np.asarray(z_xi, dtype=np.float64)
    y = np.asarray(hit).astype(np.float64)
    n = len(z_t)
    n_hit = int(y.sum())
    t_hat = softplus(z_t)
    tg = np.where(y > 0, np.asarray(t_gt, dtype=np.float64), 0.0)
    u = t_hat - tg
    l1_i = np.where(y > 0, np.minimum(np.abs(u), clamp), 0.0)
    l1 = math.fsum(l1_i) / n_hit if n_hit else 0.0
    bce_i = softplus(z_xi) - y * z_xi            # = -log-likelihood of y under sigmoid(z_xi)
    bce = math.fsum(bce_i) / n if n else 0.0
    g_t = np.where((y > 0) & (np.abs(u) <= clamp), np.sign(u), 0.0)
    g_t = g_t / n_hit if n_hit else g_t * 0.0
    dz_t = g_t * sigmoid(z_t)
    dz_xi = bce_weight * (sigmoid(z_xi) - y) / n if n else z_xi * 0.0
    return (l1 + bce_weight * bce, l1, bce), dz_t, dz_xi


def mlp_backward(desc, params, gamma, dz):
    """Gradient of sum(dz * z) w.r.t. the flat parameter vector (float64, same layout)."""
    L = layers(desc, params)
    hs, _ = mlp_forward(desc, params, gamma)
    ins = [np.asarray(gamma, dtype=np.float64)] + hs
    grads = [None] * len(L)
    dz = np.asarray(dz, dtype=np.float64)
    Wh, _ = L[-1]
    grads[-1] = (dz.T @ ins[-1], dz.sum(axis=0))
    dh = dz @ Wh
    for l in range(len(L) - 2, -1, -1):
        W, _ = L[l]
        da = dh * (hs[l] > 0.0)
        grads[l] = (da.T @ ins[l], da.sum(axis=0))
        dh = da @ W
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def mlp_backward_emulated_bf16(desc, params, gamma, dz):
    """Parameter gradient with the bf16 training path's roundings, exact arithmetic otherwise.

    Forward as mlp_forward_emulated(.., 'bf16'); every stored activation is bf16(h_l)
    and the stored features are bf16(gamma) (the hi part).  Backward: delta_n =
    bf16((dz W_head) * 1[h_n > 0]); delta_(l-1) = bf16((delta_l bf16(W_l)) * 1[h_(l-1) > 0]);
    dW_l = delta_l^T bf16(h_(l-1)) and db_l = sum delta_l over rays; the head gradient
    reads bf16(h_n)."""
    L = layers(desc, params)
    hs, _ = mlp_forward_emulated(desc, params, gamma, 'bf16')
    ins = [round_bf16(gamma)] + [round_bf16(h) for h in hs]
    dz = np.asarray(dz, dtype=np.float64)
    grads = [None] * len(L)
    Wh, _ = L[-1]
    grads[-1] = (dz.T @ ins[-1], dz.sum(axis=0))
    da = round_bf16((dz @ Wh) * (hs[-1] > 0.0))
    for l in range(len(L) - 2, -1, -1):
        W, _ = L[l]
        grads[l] = (da.T @ ins[l], da.sum(axis=0))
        if l > 0:
            da = round_bf16((da @ round_bf16(W)) * (hs[l - 1] > 0.0))
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def ddf_loss_and_grad(desc, params, rays, t_gt, hit, **kw):
    """Distillation loss terms and the flat parameter gradient for one batch."""
    g = encode(rays_to_inputs(rays), desc.n_freq)
    _, z = mlp_forward(desc, params, g)
    terms, dz_t, dz_xi = loss_terms(z[:, 0], z[:, 1], t_gt, hit, **kw)
    grad = mlp_backward(desc, params, g, np.stack([dz_t, dz_xi], axis=1))
    return terms, grad


def sdf_loss_and_grad(desc, params, points, sdf_gt):
    """Fitting loss of an SDF MLP, mean |s(p) - sdf_gt(p)| (sign(0) = 0), and its gradient."""
    g = encode(np.asarray(points, dtype=np.float64), desc.n_freq)
    _, z = mlp_forward(desc, params, g)
    u = z[:, 0] - np.asarray(sdf_gt, dtype=np.float64)
    n = len(u)
    loss = math.fsum(np.abs(u)) / n
    grad = mlp_backward(desc, params, g, (np.sign(u) / n)[:, None])
    return loss, grad


def adam_step(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba, Algorithm 1); returns new (p, m, v)."""
    p = np.asarray(p, dtype=np.float64); m = np.asarray(m, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64); g = np.asarray(g, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def lr_schedule(step, total=30000, lr0=3e-3, final_frac=0.05):
    """Cosine decay from lr0 to final_frac * lr0 over `total` steps (Sec. III-D)."""
    s = min(max(step, 0), total)
    lo = lr0 * final_frac
    return lo + 0.5 * (lr0 - lo) * (1.0 + math.cos(math.pi * s / total))


SHIFT_WALK = 1024   # rays searched for a hit from the drawn start index


def shift_rays(rays, t_gt, hit, u, frac):
    """Self-consistency points (Sec. III-B: along a ray that hits at t, the point moved
    forward by s must report t - s; Sec. III-D: 30 % of each batch).

    Slot i with u[0][i] < frac takes the first hit ray j among the SHIFT_WALK rays from
    index floor(u[1][i] n) on (cyclically) and becomes the ray from x_j + s d_j along d_j
    with target t_j - s, s = u[2][i] t_j; every other slot, and a selected slot that finds
    no hit, keeps its own ray.  The index decisions (u < frac, floor(u n)) and s are taken
    in float32, as the uniforms are float32 draws; origins and targets come back in float64.
    Returns (rays [6][n] float64, t [n] float64, hit [n] uint8, src [n] int64, shifted [n] bool)."""
    r = np.asarray(rays, dtype=np.float64)
    n = r.shape[1]
    t = np.asarray(t_gt, dtype=np.float64).copy()
    h = np.asarray(hit).astype(np.uint8).copy()
    u32 = np.asarray(u, dtype=np.float32)
    out = r.copy()
    src = np.arange(n)
    shifted = np.zeros(n, dtype=bool)
    hit_idx = np.asarray(hit).astype(bool)
    for i in range(n):
        if not (u32[0, i] < np.float32(frac)):
            continue
        c = min(int(np.floor(u32[1, i] * np.float32(n))), n - 1)
        for k in range(min(n, SHIFT_WALK)):
            j = (c + k) % n
            if hit_idx[j]:
                s = float(np.float32(u32[2, i] * np.float32(t_gt[j])))
                out[0:3, i] = r[0:3, j] + s * r[3:6, j]
                out[3:6, i] = r[3:6, j]
                t[i] = float(t_gt[j]) - s
                h[i] = 1
                src[i] = j
                shifted[i] = True
                break
    return out, t, h, src, shifted

"""Thin Python binding of libddf (include/ddf.h): argument marshalling only.

Every computation runs in the HIP library; this module only checks tensor
placement/dtypes, allocates outputs with PyTorch (device memory and streams
are PyTorch's job here) and forwards raw pointers plus the current HIP stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddf.so")

FP32, BF16, FP8 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8}


class DDFError(RuntimeError):
    pass


class NetDescC(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_freq", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("width", ctypes.c_int32), ("n_out", ctypes.c_int32), ("precision", ctypes.c_int32)]


class TrainHParamsC(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("bce_weight", ctypes.c_float), ("l1_clamp", ctypes.c_float),
                ("step", ctypes.c_int64), ("recompute_every", ctypes.c_int32)]


class HashDescC(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_feat", ctypes.c_int32), ("log2_table", ctypes.c_int32),
                ("base_res", ctypes.c_int32), ("growth", ctypes.c_float), ("dir_bands", ctypes.c_int32),
                ("width", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("box_half", ctypes.c_float)]


class CameraC(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("target", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.POINTER(NetDescC)

SIGNATURES = {
    "ddf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ddf_last_error": (ctypes.c_char_p, []),
    "ddf_param_count": (_SZ, [_D]),
    "ddf_param_offsets": (ctypes.c_int, [_D, ctypes.c_int32, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)]),
    "ddf_packed_bytes": (_SZ, [_D]),
    "ddf_pack": (ctypes.c_int, [_D, _P, ctypes.POINTER(ctypes.c_float), _P, _P]),
    "ddf_query": (ctypes.c_int, [_D, _P, _P, _I64, _P, _P, _P]),
    "ddf_query_split_workspace_bytes": (_SZ, [_D, _I64]),
    "ddf_query_split": (ctypes.c_int, [_D, _P, _P, _I64, _P, _P, _P, _SZ, _P]),
    "ddf_fp8_calib_workspace_bytes": (_SZ, [_D, _I64]),
    "ddf_fp8_act_scales": (ctypes.c_int, [_D, _P, _P, _I64, ctypes.POINTER(ctypes.c_float), _P, _SZ, _P]),
    "ddf_train_workspace_bytes": (_SZ, [_D, _I64, ctypes.c_int32]),
    "ddf_forward_train": (ctypes.c_int, [_D, _P, _P, _I64, _P, _P, ctypes.c_int32, _P, _SZ, _P]),
    "ddf_backward": (ctypes.c_int, [_D, _P, _P, _I64, _P, _P, _P, ctypes.c_int32, _P, _SZ, _P]),
    "ddf_train_step": (ctypes.c_int, [_D, _P, _P, _P, _P, _P, _P, _P, _I64, ctypes.POINTER(TrainHParamsC),
                                      _P, _P, _P, _P, _SZ, _P]),
    "sdf_trace_workspace_bytes": (_SZ, [_I64]),
    "sdf_sphere_trace": (ctypes.c_int, [_D, _P, _P, _I64, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                        _P, _P, _P, _P, _SZ, _P]),
    "sdf_sphere_trace_pool": (ctypes.c_int, [_D, _P, _P, _I64, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                             _P, _P, _P, _P, _SZ, _P]),
    "sdf_eval": (ctypes.c_int, [_D, _P, _P, _I64, _P, _P]),
    "ddf_query_hidden": (ctypes.c_int, [_D, _P, _P, _I64, _P, _P]),
    "ddf_train_kept_activation": (ctypes.c_int, [_D, _I64, ctypes.c_int32, _P, _SZ, ctypes.c_int32, _P, _P]),
    "ddf_cast_targets": (ctypes.c_int, [_P, ctypes.c_int32, _P, _I64, _P, _P, _P]),
    "ddf_scene_sdf": (ctypes.c_int, [_P, ctypes.c_int32, _P, _I64, _P, _P]),
    "ddf_shift_rays": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_float, _I64, _P, _P, _P, _P]),
    "ddf_lr_cosine": (ctypes.c_float, [_I64, _I64, ctypes.c_float, ctypes.c_float]),
    "ddf_hash_param_count": (_SZ, [ctypes.POINTER(HashDescC)]),
    "ddf_hash_level": (ctypes.c_int, [ctypes.POINTER(HashDescC), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int32)]),
    "ddf_hash_query_workspace_bytes": (_SZ, [ctypes.POINTER(HashDescC), _I64]),
    "ddf_hash_query": (ctypes.c_int, [ctypes.POINTER(HashDescC), _P, _P, _I64, _P, _P, _P, _SZ, _P]),
    "ddf_hash_query_static_max_rays": (_I64, []),
    "ddf_hash_query_static": (ctypes.c_int, [ctypes.POINTER(HashDescC), _P, _P, _I64, _P, _P, _P]),
    "ddf_hash_table_f16_bytes": (_SZ, [ctypes.POINTER(HashDescC)]),
    "ddf_hash_table_to_f16": (ctypes.c_int, [ctypes.POINTER(HashDescC), _P, _P, _P]),
    "ddf_hash_query_f16": (ctypes.c_int, [ctypes.POINTER(HashDescC), _P, _P, _P, _I64, _P, _P, _P, _SZ, _P]),
    "ddf_hash_train_workspace_bytes": (_SZ, [ctypes.POINTER(HashDescC), _I64]),
    "ddf_hash_train_step": (ctypes.c_int, [ctypes.POINTER(HashDescC), _P, _P, _P, _P, _P, _P, _I64,
                                           ctypes.POINTER(TrainHParamsC), _P, _P, _P, _P, _SZ, _P]),
    "ddf_primary_gbuffer": (ctypes.c_int, [ctypes.POINTER(CameraC), _P, ctypes.c_int32, _P, _P, _P]),
    "ddf_secondary_rays": (ctypes.c_int, [_P, _P, _I64, ctypes.POINTER(ctypes.c_float), ctypes.c_int32, _P,
                                          ctypes.c_float, _P, _P]),
    "ddf_shade": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                 ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "ddf_bounce": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, _P, _P]),
    "ddf_prim_area_cdf": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "ddf_sample_rays": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _I64, ctypes.c_int32, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_int32, _P, _P]),
    "sdf_train_step": (ctypes.c_int, [_D, _P, _P, _P, _P, _P, _P, _I64, ctypes.POINTER(TrainHParamsC),
                                      _P, _P, _P, _P, _SZ, _P]),
}


def lib():
    """The loaded libddf (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DDFError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_2606_00817_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        L = lib()
        raise DDFError(f"{L.ddf_status_string(rc).decode()}: {L.ddf_last_error().decode()}")


def desc_c(desc, precision=None) -> NetDescC:
    """ctypes descriptor from any object with n_in, n_freq, n_hidden, width, n_out."""
    p = precision if precision is not None else getattr(desc, "precision", FP32)
    if isinstance(p, str):
        p = PRECISIONS[p]
    return NetDescC(desc.n_in, desc.n_freq, desc.n_hidden, desc.width, desc.n_out, p)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise DDFError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t


def param_count(desc, precision=None) -> int:
    d = desc_c(desc, precision)
    return int(lib().ddf_param_count(ctypes.byref(d)))


def param_offsets(desc, layer, precision=None):
    """(w_off, b_off) of a layer in the master vector: 0..n_hidden-1 hidden, n_hidden the head."""
    d = desc_c(desc, precision)
    w, b = _SZ(), _SZ()
    _check(lib().ddf_param_offsets(ctypes.byref(d), int(layer), ctypes.byref(w), ctypes.byref(b)))
    return int(w.value), int(b.value)


def packed_bytes(desc, precision) -> int:
    d = desc_c(desc, precision)
    return int(lib().ddf_packed_bytes(ctypes.byref(d)))


def pack(desc, precision, master: torch.Tensor, act_scales=None, out=None) -> torch.Tensor:
    d = desc_c(desc, precision)
    _dev(master, torch.float32, "master")
    nbytes = int(lib().ddf_packed_bytes(ctypes.byref(d)))
    if nbytes == 0:
        _check(-1)
    packed = out if out is not None else torch.empty(nbytes, dtype=torch.uint8, device=master.device)
    sc = None
    if act_scales is not None:
        arr = np.ascontiguousarray(act_scales, dtype=np.float32)
        sc = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(lib().ddf_pack(ctypes.byref(d), _ptr(master), sc, _ptr(packed), _stream()))
    return packed


def query(desc, precision, packed: torch.Tensor, rays: torch.Tensor):
    """(t, xi) for float32 SoA rays [6, n]."""
    d = desc_c(desc, precision)
    _dev(rays, torch.float32, "rays")
    n = rays.shape[1]
    t = torch.empty(n, dtype=torch.float32, device=rays.device)
    xi = torch.empty(n, dtype=torch.float32, device=rays.device)
    _check(lib().ddf_query(ctypes.byref(d), _ptr(packed), _ptr(rays), n, _ptr(t), _ptr(xi), _stream()))
    return t, xi


def query_into(desc_ct: NetDescC, packed, rays, t, xi, stream=None):
    """Allocation-free query on prepared tensors (benchmark loop)."""
    _check(lib().ddf_query(ctypes.byref(desc_ct), _ptr(packed), _ptr(rays), rays.shape[1], _ptr(t), _ptr(xi),
                           stream if stream is not None else _stream()))


def query_split_workspace_bytes(desc, n) -> int:
    return int(lib().ddf_query_split_workspace_bytes(ctypes.byref(desc_c(desc, "bf16")), int(n)))


def query_split(desc, packed, rays, ws=None, t=None, xi=None):
    """The small-batch bf16 query (one launch per layer, neurons split over workgroups)."""
    _dev(rays, torch.float32, "rays")
    d = desc_c(desc, "bf16")
    n = rays.shape[1]
    t = torch.empty(n, dtype=torch.float32, device=rays.device) if t is None else t
    xi = torch.empty(n, dtype=torch.float32, device=rays.device) if xi is None else xi
    if ws is None:
        ws = torch.empty(max(256, query_split_workspace_bytes(desc, n)), dtype=torch.uint8, device=rays.device)
    _check(lib().ddf_query_split(ctypes.byref(d), _ptr(packed), _ptr(rays), n, _ptr(t), _ptr(xi), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream()))
    return t, xi


def query_hidden(desc, precision, packed, inputs):
    """The last hidden layer's float32 activations [n, width] for SoA inputs [n_in, n]."""
    d = desc_c(desc, precision)
    _dev(inputs, torch.float32, "inputs")
    n = inputs.shape[1]
    h = torch.empty((n, desc.width), dtype=torch.float32, device=inputs.device)
    _check(lib().ddf_query_hidden(ctypes.byref(d), _ptr(packed), _ptr(inputs), n, _ptr(h), _stream()))
    return h


def sdf_eval(desc, precision, packed, points):
    d = desc_c(desc, precision)
    _dev(points, torch.float32, "points")
    n = points.shape[1]
    s = torch.empty(n, dtype=torch.float32, device=points.device)
    _check(lib().sdf_eval(ctypes.byref(d), _ptr(packed), _ptr(points), n, _ptr(s), _stream()))
    return s


def sphere_trace(desc, precision, packed, rays, max_steps=128, hit_eps=1e-4, t_max=6.0, ws=None, pool=False):
    """(t, hit, steps) of sphere tracing the SDF net along float32 SoA rays [6, n]; pool=True:
    the persistent lane-refill trace (one launch), else the step-synchronous one."""
    d = desc_c(desc, precision)
    _dev(rays, torch.float32, "rays")
    n = rays.shape[1]
    dev = rays.device
    t = torch.empty(n, dtype=torch.float32, device=dev)
    hit = torch.empty(n, dtype=torch.uint8, device=dev)
    steps = torch.empty(n, dtype=torch.int32, device=dev)
    wsb = 256 if pool else int(lib().sdf_trace_workspace_bytes(n))
    if ws is None:
        ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)
    fn = lib().sdf_sphere_trace_pool if pool else lib().sdf_sphere_trace
    _check(fn(ctypes.byref(d), _ptr(packed), _ptr(rays), n, int(max_steps), float(hit_eps), float(t_max), _ptr(t),
              _ptr(hit), _ptr(steps), _ptr(ws), ws.numel(), _stream()))
    return t, hit, steps


def scene_prims(scene) -> np.ndarray:
    """Device layout of an analytic scene: float32 [P, 16] = center, 1/axes, R^T row-major, pad."""
    P = scene.n
    out = np.zeros((P, 16), dtype=np.float32)
    out[:, 0:3] = scene.centers
    out[:, 3:6] = 1.0 / np.asarray(scene.axes)
    out[:, 6:15] = np.transpose(np.asarray(scene.rot), (0, 2, 1)).reshape(P, 9)
    out[:, 15] = np.asarray(scene.axes).min(axis=1)
    return out


def cast_targets(prims: torch.Tensor, rays: torch.Tensor):
    """(t_gt, hit) by brute-force analytic ray casting on the GPU."""
    _dev(prims, torch.float32, "prims")
    _dev(rays, torch.float32, "rays")
    n = rays.shape[1]
    t = torch.empty(n, dtype=torch.float32, device=rays.device)
    hit = torch.empty(n, dtype=torch.uint8, device=rays.device)
    _check(lib().ddf_cast_targets(_ptr(prims), prims.shape[0], _ptr(rays), n, _ptr(t), _ptr(hit), _stream()))
    return t, hit


def shift_rays(rays: torch.Tensor, t_gt: torch.Tensor, hit: torch.Tensor, u: torch.Tensor, frac=0.3):
    """Self-consistency points replacing a fraction of a batch (see ddf_shift_rays)."""
    _dev(rays, torch.float32, "rays")
    _dev(t_gt, torch.float32, "t_gt")
    _dev(hit, torch.uint8, "hit")
    _dev(u, torch.float32, "u")
    n = rays.shape[1]
    ro = torch.empty_like(rays)
    to = torch.empty_like(t_gt)
    ho = torch.empty_like(hit)
    _check(lib().ddf_shift_rays(_ptr(rays), _ptr(t_gt), _ptr(hit), _ptr(u), float(frac), n, _ptr(ro), _ptr(to),
                                _ptr(ho), _stream()))
    return ro, to, ho


def lr_cosine(step, total=30000, lr0=3e-3, final_frac=0.05) -> float:
    return float(lib().ddf_lr_cosine(int(step), int(total), float(lr0), float(final_frac)))


def scene_sdf(prims: torch.Tensor, points: torch.Tensor):
    """Signed-distance bound of the analytic union at float32 SoA points [3, n]."""
    _dev(prims, torch.float32, "prims")
    _dev(points, torch.float32, "points")
    n = points.shape[1]
    s = torch.empty(n, dtype=torch.float32, device=points.device)
    _check(lib().ddf_scene_sdf(_ptr(prims), prims.shape[0], _ptr(points), n, _ptr(s), _stream()))
    return s


def sdf_train_step(desc, precision, master, m, v, packed, points, sdf_gt, hp: TrainHParamsC, ws,
                   loss_out=None, flag=None, grad_out=None):
    d = desc_c(desc, precision)
    dev = points.device
    loss_out = loss_out if loss_out is not None else torch.empty(4, dtype=torch.float32, device=dev)
    flag = flag if flag is not None else torch.empty(4, dtype=torch.int32, device=dev)
    _check(lib().sdf_train_step(ctypes.byref(d), _ptr(master), _ptr(m), _ptr(v), _ptr(packed), _ptr(points),
                                _ptr(sdf_gt), points.shape[1], ctypes.byref(hp), _ptr(loss_out), _ptr(flag),
                                _ptr(grad_out), _ptr(ws), ws.numel(), _stream()))
    return loss_out, flag


def train_workspace_bytes(desc, precision, batch, recompute_every=0) -> int:
    d = desc_c(desc, precision)
    return int(lib().ddf_train_workspace_bytes(ctypes.byref(d), int(batch), int(recompute_every)))


def forward_train(desc, precision, packed, rays, ws, recompute_every=0):
    d = desc_c(desc, precision)
    n = rays.shape[1]
    zt = torch.empty(n, dtype=torch.float32, device=rays.device)
    zx = torch.empty(n, dtype=torch.float32, device=rays.device)
    _check(lib().ddf_forward_train(ctypes.byref(d), _ptr(packed), _ptr(rays), n, _ptr(zt), _ptr(zx),
                                   int(recompute_every), _ptr(ws), ws.numel(), _stream()))
    return zt, zx


def train_kept_activation(desc, precision, n, ws, layer, recompute_every=0):
    """H_layer as the training forward kept it in ws, float32 [n, width]."""
    d = desc_c(desc, precision)
    h = torch.empty((n, desc.width), dtype=torch.float32, device=ws.device)
    _check(lib().ddf_train_kept_activation(ctypes.byref(d), int(n), int(recompute_every), _ptr(ws), ws.numel(),
                                           int(layer), _ptr(h), _stream()))
    return h


def backward(desc, precision, packed, rays, grad_zt, grad_zx, ws, recompute_every=0):
    d = desc_c(desc, precision)
    n = rays.shape[1]
    g = torch.empty(param_count(desc, precision), dtype=torch.float32, device=rays.device)
    _check(lib().ddf_backward(ctypes.byref(d), _ptr(packed), _ptr(rays), n, _ptr(grad_zt), _ptr(grad_zx),
                              _ptr(g), int(recompute_every), _ptr(ws), ws.numel(), _stream()))
    return g


def train_step(desc, precision, master, m, v, packed, rays, t_gt, hit, hp: TrainHParamsC, ws,
               loss_out=None, flag=None, grad_out=None):
    d = desc_c(desc, precision)
    dev = rays.device
    loss_out = loss_out if loss_out is not None else torch.empty(4, dtype=torch.float32, device=dev)
    flag = flag if flag is not None else torch.empty(4, dtype=torch.int32, device=dev)
    _check(lib().ddf_train_step(ctypes.byref(d), _ptr(master), _ptr(m), _ptr(v), _ptr(packed), _ptr(rays),
                                _ptr(t_gt), _ptr(hit), rays.shape[1], ctypes.byref(hp), _ptr(loss_out),
                                _ptr(flag), _ptr(grad_out), _ptr(ws), ws.numel(), _stream()))
    return loss_out, flag


def fp8_act_scales(desc, packed_fp32, rays) -> np.ndarray:
    """Power-of-two FP8 input scales of hidden layers 2..n from a calibration batch."""
    d = desc_c(desc, FP32)
    n = rays.shape[1]
    wsb = int(lib().ddf_fp8_calib_workspace_bytes(ctypes.byref(d), n))
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=rays.device)
    out = np.zeros(max(desc.n_hidden - 1, 1), dtype=np.float32)
    _check(lib().ddf_fp8_act_scales(ctypes.byref(d), _ptr(packed_fp32), _ptr(rays), n,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _ptr(ws), ws.numel(),
                                    _stream()))
    return out[:desc.n_hidden - 1]


class DDFFunction(torch.autograd.Function):
    """(z_t, z_xi) = f(params; rays): the library's training forward and backward as one
    node of a torch.autograd graph, so that a distillation loss written with torch ops
    back-propagates through the fused network.

    params           float32 master vector [param_count(desc)] on the rays' device
                     (packed into `precision` on every call).
    rays             float32 [n_in][n] SoA inputs (rays [6][n]; SDF points [3][n]).
    Returns the two logit vectors [n] (z_xi is zeros for a single-output network).  The
    gradient flows to `params` only (none to the rays)."""

    @staticmethod
    def forward(ctx, params, rays, desc, precision="bf16", recompute_every=0):
        _dev(params, torch.float32, "params")
        _dev(rays, torch.float32, "rays")
        packed = pack(desc, precision, params.detach())
        ws = torch.empty(max(train_workspace_bytes(desc, precision, rays.shape[1], recompute_every), 256),
                         dtype=torch.uint8, device=rays.device)
        zt, zx = forward_train(desc, precision, packed, rays, ws, recompute_every)
        if desc.n_out == 1:
            zx = torch.zeros_like(zt)
        ctx.save_for_backward(rays)
        ctx.state = (desc, precision, packed, ws, recompute_every)
        return zt, zx

    @staticmethod
    def backward(ctx, grad_zt, grad_zx):
        (rays,) = ctx.saved_tensors
        desc, precision, packed, ws, recompute_every = ctx.state
        gzt = grad_zt.contiguous().to(torch.float32)
        gzx = grad_zx.contiguous().to(torch.float32)
        g = backward(desc, precision, packed, rays, gzt, gzx, ws, recompute_every)
        return g, None, None, None, None


def ddf_apply(params, rays, desc, precision="bf16", recompute_every=0):
    """DDFFunction.apply with keyword defaults."""
    return DDFFunction.apply(params, rays, desc, precision, recompute_every)


# ---------------------------------------------------------------- hash-grid field


def hash_desc_c(desc) -> HashDescC:
    return HashDescC(desc.n_levels, desc.n_feat, desc.log2_table, desc.base_res, desc.growth, desc.dir_bands,
                     desc.width, desc.n_hidden, desc.n_out, desc.box_half)


def hash_param_count(desc) -> int:
    d = hash_desc_c(desc)
    n = int(lib().ddf_hash_param_count(ctypes.byref(d)))
    if n == 0:
        raise DDFError(f"unsupported hash-grid description: {lib().ddf_last_error().decode()}")
    return n


def hash_level(desc, level):
    """(resolution, entries, offset, hashed) of one level."""
    d = hash_desc_c(desc)
    res, hashed = ctypes.c_int32(), ctypes.c_int32()
    ent, off = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().ddf_hash_level(ctypes.byref(d), int(level), ctypes.byref(res), ctypes.byref(ent), ctypes.byref(off),
                                ctypes.byref(hashed)))
    return res.value, ent.value, off.value, bool(hashed.value)


def hash_query_workspace_bytes(desc, n) -> int:
    d = hash_desc_c(desc)
    return int(lib().ddf_hash_query_workspace_bytes(ctypes.byref(d), int(n)))


def hash_query(desc, params: torch.Tensor, rays: torch.Tensor, ws: torch.Tensor | None = None, fused: bool = False,
               t: torch.Tensor | None = None, xi: torch.Tensor | None = None):
    """(t, xi) of rays [6][n].  fused=True: the one-kernel path; else the two-pass path through
    `ws` (allocated here when not given).  t, xi: output tensors to fill (allocated when not
    given); with both outputs and ws given the call allocates nothing (graph capture)."""
    _dev(params, torch.float32, "params")
    _dev(rays, torch.float32, "rays")
    d = hash_desc_c(desc)
    n = rays.shape[1]
    t = torch.empty(n, dtype=torch.float32, device=rays.device) if t is None else t
    xi = torch.empty(n, dtype=torch.float32, device=rays.device) if xi is None else xi
    _dev(t, torch.float32, "t")
    _dev(xi, torch.float32, "xi")
    if not fused and ws is None and n > 0:
        ws = torch.empty(hash_query_workspace_bytes(desc, n), dtype=torch.uint8, device=rays.device)
    wp, wb = (None, 0) if fused or ws is None else (_ptr(ws), ws.numel() * ws.element_size())
    _check(lib().ddf_hash_query(ctypes.byref(d), _ptr(params), _ptr(rays), n, _ptr(t), _ptr(xi), wp, wb, _stream()))
    return t, xi


def hash_query_static_max_rays() -> int:
    return int(lib().ddf_hash_query_static_max_rays())


def hash_query_static(desc, params: torch.Tensor, rays: torch.Tensor, t: torch.Tensor, xi: torch.Tensor):
    """The two-pass query with the library's own static workspace (allocates nothing: the
    caller passes the outputs)."""
    _dev(params, torch.float32, "params")
    _dev(rays, torch.float32, "rays")
    _dev(t, torch.float32, "t")
    _dev(xi, torch.float32, "xi")
    d = hash_desc_c(desc)
    _check(lib().ddf_hash_query_static(ctypes.byref(d), _ptr(params), _ptr(rays), rays.shape[1], _ptr(t), _ptr(xi),
                                       _stream()))
    return t, xi


def hash_table_f16(desc, params: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """The float16 copy of the table (round to nearest even) for hash_query_f16."""
    _dev(params, torch.float32, "params")
    d = hash_desc_c(desc)
    nb = int(lib().ddf_hash_table_f16_bytes(ctypes.byref(d)))
    if nb == 0:
        raise DDFError(f"unsupported hash-grid description: {lib().ddf_last_error().decode()}")
    t16 = out if out is not None else torch.empty(nb // 2, dtype=torch.float16, device=params.device)
    _check(lib().ddf_hash_table_to_f16(ctypes.byref(d), _ptr(params), _ptr(t16), _stream()))
    return t16


def hash_query_f16(desc, params: torch.Tensor, table16: torch.Tensor, rays: torch.Tensor,
                   ws: torch.Tensor | None = None, t: torch.Tensor | None = None, xi: torch.Tensor | None = None):
    """(t, xi) with the lookups reading the float16 table copy (two-pass path)."""
    _dev(params, torch.float32, "params")
    _dev(table16, torch.float16, "table16")
    _dev(rays, torch.float32, "rays")
    d = hash_desc_c(desc)
    n = rays.shape[1]
    t = torch.empty(n, dtype=torch.float32, device=rays.device) if t is None else t
    xi = torch.empty(n, dtype=torch.float32, device=rays.device) if xi is None else xi
    if ws is None:
        ws = torch.empty(max(16, hash_query_workspace_bytes(desc, n)), dtype=torch.uint8, device=rays.device)
    _check(lib().ddf_hash_query_f16(ctypes.byref(d), _ptr(params), _ptr(table16), _ptr(rays), n, _ptr(t), _ptr(xi),
                                    _ptr(ws), ws.numel() * ws.element_size(), _stream()))
    return t, xi


def hash_train_workspace_bytes(desc, batch) -> int:
    d = hash_desc_c(desc)
    return int(lib().ddf_hash_train_workspace_bytes(ctypes.byref(d), int(batch)))


def hash_train_step(desc, params, m, v, rays, t_gt, hit, hp: TrainHParamsC, ws, loss_out=None, flag=None,
                    grad_out=None):
    d = hash_desc_c(desc)
    dev = rays.device
    loss_out = loss_out if loss_out is not None else torch.empty(4, dtype=torch.float32, device=dev)
    flag = flag if flag is not None else torch.empty(4, dtype=torch.int32, device=dev)
    _check(lib().ddf_hash_train_step(ctypes.byref(d), _ptr(params), _ptr(m), _ptr(v), _ptr(rays), _ptr(t_gt),
                                     _ptr(hit), rays.shape[1], ctypes.byref(hp), _ptr(loss_out), _ptr(flag),
                                     _ptr(grad_out), _ptr(ws), ws.numel(), _stream()))
    return loss_out, flag


# ---- shading consumers

def camera_c(view) -> CameraC:
    """ctypes camera from any object with eye, target, up, fov_y, width, height."""
    f3 = ctypes.c_float * 3
    return CameraC(f3(*view.eye), f3(*view.target), f3(*view.up), view.fov_y, view.width, view.height)


def primary_gbuffer(view, prims: torch.Tensor):
    """(gbuf [6][P] float32: hit point and outward normal, hit [P] uint8) of the view's pixels."""
    _dev(prims, torch.float32, "prims")
    P = view.width * view.height
    gbuf = torch.empty((6, P), dtype=torch.float32, device=prims.device)
    hit = torch.empty(P, dtype=torch.uint8, device=prims.device)
    cam = camera_c(view)
    _check(lib().ddf_primary_gbuffer(ctypes.byref(cam), _ptr(prims), prims.shape[0], _ptr(gbuf), _ptr(hit),
                                     _stream()))
    return gbuf, hit


def secondary_rays(gbuf: torch.Tensor, hit: torch.Tensor, light, n_ao: int, u: torch.Tensor | None,
                   offset: float, out: torch.Tensor | None = None):
    """Rays [6][P (1 + n_ao)]: per pixel the shadow ray, then n_ao AO rays (u [2][P n_ao])."""
    _dev(gbuf, torch.float32, "gbuf")
    _dev(hit, torch.uint8, "hit")
    P = hit.shape[0]
    if n_ao > 0:
        _dev(u, torch.float32, "u")
    rays = out if out is not None else torch.empty((6, P * (1 + n_ao)), dtype=torch.float32, device=gbuf.device)
    L = (ctypes.c_float * 3)(*light)
    _check(lib().ddf_secondary_rays(_ptr(gbuf), _ptr(hit), P, L, int(n_ao), _ptr(u) if n_ao > 0 else None,
                                    float(offset), _ptr(rays), _stream()))
    return rays


def shade(t: torch.Tensor, gbuf: torch.Tensor, hit: torch.Tensor, light, n_ao: int, offset: float,
          xi: torch.Tensor | None = None, ray_hit: torch.Tensor | None = None, ao_radius: float = float("inf")):
    """(shadow [P], ao [P]) from the answers t and xi (the field) or ray_hit (the exact cast)."""
    _dev(t, torch.float32, "t")
    P = hit.shape[0]
    shadow = torch.empty(P, dtype=torch.float32, device=t.device)
    ao = torch.empty(P, dtype=torch.float32, device=t.device)
    L = (ctypes.c_float * 3)(*light)
    _check(lib().ddf_shade(_ptr(t), _ptr(xi), _ptr(ray_hit), _ptr(gbuf), _ptr(hit), P, L, int(n_ao), float(offset),
                           float(ao_radius), _ptr(shadow), _ptr(ao), _stream()))
    return shadow, ao


def bounce(t: torch.Tensor, rays: torch.Tensor, hit: torch.Tensor, n_ao: int, radiance: torch.Tensor,
           box_half: float, sky, xi: torch.Tensor | None = None, ray_hit: torch.Tensor | None = None,
           out: torch.Tensor | None = None) -> torch.Tensor:
    """The one-bounce term [P] from the answers t and xi (the field) or ray_hit (the exact cast)
    to the secondary rays; radiance [res, res, res] the surface-radiance vertex grid."""
    _dev(t, torch.float32, "t")
    _dev(rays, torch.float32, "rays")
    _dev(radiance, torch.float32, "radiance")
    P = hit.shape[0]
    gi = torch.empty(P, dtype=torch.float32, device=t.device) if out is None else out
    _check(lib().ddf_bounce(_ptr(t), _ptr(xi), _ptr(ray_hit), _ptr(rays), _ptr(hit), P, int(n_ao), _ptr(radiance),
                            int(radiance.shape[0]), float(box_half), float(sky[0]), float(sky[1]), _ptr(gi),
                            _stream()))
    return gi


def prim_area_cdf(prims: torch.Tensor) -> torch.Tensor:
    """Cumulative surface-area weights of the primitives (once per scene)."""
    _dev(prims, torch.float32, "prims")
    cdf = torch.empty(max(1, prims.shape[0]), dtype=torch.float32, device=prims.device)
    _check(lib().ddf_prim_area_cdf(_ptr(prims), prims.shape[0], _ptr(cdf), _stream()))
    return cdf


def sample_rays(prims: torch.Tensor, u: torch.Tensor, mode: int = 2, box_half: float = 1.5, offset: float = 1e-3,
                tries: int | None = None, out: torch.Tensor | None = None, cdf: torch.Tensor | None = None):
    """Training rays [6][n] from uniforms u [3 tries + 2][n] (see ddf_sample_rays); mode 0
    surface, 1 free, 2 mixed (surface at even positions).  cdf: prim_area_cdf(prims), computed
    here when not given."""
    _dev(prims, torch.float32, "prims")
    _dev(u, torch.float32, "u")
    T = (u.shape[0] - 2) // 3 if tries is None else tries
    if u.shape[0] != 3 * T + 2:
        raise DDFError(f"u needs 3 tries + 2 = {3 * T + 2} rows, has {u.shape[0]}")
    n = u.shape[1]
    rays = out if out is not None else torch.empty((6, n), dtype=torch.float32, device=u.device)
    cdf = prim_area_cdf(prims) if cdf is None else cdf
    _dev(cdf, torch.float32, "cdf")
    _check(lib().ddf_sample_rays(_ptr(prims), prims.shape[0], _ptr(cdf), _ptr(u), n, int(mode), float(box_half),
                                 float(offset), int(T), _ptr(rays), _stream()))
    return rays

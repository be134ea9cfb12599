"""Benchmark of the DDF hot path on one MI355X; prints ONE JSON line.

Workload (the headline): the large mixed query batch -- 2^24 rays in one launch, 50 %
shadow rays (surface points of a 256-primitive sphere/ellipsoid scene, lifted along the
normal, aimed at the point light at (0, 3, 0)), 40 % ambient-occlusion rays (32
cosine-weighted hemisphere rays per surface point) and 10 % one-bounce rays (uniform over
the normal's hemisphere), in a fixed seeded interleave -- through the 16 x 1024 DDF (L = 10
encoding, 126 features), random He-init weights (seed 0).  A timed step is one query of the
whole batch (ray ingest, encoding, the fused layer chain and both heads) in the headline
precision (bf16); the JSON line's `value` is its throughput.  Further legs run in the same
invocation, each query leg with its own roofline and precision statistics:
  * the same 2^24 rays in fp8 (e4m3, per-layer scales) and fp32;
  * the ambient-occlusion batch: 512 x 512 surface points x 32 cosine rays (8,388,608 rays)
    through the 12 x 1024 DDF in bf16, fp8 and fp32;
  * 2^20 shadow rays through the 12 x 1024 DDF in fp32, bf16 and fp8, and sphere tracing of a
    signed-distance MLP of the same size along the same rays (the paper's baseline) at three
    hit thresholds and at 1K, 10K and 100K rays, with the float64 oracle's trace of the
    analytic distance bound on every 128th ray as the yardstick;
  * the bf16 and fp8 queries at 1K, 10K and 100K rays and the tiny 4 x 128 net;
  * distillation training steps (65,536 rays through the 12 x 1024 net; 262,144 rays through
    the 16 x 1024 net with activations recomputed every 4 layers; bf16 and fp32 each);
  * the paper's own 52 MB hash-grid field, queried at 1K to 2^20 rays and trained on
    16,384-ray batches, and that field distilled by the paper's recipe on one object above a
    ground slab, answering a 512 x 512 frame's shadow and AO rays (maps against exact casting).
Every reduced precision's max / mean |dt| and visibility flip rate is taken against the fp32
query over all rays, and against the float64 oracle on every 16th ray of the 2^24-ray and
8.4M-ray batches (computed on the host while the GPU legs run).  The float64 oracle is also
timed alone on the host cores over a bounded sample of the headline rays (cpu_baseline).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision bf16]
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}   # MI355X dense matrix peaks
N_HEAD = 1 << 24           # rays of the headline batch
N_SHADOW = 1 << 20         # rays of the 12 x 1024 shadow batch
AO_POINTS, AO_DIRS = 512 * 512, 32
SUBSET = 16                # the float64 oracle answers every 16th ray of the large batches

# HBM traffic of one launch of the headline query kernel, from two rocprofv3 counter passes over
# this workload (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same
# counter reads for a 1 GiB device copy in the same run (FETCH_SIZE reads 524,306 KiB for
# 1,048,576 KiB fetched: x2; WRITE_SIZE reads 1,048,576 KiB: x1).  The figures hold for the
# kernel sources they were taken on (sha256 over KERNEL_SOURCES); after any change to those
# files the bench reports null until the counters are taken again.
COUNTER_SCALE = {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
TRAFFIC_KIB = {
    "bf16": {"FETCH_SIZE": 128417968, "WRITE_SIZE": 131072,
             "sha256": "1f52d71002e4afa37bce676160a23a62610d0e7036438a71fafdcb70863603d9"},
}
KERNEL_SOURCES = {
    "fp32": ["ddf_fwd.hip", "ddf_chain.h", "ddf_fwd.h", "ddf_internal.h"],
    "bf16": ["ddf_fwd.hip", "ddf_chain.h", "ddf_fwd.h", "ddf_internal.h"],
    "fp8": ["ddf_fwd8.hip", "ddf_fwd.h", "ddf_internal.h"],
}
KERNEL_NAME = {"fp32": "fwd_kernel (fp32)", "bf16": "fwd_kernel (bf16)", "fp8": "fwd8_kernel"}


def kernel_source_hash(prec):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[prec]:
        with open(os.path.join(HERE, "paper_2606_00817_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(prec):
    """Scaled HBM bytes per launch, or None when unmeasured or the kernel changed since."""
    rec = TRAFFIC_KIB.get(prec)
    if rec is None or rec["sha256"] != kernel_source_hash(prec):
        return None
    return int(sum(rec[c] * COUNTER_SCALE[c] for c in COUNTER_SCALE) * 1024)


def flop_per_ray(desc):
    f = 2 * desc.width * desc.n_feat + 2 * (desc.n_hidden - 1) * desc.width * desc.width
    return f + 2 * desc.n_out * desc.width


class KernelTimer:
    """HIP-event timing on the stream the library launches on (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps):
        torch = self.torch
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


def cpu_oracle_baseline(desc, params, rays_np, budget_s=12.0):
    """The float64 oracle timed alone on the host cores over a bounded sample of the headline
    rays (rank 0, N = 1): about budget_s seconds of work."""
    from oracle import ddf_oracle as O
    probe = 512
    t0 = time.perf_counter()
    O.ddf_query(desc, params, rays_np[:, :probe])
    dt = time.perf_counter() - t0
    n = int(min(rays_np.shape[1], max(probe, probe * budget_s / max(dt, 1e-6))))
    n = max(probe, n // probe * probe)
    t0 = time.perf_counter()
    O.ddf_query(desc, params, rays_np[:, :n])
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "rays/s", "cores": int(blas_threads()), "kind": "oracle",
            "sample": f"first {n} of the {rays_np.shape[1]} headline rays (mixed shadow/AO/GI, "
                      f"{desc.width}x{desc.n_hidden} net), float64 numpy forward, {dt:.1f} s"}


class OracleSubsets(threading.Thread):
    """The float64 oracle on every SUBSET-th ray of the large batches, on the host while the GPU
    legs run (numpy's BLAS threads do the work; the GIL is released inside them)."""

    def __init__(self):
        super().__init__(daemon=True)
        self.jobs, self.results, self.error = [], {}, None

    def add(self, name, desc, params, rays_np):
        self.jobs.append((name, desc, params, np.ascontiguousarray(rays_np[:, ::SUBSET])))

    def run(self):
        try:
            from oracle import ddf_oracle as O
            for name, desc, params, r in self.jobs:
                t0 = time.perf_counter()
                t64, x64, _, z64 = O.ddf_query(desc, params, r)
                self.results[name] = (t64, x64, z64, r.shape[1], time.perf_counter() - t0)
        except Exception as e:   # reported in the JSON line, never hidden
            self.error = repr(e)


def dt_stats(t_ref, x_ref, t, xi):
    """max/mean |dt| and visibility flip rate (xi > 0.5) of answers against reference answers,
    and the share of reference answers within |z_xi| < 1e-3 of the decision (|xi - 0.5| <
    2.5e-4), where a flip costs nothing."""
    d = np.abs(np.asarray(t, dtype=np.float64) - np.asarray(t_ref, dtype=np.float64))
    xr = np.asarray(x_ref, dtype=np.float64)
    return {"max_abs_dt": float(d.max()), "mean_abs_dt": float(d.mean()),
            "flip_rate": float(((np.asarray(xi) > 0.5) != (xr > 0.5)).mean()),
            "near_threshold_fraction": float((np.abs(xr - 0.5) < 2.5e-4).mean()), "rays": int(d.size)}


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class QueryLeg:
    """One query batch on one net: every precision timed on the same rays, with its roofline."""

    def __init__(self, torch, ddf, dev, timer, desc, params_np, rays_np, calib):
        self.torch, self.ddf, self.dev, self.timer = torch, ddf, dev, timer
        self.desc, self.n = desc, rays_np.shape[1]
        self.rays = torch.from_numpy(rays_np).to(dev)
        self.master = torch.from_numpy(params_np).to(dev)
        self.packed32 = ddf.pack(desc, "fp32", self.master)
        self.scales = ddf.fp8_act_scales(desc, self.packed32, calib)
        self.fpr = flop_per_ray(desc)
        self.t = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.xi = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.answers = {}

    def packed(self, prec):
        if prec == "fp32":
            return self.packed32
        return self.ddf.pack(self.desc, prec, self.master, act_scales=self.scales if prec == "fp8" else None)

    def run(self, prec, steps, warmup):
        ddf, torch = self.ddf, self.torch
        pk = self.packed(prec)
        dc = ddf.desc_c(self.desc, prec)
        for _ in range(warmup):
            ddf.query_into(dc, pk, self.rays, self.t, self.xi)
        torch.cuda.synchronize()
        ms = self.timer.time(lambda: ddf.query_into(dc, pk, self.rays, self.t, self.xi), steps)
        torch.cuda.synchronize()
        self.answers[prec] = (self.t.cpu().numpy(), self.xi.cpu().numpy())
        tf = self.fpr * self.n / (ms * 1e-3) / 1e12
        return {"ms": ms, "rays_per_s": self.n / (ms * 1e-3), "launches_timed": steps,
                "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                             "frac": tf / PEAK_TFLOPS[prec], "kernel": KERNEL_NAME[prec],
                             "flop_per_launch": self.fpr * self.n}}

    def vs_fp32(self, prec):
        t32, x32 = self.answers["fp32"]
        return dt_stats(t32, x32, *self.answers[prec])

    def vs_float64(self, prec, t64, x64):
        t, xi = self.answers[prec]
        return dt_stats(t64, x64, t[::SUBSET], xi[::SUBSET])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--legs", default="precisions,ao,shadow,sparse,train,train_large,trace,distill,hash,shade,cpu",
                    help="comma list of extra legs: precisions (fp8/fp32 of the headline rays), ao, shadow, "
                         "sparse, train, train_large, trace (needs shadow), distill (needs ao), hash, shade, cpu (the "
                         "float64 oracle on the host: timed sample and the float64 answers of every statistic "
                         "against float64), copy")
    ap.add_argument("--distill-steps", type=int, default=3000,
                    help="training steps of the 12 x 1024 field distilled for the distill leg")
    ap.add_argument("--shade-steps", type=int, default=30000,
                    help="recipe steps of the hash-grid field trained for the shade leg")
    ap.add_argument("--sdf-fit-steps", type=int, default=3000,
                    help="fitting steps of the SDF MLP the trace leg sphere-traces")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout "
              f"is described but not built", file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)

    import torch
    from paper_2606_00817_amd import ddf
    from paper_2606_00817_amd import inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    timer = KernelTimer(torch)
    scene = I.scene_mixed(256, 2)
    calib = torch.from_numpy(I.free_rays(scene, 4096, 21)).to(dev)   # FP8 calibration batch
    t_in = time.perf_counter()
    head_np = I.mixed_rays(scene, N_HEAD, 15)
    head_params = I.he_init(I.NET_LARGE, 0)
    oracle = OracleSubsets()      # part of the cpu leg: the oracle runs on the host only there
    if "cpu" in legs:
        oracle.add("mixed", I.NET_LARGE, head_params, head_np)
    ao_np = I.ao_rays(scene, AO_POINTS, AO_DIRS, 13) if "ao" in legs else None
    full_params = I.he_init(I.NET_FULL, 0)
    if ao_np is not None and "cpu" in legs:
        oracle.add("ao", I.NET_FULL, full_params, ao_np)
    if oracle.jobs:
        oracle.start()
    progress(f"inputs drawn ({time.perf_counter() - t_in:.1f} s)")

    if "copy" in legs:
        # a plain copy kernel of known size (1 GiB read + 1 GiB written): the reference that
        # scales the memory counters of a profiled run
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- the timed region: K steps of the headline-precision query of the 2^24 mixed rays
    head = QueryLeg(torch, ddf, dev, timer, I.NET_LARGE, head_params, head_np, calib)
    prec = args.precision
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    hl = head.run(prec, args.steps, args.warmup)
    wall = time.perf_counter() - wall0
    ms = hl["ms"]
    roof = dict(hl["roofline"])
    roof["traffic"] = traffic_bytes(prec)
    roof["kernel"] = f"{KERNEL_NAME[prec]}, one launch per step"
    out = {
        "metric": "DDF rays/sec + MFMA util, BF16/FP8 vs FP32 at stated |dt|; train rays/sec",
        "value": N_HEAD / (ms * 1e-3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic (seeded analytic scene, He-init weights)",
        "config": {"workload": "2^24 mixed rays in one launch (50% shadow, 40% AO x32 per point, 10% one-bounce "
                               "GI), 256-primitive scene, 16x1024 DDF (L=10, 126 features)",
                   "rays": N_HEAD, "net": "126-1024x16-2", "precision": prec},
        "roofline": roof,
    }
    progress(f"headline done ({prec} {ms:.2f} ms/step)")
    res = {}
    if "precisions" in legs:
        for p in ("fp32", "bf16", "fp8"):
            if p != prec:
                res[p] = head.run(p, 3 if p == "fp32" else max(3, args.steps // 2), 1)
    if "fp32" in head.answers:
        for p in head.answers:
            if p == "fp32":
                continue
            st = head.vs_fp32(p)
            if p == prec:
                out["precision_stats"] = {"vs_fp32_all_rays": {p: st}}
            else:
                res[p]["vs_fp32_all_rays"] = st
    out["mixed_2p24_16x1024"] = res
    progress("headline precisions done")

    ao = None
    if ao_np is not None:
        ao = QueryLeg(torch, ddf, dev, timer, I.NET_FULL, full_params, ao_np, calib)
        r = {p: ao.run(p, 3 if p == "fp32" else 10, 1) for p in ("bf16", "fp8", "fp32")}
        for p in ("bf16", "fp8"):
            r[p]["vs_fp32_all_rays"] = ao.vs_fp32(p)
        out["ao_8p4M_12x1024"] = r
        progress("ao leg done")

    shadow = None
    if "shadow" in legs:
        shadow_np = I.shadow_rays(scene, N_SHADOW, 12)
        shadow = QueryLeg(torch, ddf, dev, timer, I.NET_FULL, full_params, shadow_np, calib)
        r = {p: shadow.run(p, 5 if p == "fp32" else 20, 2) for p in ("fp32", "bf16", "fp8")}
        for p in ("bf16", "fp8"):
            r[p]["vs_fp32_all_rays"] = shadow.vs_fp32(p)
        out["shadow_2p20_12x1024"] = r
        progress("shadow leg done")

    if "sparse" in legs and shadow is not None:
        out["sparse_queries"] = sparse_leg(torch, ddf, I, dev, timer, shadow)
        progress("sparse leg done")
    if "train" in legs:
        out["train"] = train_leg(torch, ddf, I, dev, timer, args.steps)
        progress("train leg done")
    if "train_large" in legs:
        out["train_large"] = train_leg(torch, ddf, I, dev, timer, 4, batch=1 << 18, desc=I.NET_LARGE,
                                       recompute_every=4, seed=1300, lr=3e-4)
        progress("train_large leg done")
    trace_host = None
    if "trace" in legs and shadow is not None:
        out["sphere_trace"], trace_host = trace_leg(torch, ddf, I, dev, shadow, timer, out["shadow_2p20_12x1024"],
                                                    scene, args.sdf_fit_steps)
        progress("trace leg done")
    distilled = None
    if "distill" in legs and ao is not None:
        distilled = distill_leg(torch, ddf, I, dev, scene, ao, calib, args.distill_steps)
        out["distilled_12x1024"] = distilled["report"]
        progress("distill leg done")
    if "hash" in legs:
        rays_h = shadow.rays if shadow is not None else torch.from_numpy(I.shadow_rays(scene, N_SHADOW, 12)).to(dev)
        out["hash_grid"] = hash_leg(torch, ddf, I, dev, rays_h, timer, args.steps)
        progress("hash leg done")
    if "shade" in legs:
        out["shading"] = shade_leg(torch, ddf, I, dev, timer, args.shade_steps)
        progress("shade leg done")

    if oracle.jobs:
        oracle.join()
        if oracle.error:
            out["oracle_subsets_error"] = oracle.error
        for name, leg, key in (("mixed", head, "mixed_2p24_16x1024"), ("ao", ao, "ao_8p4M_12x1024")):
            if name not in oracle.results or leg is None:
                continue
            t64, x64, z64, n64, secs = oracle.results[name]
            sub = {"rays": n64, "every": SUBSET, "oracle_s": secs,
                   "float64_abs_z_xi_quantiles": {q: float(np.quantile(np.abs(z64), q)) for q in (0.01, 0.05, 0.5)}}
            for p in leg.answers:
                sub[p] = leg.vs_float64(p, t64, x64)
                if p != "fp32":
                    xq = np.clip(leg.answers[p][1][::SUBSET].astype(np.float64), 1e-7, 1 - 1e-7)
                    dz = np.abs(np.log(xq / (1 - xq)) - z64)[np.abs(z64) < 15]
                    sub[p]["abs_z_xi_err_quantiles"] = {q: float(np.quantile(dz, q)) for q in (0.5, 0.9, 0.99)}
            out.setdefault(key, {})["vs_float64_subset"] = sub
            if name == "mixed":
                out.setdefault("precision_stats", {})["vs_float64_subset"] = sub
        progress("oracle subsets done")
    if "cpu" in legs and trace_host is not None:
        trace_oracle_stats(scene, trace_host, out["sphere_trace"])
        progress("trace float64 statistics done")
    if "cpu" in legs and distilled is not None:
        distilled_oracle_stats(I, distilled, ao_np, out["distilled_12x1024"])
        progress("distilled float64 statistics done")
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_oracle_baseline(I.NET_LARGE, head_params, head_np)
    out["wall_s_timed"] = wall
    print(json.dumps(out))


def distill_leg(torch, ddf, I, dev, scene, ao, calib, steps):
    """A trained field for the precision statistics (Sec. III-B, III-D): the 12 x 1024 DDF
    distilled on the 256-primitive scene by bf16 training steps of 65,536 fresh rays (the GPU
    sampler: surface rays in all directions and free rays, exact cast targets, 30 % replaced
    by self-consistency points), Adam with the learning rate decayed by cosine from 1e-3 to
    5 %.  Then the AO batch (8,388,608 rays) through it in fp32, bf16 and fp8 (scales
    calibrated on this net): quality against exact casting (hit accuracy, |t - t_gt| where
    both hit) and each reduced precision against the fp32 query over all rays."""
    import math
    desc = I.NET_FULL
    B, T = 65536, 4
    prims = torch.from_numpy(ddf.scene_prims(scene)).to(dev)
    cdf = ddf.prim_area_cdf(prims)
    master = torch.from_numpy(I.he_init(desc, 0)).to(dev)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    packed = ddf.pack(desc, "bf16", master)
    ws = torch.empty(ddf.train_workspace_bytes(desc, "bf16", B), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(61)
    U = torch.empty((3 * T + 2, B), device=dev)
    U3 = torch.empty((3, B), device=dev)
    loss = torch.empty(4, dtype=torch.float32, device=dev)
    flag = torch.empty(4, dtype=torch.int32, device=dev)
    lr0 = 1e-3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    skipped = 0
    for st in range(1, steps + 1):
        U.uniform_(generator=gen)
        U3.uniform_(generator=gen)
        rays = ddf.sample_rays(prims, U, mode=2, offset=I.NORMAL_OFFSET, cdf=cdf)
        t, h = ddf.cast_targets(prims, rays)
        t = torch.where(h > 0, t, torch.zeros_like(t))
        rs, ts, hs = ddf.shift_rays(rays, t, h, U3, 0.3)
        lr = ddf.lr_cosine(st - 1, total=steps, lr0=lr0)
        hp = ddf.TrainHParamsC(lr, 0.9, 0.999, 1e-8, 0.3, 3.0, st)
        ddf.train_step(desc, "bf16", master, m, v, packed, rs, ts, hs, hp, ws, loss_out=loss, flag=flag)
        if st % 1000 == 0 or st == steps:
            skipped += int(flag[0].item())
            progress(f"distill leg: {st} of {steps} training steps, loss {loss[0].item():.4f}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del ws
    tg, hg = ddf.cast_targets(prims, ao.rays)
    hit_gt = (hg > 0).cpu().numpy()
    t_gt = tg.cpu().numpy()
    pk32 = ddf.pack(desc, "fp32", master)
    scales = ddf.fp8_act_scales(desc, pk32, calib)
    answers = {}
    report = {"net": "126-1024x12-2", "scene": "256 spheres/ellipsoids", "train_steps": steps, "train_batch": B,
              "train_s": train_s, "final_loss": float(loss[0].item()), "lr": "cosine 1e-3 -> 5e-5",
              "skipped_steps_seen": skipped,
              "eval_rays": "the AO batch (512 x 512 points x 32 cosine rays)", "fp8_act_scales": [float(x) for x in scales]}
    for prec in ("fp32", "bf16", "fp8"):
        pk = pk32 if prec == "fp32" else ddf.pack(desc, prec, master, act_scales=scales if prec == "fp8" else None)
        tq, xq = ddf.query(desc, prec, pk, ao.rays)
        tq, xq = tq.cpu().numpy(), xq.cpu().numpy()
        answers[prec] = (tq, xq)
        hit = xq > 0.5
        both = hit & hit_gt
        d = np.abs(tq[both].astype(np.float64) - t_gt[both])
        report[prec] = {"hit_accuracy_vs_exact_cast": float((hit == hit_gt).mean()),
                        "mean_abs_t_err_on_hits": float(d.mean()), "median_abs_t_err_on_hits": float(np.median(d))}
        if prec != "fp32":
            report[prec]["vs_fp32_all_rays"] = dt_stats(*answers["fp32"], tq, xq)
    return {"report": report, "master": master.cpu().numpy(), "answers": answers, "scales": scales}


def distilled_oracle_stats(I, distilled, ao_np, report, every=128, attr_every=512):
    """cpu leg, the trained field: each precision against the float64 oracle on every 128th ray
    of the AO batch, and where the fp8 error comes from: the oracle's fp8 emulation (kernel
    roundings, exact sums) with all layers quantised and with one layer at a time (the others
    exact) on every 512th ray; the kernel's z_xi error distribution against float64."""
    from oracle import ddf_oracle as O
    desc = I.NET_FULL
    params = distilled["master"].astype(np.float64)
    r = np.ascontiguousarray(ao_np[:, ::every])
    t64, x64, _, z64 = O.ddf_query(desc, params, r)
    sub = {"rays": int(r.shape[1]), "every": every}
    for p, (tq, xq) in distilled["answers"].items():
        sub[p] = dt_stats(t64, x64, tq[::every], xq[::every])
    xf = np.clip(distilled["answers"]["fp8"][1][::every].astype(np.float64), 1e-7, 1 - 1e-7)
    dz = np.abs(np.log(xf / (1 - xf)) - z64)
    sub["fp8"]["abs_z_xi_err_quantiles"] = {q: float(np.quantile(dz[np.abs(z64) < 15], q)) for q in (0.5, 0.9, 0.99)}
    sub["float64_abs_z_xi_quantiles"] = {q: float(np.quantile(np.abs(z64), q)) for q in (0.01, 0.05, 0.5)}
    report["vs_float64_subset"] = sub
    # fp8 attribution on the oracle's emulation
    ra = np.ascontiguousarray(ao_np[:, ::attr_every])
    g = O.encode(O.rays_to_inputs(ra), desc.n_freq)
    L = O.layers(desc, params)
    scales = [float(s) for s in distilled["scales"]]
    sw = O.weight_scales_fp8(desc, params)
    _, z_ref = O.mlp_forward(desc, params, g)
    t_ref = O.softplus(z_ref[:, 0])

    def forward(quant):
        W1, b1 = L[0]
        if quant:
            hi, lo = O.split_bf16(g)
            h = np.maximum((hi + lo) @ O.round_bf16(W1).T + b1, 0.0)
        else:
            h = np.maximum(g @ W1.T + b1, 0.0)
        for li, (W, b) in enumerate(L[1:-1]):
            h = O.hidden_layer_emulated(W, b, h, "fp8" if li + 2 in quant else "fp32", scales[li], sw[li])
        Wh, bh = L[-1]
        z = h @ Wh.T + bh
        return {"mean_abs_dt": float(np.abs(O.softplus(z[:, 0]) - t_ref).mean()),
                "flip_rate": float(((z[:, 1] > 0) != (z_ref[:, 1] > 0)).mean())}
    attr = {"rays": int(ra.shape[1]), "all_layers": forward(set(range(2, desc.n_hidden + 1)))}
    for l in range(2, desc.n_hidden + 1):
        attr[f"layer_{l}_only"] = forward({l})
    report["fp8_emulated_attribution"] = attr


def sparse_leg(torch, ddf, I, dev, timer, shadow):
    """The sparse-query regime (the paper's 1K-100K ray counts): per-call time of the dense
    12 x 1024 query in each reduced precision on the first n shadow rays, and of the bf16
    small-batch path; and the tiny configuration (4,096 free rays, 4 x 128 net, fp32)."""
    sp = {}
    desc = shadow.desc
    for p in ("bf16", "fp8"):
        pk = shadow.packed(p)
        dc = ddf.desc_c(desc, p)
        row = {}
        for n in (1000, 10000, 100000):
            r = shadow.rays[:, :n].contiguous()
            tq = torch.empty(n, dtype=torch.float32, device=dev)
            xq = torch.empty(n, dtype=torch.float32, device=dev)
            for _ in range(3):
                ddf.query_into(dc, pk, r, tq, xq)
            torch.cuda.synchronize()
            msn = timer.time(lambda: ddf.query_into(dc, pk, r, tq, xq), 20)
            row[str(n)] = {"ms": msn, "rays_per_s": n / (msn * 1e-3), "us_per_ray": msn * 1e3 / n}
            if p == "bf16":
                wsq = torch.empty(ddf.query_split_workspace_bytes(desc, n), dtype=torch.uint8, device=dev)
                for _ in range(3):
                    ddf.query_split(desc, pk, r, ws=wsq, t=tq, xi=xq)
                torch.cuda.synchronize()
                msn = timer.time(lambda: ddf.query_split(desc, pk, r, ws=wsq, t=tq, xi=xq), 20)
                row[str(n)]["split"] = {"ms": msn, "rays_per_s": n / (msn * 1e-3), "us_per_ray": msn * 1e3 / n}
        sp[p] = row
    dt_ = I.NET_TINY
    pk = ddf.pack(dt_, "fp32", torch.from_numpy(I.he_init(dt_, 0)).to(dev))
    rt_ = torch.from_numpy(I.free_rays(I.scene_spheres(16, 1), 4096, 11)).to(dev)
    tq = torch.empty(4096, dtype=torch.float32, device=dev)
    xq = torch.empty(4096, dtype=torch.float32, device=dev)
    dct = ddf.desc_c(dt_, "fp32")
    for _ in range(3):
        ddf.query_into(dct, pk, rt_, tq, xq)
    torch.cuda.synchronize()
    mst = timer.time(lambda: ddf.query_into(dct, pk, rt_, tq, xq), 50)
    sp["tiny_4x128_fp32_4096_rays"] = {"us_per_launch": mst * 1e3, "rays_per_s": 4096 / (mst * 1e-3)}
    return sp


def train_flop_per_ray(desc):
    """Forward + backward (delta chain without layer 1's input gradient) + weight gradients."""
    fwd = flop_per_ray(desc)
    dx = 2 * (desc.n_hidden - 1) * desc.width * desc.width + 2 * desc.n_out * desc.width
    dw = 2 * desc.width * desc.n_feat + 2 * (desc.n_hidden - 1) * desc.width * desc.width + 2 * desc.n_out * desc.width
    return fwd + dx + dw


def train_leg(torch, ddf, I, dev, timer, steps, batch=65536, desc=None, recompute_every=0, seed=1000, lr=1e-3):
    """One distillation step per timed step: `batch` rays (half surface-anchored, half free)
    against 1,024 random ellipsoids, targets by exact ray casting on the GPU; bf16 (then
    fp32) forward and backward with the fp32 master, then Adam and the repack.  Defaults:
    65,536 rays, 12 x 1024; the large configuration is 262,144 rays, 16 x 1024, activations
    recomputed every 4 layers."""
    desc = desc or I.NET_FULL
    scene = I.scene_ellipsoids(1024, 3)
    prims = torch.from_numpy(ddf.scene_prims(scene)).to(dev)
    rays = torch.from_numpy(I.train_rays(scene, batch, seed)).to(dev)
    t_gt, hit = ddf.cast_targets(prims, rays)
    t_gt = torch.where(hit > 0, t_gt, torch.zeros_like(t_gt))
    res = {"batch": batch, "net": f"{desc.n_feat}-{desc.width}x{desc.n_hidden}-{desc.n_out}",
           "recompute_every": recompute_every, "targets": "exact ray casting, 1024 ellipsoids",
           "hit_fraction": float(hit.float().mean().item())}
    fpr = train_flop_per_ray(desc)
    for prec in ("bf16", "fp32"):
        master = torch.from_numpy(I.he_init(desc, 0)).to(dev)
        m = torch.zeros_like(master)
        v = torch.zeros_like(master)
        packed = ddf.pack(desc, prec, master)
        ws = torch.empty(ddf.train_workspace_bytes(desc, prec, batch, recompute_every), dtype=torch.uint8,
                         device=dev)
        loss = torch.empty(4, dtype=torch.float32, device=dev)
        flag = torch.empty(4, dtype=torch.int32, device=dev)
        step = [0]

        def one():
            step[0] += 1
            hp = ddf.TrainHParamsC(lr, 0.9, 0.999, 1e-8, 0.3, 3.0, step[0], recompute_every)
            ddf.train_step(desc, prec, master, m, v, packed, rays, t_gt, hit, hp, ws, loss_out=loss, flag=flag)
        one()
        torch.cuda.synchronize()
        l0 = float(loss[0].item())
        k = max(2, steps // 2) if prec == "bf16" else 2
        ms = timer.time(one, k)
        res[prec] = {"ms_per_step": ms, "train_rays_per_s": batch / (ms * 1e-3),
                     "tflops": fpr * batch / (ms * 1e-3) / 1e12, "loss_first": l0,
                     "loss_last": float(loss[0].item()), "steps": step[0],
                     "skipped": int(flag[0].item()), "workspace_bytes": ws.numel()}
        del ws
    res["flop_per_ray"] = fpr
    return res


def hash_leg(torch, ddf, I, dev, rays, timer, steps):
    """The paper's own field, the 52 MB hash grid (16 levels x 2^19 x 2 features, 4 direction
    bands, 2 x 64 MLP), random table N(0, 0.3): queries of the same shadow rays at 1K, 10K,
    100K and 2^20 rays (the ray counts of the paper's latency table), and distillation steps of
    16,384 rays (the paper's batch) against exact ray-cast targets of 1,024 ellipsoids.
    Both query paths are timed: two-pass (lookups with level groups pinned to XCDs, then the
    MLP) and fused (one kernel); and the two-pass path reading a float16 copy of the table
    (the paper's reduced-precision inference setting).  Algorithmic bytes per queried ray: the ray (24 B), both
    outputs (8 B) and 16 levels x 8 corners x 2 float32 features gathered (1,024 B)."""
    desc = I.HASH_PAPER
    n_par = ddf.hash_param_count(desc)
    n_entries = sum(ddf.hash_level(desc, l)[1] for l in range(desc.n_levels))
    params = torch.from_numpy(I.hash_params(desc, n_entries, 7, table_std=0.3)).to(dev)
    bpr = 24 + 8 + desc.n_levels * 8 * desc.n_feat * 4
    res = {"field": "hash grid 16 x 2^19 x 2, 4 bands, 2x64 MLP", "params": n_par,
           "bytes": 4 * n_par, "algorithmic_bytes_per_ray": bpr, "query": {}}
    ws = torch.empty(ddf.hash_query_workspace_bytes(desc, rays.shape[1]), dtype=torch.uint8, device=dev)
    table16 = ddf.hash_table_f16(desc, params)
    for n in (1000, 10000, 100000, rays.shape[1]):
        r = rays[:, :n].contiguous()
        row = {}
        for path in ("two_pass", "fused"):
            kw = {"fused": True} if path == "fused" else {"ws": ws}
            for _ in range(3):
                ddf.hash_query(desc, params, r, **kw)
            torch.cuda.synchronize()
            ms = timer.time(lambda: ddf.hash_query(desc, params, r, **kw), max(10, steps))
            row[path] = {"ms": ms, "rays_per_s": n / (ms * 1e-3), "us_per_ray": ms * 1e3 / n,
                         "gathered_GBps": bpr * n / (ms * 1e-3) / 1e9}
        # the reduced-precision lookups (float16 table copy)
        tq = torch.empty(n, dtype=torch.float32, device=dev)
        xq = torch.empty(n, dtype=torch.float32, device=dev)
        for _ in range(3):
            ddf.hash_query_f16(desc, params, table16, r, ws=ws, t=tq, xi=xq)
        torch.cuda.synchronize()
        ms = timer.time(lambda: ddf.hash_query_f16(desc, params, table16, r, ws=ws, t=tq, xi=xq), max(10, steps))
        row["two_pass_f16_table"] = {"ms": ms, "rays_per_s": n / (ms * 1e-3), "us_per_ray": ms * 1e3 / n}
        if n <= 100000:
            # the sparse regime: the two-pass query captured once, replayed (no host launch cost)
            tq = torch.empty(n, dtype=torch.float32, device=dev)
            xq = torch.empty(n, dtype=torch.float32, device=dev)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                ddf.hash_query(desc, params, r, ws=ws, t=tq, xi=xq)
            torch.cuda.current_stream().wait_stream(side)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                ddf.hash_query(desc, params, r, ws=ws, t=tq, xi=xq)
            g.replay()
            torch.cuda.synchronize()
            ms = timer.time(g.replay, max(10, steps))
            row["two_pass_graph"] = {"ms": ms, "rays_per_s": n / (ms * 1e-3), "us_per_ray": ms * 1e3 / n}
        res["query"][str(n)] = row
    B = 16384
    sc = I.scene_ellipsoids(1024, 3)
    prims = torch.from_numpy(ddf.scene_prims(sc)).to(dev)
    tr = torch.from_numpy(I.train_rays(sc, B, 1000)).to(dev)
    t_gt, hit = ddf.cast_targets(prims, tr)
    t_gt = torch.where(hit > 0, t_gt, torch.zeros_like(t_gt))
    p = torch.from_numpy(I.hash_params(desc, n_entries, 36)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ws = torch.empty(ddf.hash_train_workspace_bytes(desc, B), dtype=torch.uint8, device=dev)
    loss = torch.empty(4, dtype=torch.float32, device=dev)
    flag = torch.empty(4, dtype=torch.int32, device=dev)
    step = [0]

    def one():
        step[0] += 1
        hp = ddf.TrainHParamsC(3e-3, 0.9, 0.999, 1e-8, 0.3, 3.0, step[0], 0)
        ddf.hash_train_step(desc, p, m, v, tr, t_gt, hit, hp, ws, loss_out=loss, flag=flag)
    one()
    torch.cuda.synchronize()
    l0 = float(loss[0].item())
    ms = timer.time(one, max(10, steps))
    res["train"] = {"batch": B, "ms_per_step": ms, "train_rays_per_s": B / (ms * 1e-3), "loss_first": l0,
                    "loss_last": float(loss[0].item()), "steps": step[0], "skipped": int(flag[0].item())}
    return res


def shade_leg(torch, ddf, I, dev, timer, steps):
    """The renderer's use of the field (shadows, AO and one bounce; the paper's Table VI
    analogue): the paper's hash-grid field distilled by its recipe (`steps` steps of 16,384
    fresh GPU-sampled rays, 30 % self-consistency points, cosine lr from 3e-3 to 5 %) on one
    compound object above a ground slab; then one timed 512 x 512 frame: G-buffer from the
    exact scene, one shadow ray and 16 cosine-weighted hemisphere rays per pixel, the field's
    answers (two-pass hash query), the per-pixel shadow and AO maps and the one-bounce term
    (the radiance each hemisphere ray sees: a seeded surface-radiance grid at its hit point, or
    the sky).  Quality against the same rays cast exactly."""
    import time
    sc = I.scene_object(8, 5)
    desc = I.HASH_PAPER
    prims = torch.from_numpy(ddf.scene_prims(sc)).to(dev)
    cdf = ddf.prim_area_cdf(prims)
    n_entries = sum(ddf.hash_level(desc, l)[1] for l in range(desc.n_levels))
    p = torch.from_numpy(I.hash_params(desc, n_entries, 46)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    B, T = 16384, 4
    ws = torch.empty(ddf.hash_train_workspace_bytes(desc, B), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(48)
    U = torch.empty((3 * T + 2, B), device=dev)
    U3 = torch.empty((3, B), device=dev)
    loss = torch.empty(4, dtype=torch.float32, device=dev)
    flag = torch.empty(4, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(1, steps + 1):
        U.uniform_(generator=gen)
        U3.uniform_(generator=gen)
        rays = ddf.sample_rays(prims, U, mode=2, offset=I.NORMAL_OFFSET, cdf=cdf)
        t, h = ddf.cast_targets(prims, rays)
        t = torch.where(h > 0, t, torch.zeros_like(t))
        rs, ts, hs = ddf.shift_rays(rays, t, h, U3, 0.3)
        hp = ddf.TrainHParamsC(ddf.lr_cosine(st - 1, total=steps), 0.9, 0.999, 1e-8, 0.3, 3.0, st)
        ddf.hash_train_step(desc, p, m, v, rs, ts, hs, hp, ws, loss_out=loss, flag=flag)
        if st % 10000 == 0:
            torch.cuda.synchronize()
            progress(f"shade leg: {st} of {steps} training steps")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    view = I.View()
    K = I.AO_RAYS
    P = view.width * view.height
    u = torch.from_numpy(I.uniforms(2, P * K, 47)).to(dev)
    rays = torch.empty((6, P * (1 + K)), dtype=torch.float32, device=dev)
    qws = torch.empty(ddf.hash_query_workspace_bytes(desc, P * (1 + K)), dtype=torch.uint8, device=dev)
    res = {}

    radiance = torch.from_numpy(I.radiance_grid(I.RADIANCE_RES, 49)).to(dev)

    def frame():
        gb, hit = ddf.primary_gbuffer(view, prims)
        ddf.secondary_rays(gb, hit, I.SHADE_LIGHT, K, u, I.NORMAL_OFFSET, out=rays)
        tf, xf = ddf.hash_query(desc, p, rays, ws=qws)
        sh, ao = ddf.shade(tf, gb, hit, I.SHADE_LIGHT, K, I.NORMAL_OFFSET, xi=xf)
        gi = ddf.bounce(tf, rays, hit, K, radiance, I.BOX_HALF, I.SKY, xi=xf)
        res.update(gb=gb, hit=hit, sh=sh, ao=ao, gi=gi)
    for _ in range(2):
        frame()
    torch.cuda.synchronize()
    ms = timer.time(frame, 10)
    tg, rh = ddf.cast_targets(prims, rays)
    shr, aor = ddf.shade(tg, res["gb"], res["hit"], I.SHADE_LIGHT, K, I.NORMAL_OFFSET, ray_hit=rh)
    gir = ddf.bounce(tg, rays, res["hit"], K, radiance, I.BOX_HALF, I.SKY, ray_hit=rh)
    torch.cuda.synchronize()
    hm = res["hit"].cpu().numpy().astype(bool)
    sh, ao, gi, shr, aor, gir = (x.cpu().numpy().astype(np.float64)[hm]
                                 for x in (res["sh"], res["ao"], res["gi"], shr, aor, gir))

    def psnr(a, b):
        mse = float(np.mean((a - b) ** 2))
        return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)
    n_rays = P * (1 + K)
    return {"scene": "compound object of 8 ellipsoids on a ground slab", "train_steps": steps, "train_batch": B,
            "train_s": train_s, "train_ms_per_step": train_s * 1e3 / steps, "final_loss": float(loss[0].item()),
            "frame": f"{view.width}x{view.height}, 1 shadow + {K} AO rays per pixel", "frame_ms": ms,
            "secondary_rays": n_rays, "secondary_rays_per_s": n_rays / (ms * 1e-3),
            "pixels_hit": int(hm.sum()), "shadow_psnr_db": psnr(sh, shr), "ao_psnr_db": psnr(ao, aor),
            "ao_mae": float(np.mean(np.abs(ao - aor))), "bounce_psnr_db": psnr(gi, gir),
            "bounce_mae": float(np.mean(np.abs(gi - gir))),
            "paper_table6": {"shadow_psnr_db": 30.3, "ao_psnr_db": 21.3}}


def fit_sdf(torch, ddf, I, dev, scene, steps=3000, batch=65536, prec="bf16", seed=100, n_batches=48):
    """Fit the 12 x 1024 signed-distance MLP to the scene's analytic distance bound with the
    library's own fitting step (L1 on the distance, Adam, lr cosine-decayed from 1e-3 to
    1e-5), cycling through n_batches fixed batches of fitting points (half uniform in the
    box, half in two bands about the surface).  The default is the distilled DDF's budget:
    3,000 bf16 steps of 65,536 samples."""
    import math
    desc = I.NET_SDF
    prims = torch.from_numpy(ddf.scene_prims(scene)).to(dev)
    pool = [torch.from_numpy(I.sdf_fit_points(scene, batch, 40 + j)).to(dev) for j in range(n_batches)]
    gts = [ddf.scene_sdf(prims, p) for p in pool]
    master = torch.from_numpy(I.he_init(desc, seed)).to(dev)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    packed = ddf.pack(desc, prec, master)
    ws = torch.empty(ddf.train_workspace_bytes(desc, prec, batch), dtype=torch.uint8, device=dev)
    loss = torch.empty(4, dtype=torch.float32, device=dev)
    flag = torch.empty(4, dtype=torch.int32, device=dev)
    lr0, lr1 = 1e-3, 1e-5
    t0 = time.perf_counter()
    for s in range(1, steps + 1):
        lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * (s - 1) / steps))
        hp = ddf.TrainHParamsC(lr, 0.9, 0.999, 1e-8, 0.0, 1.0, s)
        j = (s - 1) % len(pool)
        ddf.sdf_train_step(desc, prec, master, m, v, packed, pool[j], gts[j], hp, ws, loss_out=loss, flag=flag)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    packed32 = ddf.pack(desc, "fp32", master)
    fit = {"steps": steps, "batch": batch, "batches": n_batches, "precision": prec, "lr": [lr0, lr1],
           "fit_s": fit_s, "final_loss": float(loss[0].item())}
    for name, pts in (("heldout", I.sdf_train_points(scene, batch, 99)),
                      ("heldout_near_surface", I.sdf_train_points(scene, batch, 98, sigma=0.005))):
        p = torch.from_numpy(pts).to(dev)
        err = (ddf.sdf_eval(desc, "fp32", packed32, p) - ddf.scene_sdf(prims, p)).abs()
        fit[f"{name}_mean_abs_err"] = float(err.mean().item())
        fit[f"{name}_p90_abs_err"] = float(err.quantile(0.9).item())
    return (packed32, ddf.pack(desc, "bf16", master)), fit


def trace_leg(torch, ddf, I, dev, shadow, timer, out, scene, fit_steps=3000):
    """Sphere tracing of a 12 x 1024 signed-distance MLP along the shadow leg's rays.

    The SDF MLP is fitted to the scene first (fit_sdf).  fp32, at most 128 steps, miss beyond
    t = 6: the persistent lane-refill trace (one launch) over 2^20 shadow rays at hit
    thresholds 1e-2, 1e-3 and 1e-4, each with its unconverged share and its ratio to the DDF
    query of the shadow leg.  A trace stops wherever |s| < threshold, also at its own origin,
    so for each threshold the ray origins are lifted max(1e-3, 2 x threshold) off the surface
    (the same surface points, and the 1e-3 lift of the DDF's rays at 1e-4); the share of rays
    that stop at their first evaluation is reported.  Then the step-synchronous trace at 1e-4
    (same answers bit for bit, its time for comparison); the bf16 trace at 1e-4 (the
    same-precision comparison with the bf16 DDF query); and, as in the paper's table of ray
    counts (Sec. IV-D, Table IV), the first 1K, 10K and 100K rays traced at 1e-3 and 1e-4
    against the fp32 and bf16 DDF queries of as many rays.  Rays still running after 128
    steps at 1e-4 are described by the network's value at their last point and its slope
    along the ray there (a central difference over +-1e-4): a step t + s converges on a root
    only where that slope lies in (-2, 0).  Returns the report and, per threshold, every
    128th ray of the traced set (host float32) for the cpu leg's float64 trace."""
    desc = I.NET_SDF
    (packed, packed_bf16), fit = fit_sdf(torch, ddf, I, dev, scene, steps=fit_steps)
    n = shadow.n
    prims = torch.from_numpy(ddf.scene_prims(scene)).to(dev)
    prec = out   # the shadow leg's query timings on the same rays, per precision
    edges = [1, 2, 4, 8, 16, 32, 64, 128, 129]
    sets = {}
    for eps in (1e-2, 1e-3, 1e-4):
        lift = max(I.NORMAL_OFFSET, 2 * eps)
        r = shadow.rays if lift == I.NORMAL_OFFSET else torch.from_numpy(I.shadow_rays(scene, n, 12, offset=lift)).to(dev)
        sets[eps] = (lift, r, ddf.cast_targets(prims, r)[1])

    def stuck(rays, hg, t, steps):
        u = (steps >= 128).nonzero().flatten()
        if u.numel() == 0:
            return {}
        o, d = rays[0:3, u], rays[3:6, u]
        h = 1e-4
        ev = lambda tt: ddf.sdf_eval(desc, "fp32", packed, (o + tt[None, :] * d).contiguous())
        s = ev(t[u])
        slope = (ev(t[u] + h) - ev(t[u] - h)) / (2 * h)
        return {"inside_fraction": float((s < 0).float().mean().item()),
                "abs_s_p10_p50_p90": [float(s.abs().quantile(q).item()) for q in (0.1, 0.5, 0.9)],
                "slope_along_ray_p10_p50_p90": [float(slope.quantile(q).item()) for q in (0.1, 0.5, 0.9)],
                "slope_below_minus2_fraction": float((slope <= -2).float().mean().item()),
                "exact_cast_hit_fraction": float((hg[u] > 0).float().mean().item())}

    def stats(ms, res_t, hg, m=n):
        t, hit, steps = res_t
        st = steps.float()
        hist = torch.bincount(steps.long().clamp(0, 128), minlength=129).cpu().numpy()
        r = {"ms": ms, "rays_per_s": m / (ms * 1e-3), "mean_steps": float(st.mean().item()),
             "p50_steps": float(st.median().item()), "unconverged_fraction": float((steps >= 128).float().mean().item()),
             "stopped_at_first_evaluation_fraction": float(((steps == 1) & (hit > 0)).float().mean().item()),
             "hit_rate": float(hit.float().mean().item()),
             "hit_agreement_vs_exact_cast": float((hit == hg[:m]).float().mean().item()),
             "steps_histogram": {f"{edges[i]}-{edges[i + 1] - 1}": int(hist[edges[i]:edges[i + 1]].sum())
                                 for i in range(len(edges) - 1)}}
        if m == n:
            for p in ("fp32", "bf16", "fp8"):
                msp = prec.get(p, {}).get("ms")
                if msp:
                    r[f"speedup_vs_ddf_{p}"] = ms / msp
        return r

    res = {"sdf": "12x1024 SDF MLP (L=10, 63 features) fitted to the scene's distance bound", "fit": fit,
           "max_steps": 128, "t_max": 6.0, "precision": "fp32", "pool": {}}
    wsp = torch.empty(256, dtype=torch.uint8, device=dev)
    for eps, (lift, r, hg) in sets.items():
        run = lambda: ddf.sphere_trace(desc, "fp32", packed, r, 128, eps, 6.0, ws=wsp, pool=True)
        ms = timer.time(run, 1)
        got = run()
        res["pool"][f"{eps:g}"] = dict(origin_lift=lift, **stats(ms, got, hg))
        if eps == 1e-4:
            res["pool"][f"{eps:g}"]["unconverged_rays"] = stuck(r, hg, got[0], got[2])
    lift, rays, hg = sets[1e-4]
    ws = torch.empty(int(ddf.lib().sdf_trace_workspace_bytes(n)), dtype=torch.uint8, device=dev)
    run = lambda: ddf.sphere_trace(desc, "fp32", packed, rays, 128, 1e-4, 6.0, ws=ws)
    ms = timer.time(run, 1)
    res["step_synchronous_1e-4"] = stats(ms, run(), hg)
    run = lambda: ddf.sphere_trace(desc, "bf16", packed_bf16, rays, 128, 1e-4, 6.0, ws=wsp, pool=True)
    ms16 = timer.time(run, 1)
    r16 = stats(ms16, run(), hg)
    res["bf16_pool_1e-4"] = {k: v for k, v in r16.items() if k != "steps_histogram"}

    by_n = {}
    for m in (1000, 10000, 100000):
        row = {}
        tq = torch.empty(m, dtype=torch.float32, device=dev)
        xq = torch.empty(m, dtype=torch.float32, device=dev)
        rq = shadow.rays[:, :m].contiguous()
        for p in ("fp32", "bf16"):
            pk, dc = shadow.packed(p), ddf.desc_c(shadow.desc, p)
            for _ in range(3):
                ddf.query_into(dc, pk, rq, tq, xq)
            torch.cuda.synchronize()
            row[f"ddf_{p}_ms"] = timer.time(lambda: ddf.query_into(dc, pk, rq, tq, xq), 20)
        for eps in (1e-3, 1e-4):
            lift, r, hg = sets[eps]
            r = r[:, :m].contiguous()
            run = lambda: ddf.sphere_trace(desc, "fp32", packed, r, 128, eps, 6.0, ws=wsp, pool=True)
            run()
            ms = timer.time(run, 3)
            s = {k: v for k, v in stats(ms, run(), hg, m).items() if k not in ("steps_histogram", "rays_per_s")}
            s.update({f"speedup_vs_ddf_{p}": ms / row[f"ddf_{p}_ms"] for p in ("fp32", "bf16")})
            row[f"trace_{eps:g}"] = s
        by_n[str(m)] = row
    res["by_ray_count"] = by_n
    host = {eps: (lift, r[:, ::128].cpu().numpy()) for eps, (lift, r, hg) in sets.items()}
    return res, host


def trace_oracle_stats(scene, host_sets, report, max_steps=128, t_max=6.0):
    """cpu leg, the trace baseline's yardstick: the float64 oracle sphere-traces the scene's
    analytic distance bound itself (the function the SDF MLP was fitted to) along every 128th
    ray of each threshold's traced set: evaluations per ray, unconverged share, rays stopping
    at their first evaluation and hits against exact casting."""
    from oracle import geometry as G
    out = {}
    for eps, (lift, r) in host_sets.items():
        o = r[0:3].T.astype(np.float64)
        d = r[3:6].T.astype(np.float64)
        t0 = time.perf_counter()
        _, hg = G.intersect(scene, o, d)[:2]
        _, hit, steps, _ = G.sphere_trace(lambda p: G.sdf(scene, p), o, d, max_steps, eps, t_max)
        out[f"{eps:g}"] = {"rays": int(len(o)), "origin_lift": lift, "mean_steps": float(steps.mean()),
                           "unconverged_fraction": float((steps >= max_steps).mean()),
                           "stopped_at_first_evaluation_fraction": float(((steps == 1) & hit).mean()),
                           "hit_agreement_vs_exact_cast": float((hit == hg).mean()),
                           "oracle_s": time.perf_counter() - t0}
    report["exact_bound_float64"] = out


if __name__ == "__main__":
    main()

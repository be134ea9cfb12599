/*
 * ddf.h -- C ABI of the MI355X (gfx950) directed-distance-field hot path.
 *
 * A directed distance field (DDF) maps a ray, origin x in R^3 and unit
 * direction d, to (t, xi): the distance from x along d to the first surface
 * and the probability that the ray hits anything (paper Sec. III-A, Eq. 1).
 * The field here is the sinusoidal-encoding MLP form (Sec. IV-C, Table II):
 *
 *   gamma(v) = [v, sin(pi 2^0 v), cos(pi 2^0 v), ..., sin(pi 2^(L-1) v), cos(pi 2^(L-1) v)]
 *   h_1 = relu(W_1 gamma + b_1),  h_l = relu(W_l h_(l-1) + b_l)  (l = 2..n_hidden)
 *   z   = W_head h_n + b_head,    t = softplus(z_0),  xi = sigmoid(z_1)
 *
 * Every query is one forward pass (Sec. III-C).  The same network shape with
 * n_in = 3 and one linear output is the signed-distance MLP that the SDF
 * sphere-tracing baseline evaluates once per step (Sec. IV-D, Table IV).
 *
 * Conventions for every entry point:
 *  - Buffer pointers are DEVICE pointers owned by the caller, 16-byte
 *    aligned.  Descriptors and hyper-parameters are host structs.  The
 *    library never allocates, frees or synchronises; all work is enqueued
 *    on `stream` (a hipStream_t passed as void*, NULL = the null stream).
 *  - Arguments are validated on the host before anything is enqueued; on a
 *    failure nothing is written, the call returns a negative ddf_status and
 *    ddf_last_error() holds a message (thread-local).
 *  - n == 0 is a valid no-op.
 *  - Rays are float32 SoA [6][n]: rows x0, x1, x2, d0, d1, d2 (row stride n).
 *    Directions are expected to be unit length; they are not renormalised.
 *    A NaN in a ray only affects that ray's outputs.
 *  - The float32 master parameter vector is flat: for each hidden layer
 *    W_l [width][fan_in] row-major then b_l [width]; then W_head
 *    [n_out][width] and b_head [n_out].  fan_in of layer 1 is
 *    n_in (1 + 2 n_freq).
 */
#ifndef DDF_H_
#define DDF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DDF_OK = 0,
  DDF_ERR_INVALID_ARG = -1,  /* bad pointer, size, descriptor field or alignment */
  DDF_ERR_UNSUPPORTED = -2,  /* valid but not built: width/precision combination */
  DDF_ERR_WORKSPACE = -3,    /* workspace smaller than the sizing call returned */
  DDF_ERR_HIP = -4           /* a HIP launch or runtime call failed */
} ddf_status;

typedef enum {
  DDF_FP32 = 0,      /* float32 operands on the fp32 matrix cores */
  DDF_BF16 = 1,      /* bf16 operands, fp32 accumulation */
  DDF_FP8_E4M3 = 2   /* OCP e4m3 hidden layers with per-layer power-of-two scales */
} ddf_precision;

typedef struct {
  int32_t n_in;       /* 6 = DDF ray (x, d); 3 = SDF point p */
  int32_t n_freq;     /* L, frequency bands of the encoding (1..12) */
  int32_t n_hidden;   /* Linear+ReLU layers, 1..32; the first maps the features to width */
  int32_t width;      /* 128, 256, 512 or 1024 */
  int32_t n_out;      /* 2 = (z_t, z_xi) for a DDF; 1 = signed distance */
  int32_t precision;  /* ddf_precision of the hidden-layer products */
} ddf_net_desc;

/* Human-readable name of a status code; static storage. */
const char* ddf_status_string(int status);
/* Detail of the last failure on the calling thread ("" if none). */
const char* ddf_last_error(void);

/* Length of the float32 master parameter vector (layout above); 0 if desc is invalid. */
size_t ddf_param_count(const ddf_net_desc* desc);

/* Float offsets of one layer's weight and bias in the master vector (the layout above).
 *   layer  0 .. n_hidden - 1: hidden layer layer + 1 (W [width][fan_in], then b [width]);
 *          n_hidden: the head (W_head [n_out][width], then b_head [n_out]).
 *   w_off, b_off  host, written on success.
 * Returns DDF_ERR_INVALID_ARG (nothing written) for an invalid desc, a layer outside
 * 0..n_hidden or a NULL output. */
int ddf_param_offsets(const ddf_net_desc* desc, int32_t layer, size_t* w_off, size_t* b_off);

/* Bytes of the packed working copy of the network for desc->precision; 0 if invalid.
 * The packed form is opaque: weights pre-arranged in matrix-core operand order,
 * fp32 biases and heads, and (FP8) the per-layer scales. */
size_t ddf_packed_bytes(const ddf_net_desc* desc);

/* Build the packed working copy from the float32 master.
 *   master      device, ddf_param_count floats, read only.
 *   act_scales  host, FP8 only (else may be NULL): n_hidden - 1 power-of-two scales
 *               s_A of the inputs of hidden layers 2..n_hidden (an input h is stored as
 *               e4m3(h / s_A)); see ddf_fp8_act_scales.
 *   packed      device, ddf_packed_bytes bytes, written.
 * FP8 weight scales are computed here, per hidden layer l >= 2, as the smallest power of
 * two s_W with max|W_l| / s_W <= 448.  Layer 1 stays bf16 (hi + lo split input) and the
 * heads fp32 in every reduced precision. */
int ddf_pack(const ddf_net_desc* desc, const float* master, const float* act_scales,
             void* packed, void* stream);

/* The batched DDF query (Sec. III-A Eq. 1, Sec. III-C): one forward pass per ray.
 *   packed  device, from ddf_pack with the same desc.
 *   rays    device float32 [6][n] SoA.
 *   t, xi   device float32 [n]: t = softplus(z_t) >= 0, xi = sigmoid(z_xi) in [0, 1].
 * desc->n_in must be 6 and desc->n_out 2. */
int ddf_query(const ddf_net_desc* desc, const void* packed, const float* rays, int64_t n,
              float* t, float* xi, void* stream);

/* The last hidden layer's activations, h_n = relu(W_n h_(n-1) + b_n) in float32 exactly as
 * the heads of ddf_query read them (before any rounding to the next layer's operand type),
 * for inspection of one layer at a time: querying the network cut after layer l (the first l
 * hidden layers of a master vector, any head, packed with n_hidden = l and, for FP8, the
 * first l - 1 activation scales) gives the kernel's own h_l, and the layer above it is then
 * checked in isolation against its definition (Sec. III-A network, Sec. III-C reduced
 * precision).
 *   packed  device, from ddf_pack with the same desc.
 *   in      device float32 [n_in][n] SoA (rays, or points for n_in 3).
 *   h       device float32 [n][width], row per ray, written.
 * Same launch shape and arithmetic as ddf_query / sdf_eval on the same desc. */
int ddf_query_hidden(const ddf_net_desc* desc, const void* packed, const float* in, int64_t n,
                     float* h, void* stream);

/* Per-layer power-of-two FP8 input scales from a calibration batch (host result).
 * Runs the float32 forward of `master` (desc with precision DDF_FP32 semantics) over
 * `rays` [6][n] and returns in act_scales_host[0 .. n_hidden-2] the smallest power of
 * two s with max(h_(l-1)) / s <= 448 for l = 2..n_hidden.  Synchronises `stream`.
 *   packed_fp32  device, ddf_packed_bytes of desc with precision DDF_FP32, from ddf_pack.
 *   ws           device workspace, ddf_fp8_calib_workspace_bytes(desc, n) bytes. */
size_t ddf_fp8_calib_workspace_bytes(const ddf_net_desc* desc, int64_t n);
int ddf_fp8_act_scales(const ddf_net_desc* desc, const void* packed_fp32, const float* rays,
                       int64_t n, float* act_scales_host, void* ws, size_t ws_bytes,
                       void* stream);

/* ------------------------------------------------------------------ training */

typedef struct {
  float lr;            /* learning rate of this step (the caller applies the schedule) */
  float beta1, beta2;  /* Adam moments, e.g. 0.9, 0.999 */
  float eps;           /* Adam epsilon, e.g. 1e-8 */
  float bce_weight;    /* weight of the hit cross-entropy, 0.3 (Sec. III-D) */
  float l1_clamp;      /* clamp of the per-ray L1 distance error, e.g. 3.0 (box scale) */
  int64_t step;        /* 1-based Adam step count (bias correction) */
  int32_t recompute_every; /* activation recomputation span k (see below); 0 = keep all */
} ddf_train_hparams;

/* Activation recomputation (the deep-net training mode): with recompute_every = k,
 * 0 < k < n_hidden, the training forward keeps only the encoded features and the
 * checkpoints H_k, H_2k, .., H_n; the backward pass walks the layers in segments from the
 * top and reruns each segment's forward from the checkpoint below it (bit-identical to the
 * first pass) before its deltas and weight gradients.  Costs up to one extra forward pass;
 * keeps ceil(n/k) + k - 1 activation slabs and k + 1 delta slabs instead of n and n.
 * k = 0 or k >= n_hidden keeps every activation.  Negative k is DDF_ERR_INVALID_ARG.
 * The same k must be used for the workspace size, the forward and the backward call. */

/* Workspace for one training step / backward pass over `batch` rays. */
size_t ddf_train_workspace_bytes(const ddf_net_desc* desc, int64_t batch, int32_t recompute_every);

/* Training-mode forward: z_t and z_xi logits per ray [n], and the activations the
 * backward pass needs kept in `ws`.  Same numerics as ddf_query. */
int ddf_forward_train(const ddf_net_desc* desc, const void* packed, const float* rays,
                      int64_t n, float* z_t, float* z_xi, int32_t recompute_every, void* ws,
                      size_t ws_bytes, void* stream);

/* Backward pass of the network for given logit gradients (dL/dz_t, dL/dz_xi), each
 * device float32 [n]; must follow ddf_forward_train on the same rays, recompute_every and
 * ws (rays are read again when the first segment is recomputed).  Writes the float32
 * gradient of every parameter (master layout) to grad_params (device). */
int ddf_backward(const ddf_net_desc* desc, const void* packed, const float* rays, int64_t n,
                 const float* grad_z_t, const float* grad_z_xi, float* grad_params,
                 int32_t recompute_every, void* ws, size_t ws_bytes, void* stream);

/* The activation H_layer (1 <= layer <= n_hidden, post-ReLU) that ddf_forward_train kept in
 * ws for n rays, as float32 [n][width] (device, written): the values the backward pass reads,
 * in the operand type they were kept in (bf16 for the reduced precisions), so that H > 0 are
 * the ReLU masks the backward pass applies (Sec. III-B distillation; for inspecting one
 * layer of the training path).  desc, n and recompute_every as for the forward call; with
 * recomputation only checkpoint layers (multiples of k, and n_hidden) are kept, any other
 * layer is DDF_ERR_INVALID_ARG.  ws must still hold that forward pass's activations. */
int ddf_train_kept_activation(const ddf_net_desc* desc, int64_t n, int32_t recompute_every,
                              const void* ws, size_t ws_bytes, int32_t layer, float* h,
                              void* stream);

/* One distillation step (Sec. III-B, III-D): forward, loss, backward, Adam, repack.
 *   loss = mean over hit rays of min(|softplus(z_t) - t_gt|, l1_clamp)
 *        + bce_weight * mean over all rays of BCE(sigmoid(z_xi), hit_gt)
 *   master, adam_m, adam_v   device float32 [ddf_param_count], updated in place.
 *   packed                   device, rebuilt from the new master (FP8 keeps its
 *                            activation scales).
 *   t_gt                     device float32 [batch], ignored where hit_gt == 0.
 *   hit_gt                   device uint8 [batch], 0 or 1.
 *   loss_out                 device float32 [3]: total, l1 term, bce term.
 *   nonfinite_flag           device int32 [1]: set to 1 and the update skipped (master,
 *                            m, v untouched) when any gradient is not finite, else 0.
 *   grad_out                 device float32 [ddf_param_count] or NULL: the gradient.
 *   ws                       ddf_train_workspace_bytes(desc, batch, hp->recompute_every). */
int ddf_train_step(const ddf_net_desc* desc, float* master, float* adam_m, float* adam_v,
                   void* packed, const float* rays, const float* t_gt, const uint8_t* hit_gt,
                   int64_t batch, const ddf_train_hparams* hp, float* loss_out,
                   int32_t* nonfinite_flag, float* grad_out, void* ws, size_t ws_bytes,
                   void* stream);

/* ------------------------------------------------------------------ baselines / data */

/* Sphere tracing of an SDF MLP (the baseline of Sec. IV-D, Table IV): per ray, from
 * t = 0, evaluate s = sdf(x + t d); |s| < hit_eps is a hit, else t += s; t > t_max is a
 * miss; max_steps evaluations without either is a miss that did not converge.
 *   desc    n_in 3, n_out 1.   packed from ddf_pack.   rays [6][n].
 *   t       device float32 [n], final t.   hit device uint8 [n].
 *   steps   device int32 [n] or NULL: SDF evaluations used by each ray.
 *   ws      sdf_trace_workspace_bytes(n) bytes. */
size_t sdf_trace_workspace_bytes(int64_t n);
int sdf_sphere_trace(const ddf_net_desc* desc, const void* packed, const float* rays,
                     int64_t n, int32_t max_steps, float hit_eps, float t_max, float* t,
                     uint8_t* hit, int32_t* steps, void* ws, size_t ws_bytes, void* stream);

/* The same sphere trace as one persistent launch with lane refill (the baseline given its best
 * form for this chip): one workgroup per compute unit holds a tile of ray slots for the whole
 * trace; whenever rays finish (hit, t > t_max, or max_steps evaluations) their slots take the
 * next rays of the pool, so every evaluation runs on a full tile until the pool is exhausted,
 * with no per-step launches or active-list compaction.  Same arguments and results as
 * sdf_sphere_trace, bit for bit (t, hit, steps); ws: device, >= 256 bytes (the pool counter),
 * overwritten.  fp32 and bf16 nets of width 256, 512 or 1024 (else DDF_ERR_UNSUPPORTED). */
int sdf_sphere_trace_pool(const ddf_net_desc* desc, const void* packed, const float* rays, int64_t n,
                          int32_t max_steps, float hit_eps, float t_max, float* t, uint8_t* hit,
                          int32_t* steps, void* ws, size_t ws_bytes, void* stream);

/* The small-batch query (the sparse regime, ~1K-5K rays): bf16 nets of width 256, 512
 * or 1024 only.  One launch per layer with the layer's neurons split over workgroups (64
 * rays x 256 neurons each), so that a small batch still spreads over every CU; the
 * activations pass through ws between layers.  Hidden activations are bit-identical to
 * ddf_query's; the heads' sums run in another order (float32 rounding).  ws: device,
 * >= ddf_query_split_workspace_bytes(desc, n) (else DDF_ERR_WORKSPACE), overwritten; n <=
 * 2^25.  Faster than ddf_query below ~5K rays (half the time at 1K), slower above. */
size_t ddf_query_split_workspace_bytes(const ddf_net_desc* desc, int64_t n);
int ddf_query_split(const ddf_net_desc* desc, const void* packed, const float* rays, int64_t n, float* t,
                    float* xi, void* ws, size_t ws_bytes, void* stream);

/* Signed-distance MLP at points: sdf [n] for points float32 SoA [3][n]. */
int sdf_eval(const ddf_net_desc* desc, const void* packed, const float* points, int64_t n,
             float* sdf, void* stream);

/* Exact supervision targets by brute-force ray casting against an analytic union of
 * spheres/ellipsoids (the paper's exact ray-cast supervision source, Sec. III-B).
 *   prims  device float32 [n_prims][16]: center(3), 1/semi-axes(3), R^T row-major(9),
 *          min semi-axis(1), where a primitive is {c + R (a * u) : |u| <= 1}.
 *   t_gt   device float32 [n]: first root > 0 over all primitives (+inf on a miss).
 *   hit    device uint8 [n]. */
int ddf_cast_targets(const float* prims, int32_t n_prims, const float* rays, int64_t n,
                     float* t_gt, uint8_t* hit, void* stream);

/* Signed-distance bound of the same analytic union at points (targets for fitting an SDF
 * MLP): min over primitives of (|R^T (p - c) / a| - 1) * min(a), exact for spheres and a
 * lower bound for ellipsoids.  prims as for ddf_cast_targets with slot 15 = min(a).
 *   points  device float32 [3][n] SoA.   sdf  device float32 [n]. */
int ddf_scene_sdf(const float* prims, int32_t n_prims, const float* points, int64_t n, float* sdf,
                  void* stream);

/* Self-consistency points for distillation (Sec. III-B; Sec. III-D replaces 30 % of each
 * batch with them): along a ray that hits at t, the point moved forward by s must report
 * t - s.  For every slot i of a batch of n rays with targets:
 *   u[0][i] < frac: the slot takes the first hit ray j among the 1024 rays from index
 *                   floor(u[1][i] n) on (cyclic), origin x_j + s d_j with s = u[2][i] t_j,
 *                   direction d_j, t_out = t_j - s, hit_out = 1 (the slot is copied when
 *                   none of them hits);
 *   otherwise:      a copy of ray i, t_gt[i], hit[i].
 *   rays, rays_out  device float32 [6][n] SoA (must not alias).
 *   t_gt, t_out     device float32 [n].   hit, hit_out  device uint8 [n].
 *   u               device float32 [3][n], uniforms in [0, 1) drawn by the caller.
 *   frac            in [0, 1], e.g. 0.3. */
int ddf_shift_rays(const float* rays, const float* t_gt, const uint8_t* hit, const float* u, float frac,
                   int64_t n, float* rays_out, float* t_out, uint8_t* hit_out, void* stream);

/* The distillation learning rate at `step` (host function, Sec. III-D): cosine decay from
 * lr0 to final_frac * lr0 over `total` steps, held after; e.g. (3e-3, 0.05, 30000). */
float ddf_lr_cosine(int64_t step, int64_t total, float lr0, float final_frac);

/* One fitting step of an SDF MLP (desc n_in 3, n_out 1) by Adam on the L1 error
 *   loss = mean over points of |s(p) - sdf_gt(p)|
 * with the same forward, backward, Adam and repack as ddf_train_step (hp->bce_weight and
 * hp->l1_clamp are ignored).  points [3][n], sdf_gt [n]; loss_out device float32 [3]
 * (loss, loss, 0); workspace ddf_train_workspace_bytes(desc, n, hp->recompute_every). */
int sdf_train_step(const ddf_net_desc* desc, float* master, float* adam_m, float* adam_v, void* packed,
                   const float* points, const float* sdf_gt, int64_t n, const ddf_train_hparams* hp,
                   float* loss_out, int32_t* nonfinite_flag, float* grad_out, void* ws, size_t ws_bytes,
                   void* stream);

/* ------------------------------------------------------------------ hash-grid field */

/* The paper's fast field (Sec. III-D): the ray origin through a multiresolution hash
 * encoding (level l of resolution N_l = floor(base_res growth^l) over the box
 * [-box_half, box_half]^3, n_feat features per vertex, trilinear lookups, dense indexing
 * while (N_l + 1)^3 <= 2^log2_table, else the spatial hash (v0 XOR 2654435761 v1 XOR
 * 805459861 v2) mod 2^log2_table), the direction through dir_bands sinusoidal bands
 * ([d, sin(pi 2^k d), cos(pi 2^k d)]), a ReLU MLP of n_hidden layers of width 64, and the
 * heads t = softplus(z_t), xi = sigmoid(z_xi).  The paper's field: 16 levels, 2 features,
 * 2^19, 16, 1.5, 4 bands, 2 x 64, box 1.5: 13.07M parameters, 52 MB in float32.
 * Points outside the box are clamped to it; in float32, p = (x + box_half) (0.5 / box_half)
 * clamped to [0, 1], s = p N, and the cell is min(floor(s), N - 1).  Compiled shapes:
 * n_levels 16 or 6, dir_bands 4, n_feat 2, width 64, n_hidden 2, n_out 2; any other desc
 * returns DDF_ERR_UNSUPPORTED (DDF_ERR_INVALID_ARG for base_res < 1, growth outside
 * [1, 8], box_half <= 0), and the finest resolution must stay below 1e6. */
typedef struct {
  int32_t n_levels, n_feat, log2_table, base_res;
  float growth;
  int32_t dir_bands, width, n_hidden, n_out;
  float box_half;
} ddf_hash_desc;

/* Parameter vector length (0 for an unsupported desc): the table, level after level,
 * n_feat floats per entry; then W1 [64][D], b1, W_l [64][64], b_l, heads [2][64], [2]
 * with D = 2 n_levels + 3 (1 + 2 dir_bands). */
size_t ddf_hash_param_count(const ddf_hash_desc* desc);

/* Level `level`'s resolution, table entries, entry offset and whether it is hashed
 * (host; any output pointer may be NULL). */
int ddf_hash_level(const ddf_hash_desc* desc, int32_t level, int32_t* resolution, int64_t* entries,
                   int64_t* offset, int32_t* hashed);

/* Bytes of the two-pass query's workspace for n rays (8 x n x 16: each ray's lookups,
 * 2 levels per group); 0 for an unsupported desc or n < 0. */
size_t ddf_hash_query_workspace_bytes(const ddf_hash_desc* desc, int64_t n);

/* Query: params device float32 [ddf_hash_param_count]; rays [6][n]; t, xi [n]; n <= 2^31 - 1.
 * ws == NULL: one fused kernel per ray block (lookups, direction code, MLP, heads).
 * ws != NULL (device, >= ddf_hash_query_workspace_bytes(desc, n), else DDF_ERR_INVALID_ARG):
 * two passes, the lookups with the table's level groups pinned to XCDs (each XCD's L2 then
 * holds 2 of the 16 levels), then the MLP on the matrix cores (fp32); the lookups are
 * bit-identical to the fused path's, the MLP sums in another order (float32 rounding).
 * ws is scratch, overwritten; calls sharing one ws must not overlap. */
int ddf_hash_query(const ddf_hash_desc* desc, const float* params, const float* rays, int64_t n,
                   float* t, float* xi, void* ws, size_t ws_bytes, void* stream);

/* The two-pass query without a caller workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same kernels and results as ddf_hash_query with ws, bit for bit, with the lookups staged in
 * a 64 MiB array inside the library (held by every GPU the library runs on until the process
 * ends).  The call allocates nothing.  n <= ddf_hash_query_static_max_rays() (524,288), else
 * DDF_ERR_INVALID_ARG with nothing written; other arguments as for ddf_hash_query.  Every
 * call on a GPU uses that GPU's one array, fully overwritten before it is read: calls that
 * overlap on one GPU (other streams, other threads) race and must be serialised by the
 * caller. */
int64_t ddf_hash_query_static_max_rays(void);
int ddf_hash_query_static(const ddf_hash_desc* desc, const float* params, const float* rays, int64_t n,
                          float* t, float* xi, void* stream);

/* The reduced-precision query (Sec. III-C: inference runs in reduced precision): a float16
 * copy of the table, round to nearest even, [entries][2] (ddf_hash_table_f16_bytes bytes,
 * device), made after each change to params; the lookups read it (half the bytes and cache
 * lines of the float32 table), the interpolation and the MLP stay float32.  Results equal
 * the float32 query's on a table rounded to float16.  Two-pass only: ws as for
 * ddf_hash_query, required. */
size_t ddf_hash_table_f16_bytes(const ddf_hash_desc* desc);
int ddf_hash_table_to_f16(const ddf_hash_desc* desc, const float* params, void* table16, void* stream);
int ddf_hash_query_f16(const ddf_hash_desc* desc, const float* params, const void* table16, const float* rays,
                       int64_t n, float* t, float* xi, void* ws, size_t ws_bytes, void* stream);

/* One distillation step of the hash-grid field: forward, the loss of ddf_train_step,
 * backward (the table gradient gathered with float atomics: its summation order is not
 * fixed; every other reduction is), Adam over all parameters (skipped on a non-finite
 * gradient).  Arguments as ddf_train_step; hp->recompute_every is ignored; workspace
 * ddf_hash_train_workspace_bytes(desc, batch). */
size_t ddf_hash_train_workspace_bytes(const ddf_hash_desc* desc, int64_t batch);
int ddf_hash_train_step(const ddf_hash_desc* desc, float* params, float* adam_m, float* adam_v,
                        const float* rays, const float* t_gt, const uint8_t* hit_gt, int64_t batch,
                        const ddf_train_hparams* hp, float* loss_out, int32_t* nonfinite_flag,
                        float* grad_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ shading consumers */

/* A renderer's use of the field (Sec. III-C; shadows and ambient occlusion against a
 * reference ray tracer, Sec. IV-F, Table VI).  Primary visibility comes from the exact scene;
 * the secondary rays go to the field (ddf_query / ddf_hash_query) or, for the reference maps,
 * to ddf_cast_targets; ddf_shade turns the answers into per-pixel maps.
 *
 * Pinhole camera: pixel (i, j), row 0 at the top, looks along
 * normalise(f + s_x r + s_y u), s_x = (2 (i + 0.5) / W - 1) tan(fov_y / 2) W / H,
 * s_y = (1 - 2 (j + 0.5) / H) tan(fov_y / 2), f = normalise(target - eye),
 * r = normalise(f x up), u = r x f (frame computed on the host in double). */
typedef struct {
  float eye[3], target[3], up[3];
  float fov_y;                /* radians, in (0, 3.1) */
  int32_t width, height;      /* width * height <= 2^31 - 1 */
} ddf_camera;

/* G-buffer of the W x H pixels (P = W H, row-major): gbuf [6][P] float32 = hit point and
 * outward unit normal (zeros for background), hit [P] uint8.  prims [n_prims][16] as for
 * ddf_cast_targets (device); all device pointers 16-byte aligned. */
int ddf_primary_gbuffer(const ddf_camera* cam, const float* prims, int32_t n_prims, float* gbuf, uint8_t* hit,
                        void* stream);

/* Secondary rays [6][n_px (1 + n_ao)], pixel-major: for pixel i, ray i (1 + n_ao) goes from
 * o = p + offset n toward light (host, 3 floats), rays i (1 + n_ao) + 1 + k are cosine-weighted
 * over the hemisphere around n (Malley's method in the orthonormal basis of Duff et al.
 * 2017) from uniforms u [2][n_px n_ao] (device; u[0] the radius draw, u[1] the angle draw).
 * Background pixels get finite dummy rays (p, +z).  0 <= n_ao <= 1024, offset >= 0,
 * n_px (1 + n_ao) <= 2^31 - 1. */
int ddf_secondary_rays(const float* gbuf, const uint8_t* hit, int64_t n_px, const float* light, int32_t n_ao,
                       const float* u, float offset, float* rays, void* stream);

/* Per-pixel maps from the answers t [n_px (1 + n_ao)] and exactly one of xi (the field's,
 * a ray hits when xi > 0.5) or ray_hit (uint8, the exact cast's): shadow[i] = 1 when the
 * shadow ray hits with t < |light - o|, ao[i] = the share of AO rays that hit with
 * t < ao_radius (> 0; +inf counts every hit).  Background pixels get 0 and 0. */
int ddf_shade(const float* t, const float* xi, const uint8_t* ray_hit, const float* gbuf, const uint8_t* hit,
              int64_t n_px, const float* light, int32_t n_ao, float offset, float ao_radius, float* shadow, float* ao,
              void* stream);

/* One bounce of global illumination (Sec. I: a bounce query asks what a surface point sees in
 * some direction; the renderer's use of the oracle, Sec. IV-F): per pixel, the mean over its
 * n_ao cosine-weighted hemisphere rays (rays i (1 + n_ao) + 1 .. + n_ao of ddf_secondary_rays;
 * cosine-weighted, so each carries the same weight for a diffuse surface) of the radiance the
 * ray sees:
 *   a hit (xi > 0.5, or ray_hit set): the surface radiance at o + t d, trilinear in the vertex
 *     grid radiance over [-box_half, box_half]^3 (the point clamped to the box);
 *   a miss: the sky, sky_lo + (sky_hi - sky_lo) (d_y + 1) / 2.
 *   t, and exactly one of xi / ray_hit   [n_px (1 + n_ao)], the answers to the secondary rays.
 *   rays        [6][n_px (1 + n_ao)] the secondary rays.   hit [n_px] primary hits (G-buffer).
 *   radiance    device float32 [res][res][res], vertex (x, y, z) at index x + res (y + res z),
 *               vertex coordinate -box_half + 2 box_half j / (res - 1); 2 <= res <= 1024.
 *   gi          device float32 [n_px]: the bounce term, 0 for background pixels.
 * 0 <= n_ao <= 1024 (n_ao = 0 gives 0), n_px (1 + n_ao) <= 2^31 - 1. */
int ddf_bounce(const float* t, const float* xi, const uint8_t* ray_hit, const float* rays, const uint8_t* hit,
               int64_t n_px, int32_t n_ao, const float* radiance, int32_t res, float box_half, float sky_lo,
               float sky_hi, float* gi, void* stream);

/* ------------------------------------------------------------------ training rays */

/* Training rays [6][n] on the GPU (Sec. III-B: rays from the surface in every direction,
 * for the secondary visibility shadows and AO need, and rays of the rendered views, here
 * free rays from the box).  mode 0: surface rays, 1: free rays, 2: surface at even and free
 * at odd positions.  A surface ray starts at c + R (a s) + offset n on a primitive chosen
 * with probability proportional to its surface area (Thomsen's ellipsoid approximation),
 * s uniform on the sphere, n the outward normal; a free ray starts uniform in
 * [-box_half, box_half]^3; a start strictly inside another (any, for free rays) primitive is
 * rejected and the next candidate taken, up to `tries` (1..16; the last is kept).
 * Directions are uniform on the sphere.  u [3 tries + 2][n] device uniforms in [0, 1): rows
 * 3j .. 3j + 2 drive candidate j (primitive choice and sphere point, or x, y, z), the last
 * two the direction (z = 1 - 2 u, phi = 2 pi u').  cdf [n_prims]: the cumulative area
 * weights from ddf_prim_area_cdf (once per scene).  n <= 2^26. */
int ddf_sample_rays(const float* prims, int32_t n_prims, const float* cdf, const float* u, int64_t n, int32_t mode,
                    float box_half, float offset, int32_t tries, float* rays, void* stream);

/* Cumulative surface-area weights of the primitives, cdf [n_prims] (device), normalised to
 * end at exactly 1 (computed in double). */
int ddf_prim_area_cdf(const float* prims, int32_t n_prims, float* cdf, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DDF_H_ */

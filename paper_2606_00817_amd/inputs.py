"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no encoding, no network, no loss, no intersection, no
distance evaluation).  Everything is drawn with numpy's PCG64 in float64 and
stored as float32, so both sides of a parity test start from the same bits.

Workloads follow the paper's query types (Sec. III-C: shadow, ambient
occlusion, one-bounce rays; Sec. III-B: camera/free rays and surface-anchored
rays for training) on analytic scenes of spheres and ellipsoids placed in the
normalised object box [-1.5, 1.5]^3 (Sec. III-D: the box that bounds the
normalised object).  Scenes stand in for the paper's object datasets.

Layouts
-------
* rays: float32 SoA array of shape [6, N]: rows x0, x1, x2, d0, d1, d2.
* params: flat float32 master vector.  For each hidden layer l (1-based,
  n_hidden of them) the weight W_l stored [out][in] row-major, then its bias
  b_l; then the head weight [n_out][width] and head bias [n_out].  For the
  DDF head row 0 is the distance logit z_t and row 1 the visibility logit
  z_xi; for the SDF net the single row is the signed distance.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LIGHT_POS = (0.0, 3.0, 0.0)     # point light of the shadow workload
BOX_HALF = 1.5                  # the normalised object box is [-1.5, 1.5]^3
NORMAL_OFFSET = 1e-3            # shadow/AO/GI origins are lifted along the normal


@dataclasses.dataclass(frozen=True)
class NetDesc:
    """Shape of a positional-encoding MLP (sinusoidal encoding, Sec. IV-C)."""
    n_in: int = 6        # 6 for a DDF ray (x, d); 3 for an SDF point p
    n_freq: int = 10     # number of frequency bands L
    n_hidden: int = 12   # Linear+ReLU layers, the first maps D -> width
    width: int = 1024
    n_out: int = 2       # 2 = (z_t, z_xi); 1 = signed distance

    @property
    def n_feat(self) -> int:
        return self.n_in * (1 + 2 * self.n_freq)

    def layer_shapes(self):
        """(out, in) of every weight matrix, hidden layers then the head."""
        shapes = []
        fan_in = self.n_feat
        for _ in range(self.n_hidden):
            shapes.append((self.width, fan_in))
            fan_in = self.width
        shapes.append((self.n_out, self.width))
        return shapes

    def param_count(self) -> int:
        return sum(o * i + o for o, i in self.layer_shapes())

    def offsets(self):
        """[(w_off, b_off, out, in)] for each layer, head last."""
        res, off = [], 0
        for o, i in self.layer_shapes():
            res.append((off, off + o * i, o, i))
            off += o * i + o
        return res


@dataclasses.dataclass(frozen=True)
class HashDesc:
    """Shape of the hash-grid field (Sec. III-D): a multiresolution hash encoding of the
    origin, a sinusoidal code of the direction, and a small ReLU MLP."""
    n_levels: int = 16
    n_feat: int = 2          # features per level
    log2_table: int = 19     # entries per level (at most)
    base_res: int = 16       # resolution of the coarsest level
    growth: float = 1.5      # resolution factor between levels
    dir_bands: int = 4
    width: int = 64
    n_hidden: int = 2
    n_out: int = 2
    box_half: float = BOX_HALF


HASH_PAPER = HashDesc()                                   # the paper's 52 MB field
HASH_SMALL = HashDesc(n_levels=6, log2_table=12, base_res=4, growth=2.0, width=64)   # tests: dense and hashed levels


def hash_params(desc: HashDesc, n_entries: int, seed: int, table_std: float = 1e-4) -> np.ndarray:
    """Flat float32 parameters of a hash-grid field: the table ([n_entries][n_feat],
    N(0, table_std), level after level) then the MLP (He-normal weights, N(0, 0.1) biases,
    heads N(0, 1/fan_in)).  n_entries comes from the caller (the library's or the oracle's
    level layout); the MLP input width is n_levels n_feat + 3 (1 + 2 dir_bands)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.standard_normal(n_entries * desc.n_feat) * table_std]
    fan_in = desc.n_levels * desc.n_feat + 3 * (1 + 2 * desc.dir_bands)
    for layer in range(desc.n_hidden + 1):
        out = desc.width if layer < desc.n_hidden else desc.n_out
        std = math.sqrt(2.0 / fan_in) if layer < desc.n_hidden else math.sqrt(1.0 / fan_in)
        parts.append(rng.standard_normal(out * fan_in) * std)
        parts.append(rng.standard_normal(out) * 0.1)
        fan_in = out
    return np.concatenate(parts).astype(np.float32)


# Workload nets.
NET_TINY = NetDesc(6, 4, 4, 128, 2)        # 54 -> 128 x4 -> 2
NET_FULL = NetDesc(6, 10, 12, 1024, 2)     # 126 -> 1024 x12 -> 2 (46.7 MB fp32)
NET_LARGE = NetDesc(6, 10, 16, 1024, 2)    # 126 -> 1024 x16 -> 2
NET_SDF = NetDesc(3, 10, 12, 1024, 1)      # 63 -> 1024 x12 -> 1


def split_params(desc: NetDesc, params: np.ndarray):
    """View a flat parameter vector as [(W, b)] per layer, head last."""
    out = []
    for w_off, b_off, o, i in desc.offsets():
        out.append((params[w_off:w_off + o * i].reshape(o, i), params[b_off:b_off + o]))
    return out


def he_init(desc: NetDesc, seed: int) -> np.ndarray:
    """He-normal hidden weights N(0, 2/fan_in), head weights N(0, 1/fan_in), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    shapes = desc.layer_shapes()
    for li, (o, i) in enumerate(shapes):
        std = math.sqrt((1.0 if li == len(shapes) - 1 else 2.0) / i)
        parts.append(rng.standard_normal(o * i) * std)
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def test_params(desc: NetDesc, seed: int, bias_std: float = 0.1) -> np.ndarray:
    """He-init weights plus non-zero random biases (parity tests must see biases)."""
    p = he_init(desc, seed).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    for _, b_off, o, _ in desc.offsets():
        p[b_off:b_off + o] = rng.standard_normal(o) * bias_std
    return p.astype(np.float32)


# ----------------------------------------------------------------------------
# Scenes: unions of spheres and ellipsoids.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    """centers [P,3], axes [P,3] (semi-axes, equal for a sphere), rot [P,3,3].

    A primitive is the set {c + R (a * u) : |u| <= 1}; R maps local to world.
    """
    centers: np.ndarray
    axes: np.ndarray
    rot: np.ndarray

    @property
    def n(self) -> int:
        return len(self.centers)


def _random_rotations(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z); r[:, 0, 1] = 2 * (x * y - z * w); r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w); r[:, 1, 1] = 1 - 2 * (x * x + z * z); r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w); r[:, 2, 1] = 2 * (y * z + x * w); r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def scene_spheres(n: int, seed: int, rmin=0.05, rmax=0.3) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(-1.0, 1.0, (n, 3))
    r = rng.uniform(rmin, rmax, n)
    return Scene(c, np.repeat(r[:, None], 3, axis=1), np.repeat(np.eye(3)[None], n, axis=0))


def scene_ellipsoids(n: int, seed: int, amin=0.02, amax=0.25) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(-1.0, 1.0, (n, 3))
    a = rng.uniform(amin, amax, (n, 3))
    return Scene(c, a, _random_rotations(rng, n))


def scene_mixed(n: int, seed: int) -> Scene:
    """Each primitive a sphere (r ~ U[0.05,0.3]) or an ellipsoid (axes ~ U[0.02,0.25]) with p=1/2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(-1.0, 1.0, (n, 3))
    is_sphere = rng.uniform(size=n) < 0.5
    r = rng.uniform(0.05, 0.3, n)
    a = rng.uniform(0.02, 0.25, (n, 3))
    axes = np.where(is_sphere[:, None], r[:, None], a)
    rots = _random_rotations(rng, n)
    rots[is_sphere] = np.eye(3)
    return Scene(c, axes, rots)


def _inside_any(scene: Scene, p: np.ndarray, exclude=None) -> np.ndarray:
    """Point-in-primitive test (scene sampling only: used to reject samples).

    A k-d tree over the points limits each primitive's exact test to the points
    inside its bounding ball."""
    from scipy.spatial import cKDTree
    inside = np.zeros(len(p), dtype=bool)
    tree = cKDTree(p)
    for k in range(scene.n):
        idx = np.asarray(tree.query_ball_point(scene.centers[k], float(scene.axes[k].max()) * 1.0001),
                         dtype=np.int64)
        if idx.size == 0:
            continue
        loc = ((p[idx] - scene.centers[k]) @ scene.rot[k]) / scene.axes[k]
        q = np.einsum('ni,ni->n', loc, loc) < 1.0
        if exclude is not None:
            q &= exclude[idx] != k
        inside[idx[q]] = True
    return inside


def _inside_other(scene: Scene, p: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Is the point p[i], drawn on the surface of primitive k[i], inside another primitive?

    The same test as _inside_any(scene, p, exclude=k), organised per primitive: a point of
    primitive a can only lie inside a primitive j whose bounding ball meets a's, so each
    primitive's points are tested against those neighbours alone."""
    inside = np.zeros(len(p), dtype=bool)
    rad = scene.axes.max(axis=1) * 1.0001
    dist = np.linalg.norm(scene.centers[:, None, :] - scene.centers[None, :, :], axis=2)
    order = np.argsort(k, kind="stable")
    bounds = np.searchsorted(k[order], np.arange(scene.n + 1))
    for a in range(scene.n):
        idx = order[bounds[a]:bounds[a + 1]]
        if idx.size == 0:
            continue
        pa = p[idx]
        for j in np.nonzero(dist[a] <= rad[a] + rad)[0]:
            if j == a:
                continue
            loc = ((pa - scene.centers[j]) @ scene.rot[j]) / scene.axes[j]
            inside[idx[np.einsum('ni,ni->n', loc, loc) < 1.0]] = True
    return inside


def _unit_sphere_dirs(rng, n):
    z = 1.0 - 2.0 * rng.uniform(size=n)
    phi = 2.0 * np.pi * rng.uniform(size=n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def _soa(o, d) -> np.ndarray:
    """Pack origins and directions (float64) into the float32 [6, N] SoA layout.

    Directions are normalised in float64 before rounding to float32."""
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    return np.ascontiguousarray(np.concatenate([o, d], axis=1).T.astype(np.float32))


def free_rays(scene: Scene, n: int, seed: int) -> np.ndarray:
    """Origins uniform in the object box (outside every primitive), directions uniform on S^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((0, 3))
    while len(out) < n:
        cand = rng.uniform(-BOX_HALF, BOX_HALF, (max(2 * (n - len(out)), 64), 3))
        cand = cand[~_inside_any(scene, cand)]
        out = np.concatenate([out, cand])
    o = out[:n]
    return _soa(o, _unit_sphere_dirs(rng, n))


def surface_points(scene: Scene, n: int, seed: int):
    """Points on the visible union surface with outward unit normals.

    p = c + R (a * u), u uniform on S^2 for a uniformly chosen primitive; the
    normal is R (u / a) normalised.  Points inside another primitive are
    rejected.  The density is uniform in u per primitive, not in area."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ps, ns = [], []
    have = 0
    while have < n:
        m = max(2 * (n - have), 64)
        k = rng.integers(0, scene.n, m)
        u = _unit_sphere_dirs(rng, m)
        R = scene.rot[k]; a = scene.axes[k]
        p = scene.centers[k] + np.einsum('mij,mj->mi', R, a * u)
        nrm = np.einsum('mij,mj->mi', R, u / a)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        keep = ~_inside_other(scene, p, k)
        ps.append(p[keep]); ns.append(nrm[keep]); have += int(keep.sum())
    return np.concatenate(ps)[:n], np.concatenate(ns)[:n]


def shadow_rays(scene: Scene, n: int, seed: int, light=LIGHT_POS, offset=NORMAL_OFFSET) -> np.ndarray:
    """Surface point lifted by `offset` (default NORMAL_OFFSET) along its normal, pointing at
    the light."""
    p, nrm = surface_points(scene, n, seed)
    o = p + offset * nrm
    return _soa(o, np.asarray(light)[None] - o)


def _basis(nrm):
    """Branchless orthonormal basis (t, b) around unit n (Duff et al. 2017)."""
    sign = np.where(nrm[:, 2] >= 0, 1.0, -1.0)
    a = -1.0 / (sign + nrm[:, 2])
    b = nrm[:, 0] * nrm[:, 1] * a
    t = np.stack([1 + sign * nrm[:, 0] ** 2 * a, sign * b, -sign * nrm[:, 0]], axis=1)
    bb = np.stack([b, sign + nrm[:, 1] ** 2 * a, -nrm[:, 1]], axis=1)
    return t, bb


def ao_rays(scene: Scene, n_points: int, n_dirs: int, seed: int) -> np.ndarray:
    """n_points surface points x n_dirs cosine-weighted hemisphere rays (Malley), point-major."""
    p, nrm = surface_points(scene, n_points, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    u1 = rng.uniform(size=(n_points, n_dirs)); u2 = rng.uniform(size=(n_points, n_dirs))
    r = np.sqrt(u1); phi = 2 * np.pi * u2
    lx, ly, lz = r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1 - u1))
    t, b = _basis(nrm)
    d = lx[..., None] * t[:, None] + ly[..., None] * b[:, None] + lz[..., None] * nrm[:, None]
    o = np.repeat((p + NORMAL_OFFSET * nrm)[:, None], n_dirs, axis=1)
    return _soa(o.reshape(-1, 3), d.reshape(-1, 3))


def gi_rays(scene: Scene, n: int, seed: int) -> np.ndarray:
    """One-bounce rays: surface points, directions uniform over the normal's hemisphere."""
    p, nrm = surface_points(scene, n, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    d = _unit_sphere_dirs(rng, n)
    d = np.where((np.sum(d * nrm, axis=1) < 0)[:, None], -d, d)
    return _soa(p + NORMAL_OFFSET * nrm, d)


def surface_anchored_rays(scene: Scene, n: int, seed: int) -> np.ndarray:
    """Surface points (lifted) with directions uniform on the full sphere."""
    p, nrm = surface_points(scene, n, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return _soa(p + NORMAL_OFFSET * nrm, _unit_sphere_dirs(rng, n))


def train_rays(scene: Scene, n: int, seed: int) -> np.ndarray:
    """Training batch: half surface-anchored rays, half free-space rays, interleaved."""
    h = n // 2
    a = surface_anchored_rays(scene, h, seed)
    b = free_rays(scene, n - h, seed + 500)
    out = np.empty((6, n), dtype=np.float32)
    out[:, 0:2 * h:2] = a
    out[:, 1:2 * h:2] = b[:, :h]
    out[:, 2 * h:] = b[:, h:]
    return out


def mixed_rays(scene: Scene, n: int, seed: int) -> np.ndarray:
    """Large mixed workload: 50% shadow, 40% AO (32 per point), 10% GI, fixed seeded interleave."""
    n_sh = n // 2
    n_ao_pts = max(1, int(round(0.4 * n)) // 32)
    n_ao = n_ao_pts * 32
    n_gi = n - n_sh - n_ao
    parts = [shadow_rays(scene, n_sh, seed), ao_rays(scene, n_ao_pts, 32, seed + 10),
             gi_rays(scene, n_gi, seed + 20)]
    allr = np.concatenate(parts, axis=1)
    perm = np.random.Generator(np.random.PCG64(seed + 30)).permutation(n)
    return np.ascontiguousarray(allr[:, perm])


def uniforms(rows: int, n: int, seed: int) -> np.ndarray:
    """float32 [rows][n] uniform draws in [0, 1) (e.g. the selection, start index and shift
    of the self-consistency points of a training batch)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.random((rows, n)).astype(np.float32))


def sdf_train_points(scene: Scene, n: int, seed: int, sigma: float = 0.05) -> np.ndarray:
    """SDF fitting samples, float32 [3, N]: half uniform in the box, half surface points
    displaced by isotropic N(0, sigma^2) noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = n // 2
    u = rng.uniform(-BOX_HALF, BOX_HALF, (h, 3))
    p, _ = surface_points(scene, n - h, seed + 1)
    p = p + rng.standard_normal(p.shape) * sigma
    return np.ascontiguousarray(np.concatenate([u, p]).T.astype(np.float32))


def sdf_fit_points(scene: Scene, n: int, seed: int) -> np.ndarray:
    """SDF fitting samples with a tighter band at the surface, float32 [3, N]: half uniform in
    the box, a quarter displaced from the surface by N(0, 0.05^2), a quarter by N(0, 0.005^2)."""
    h = n // 2
    a = sdf_train_points(scene, h, seed, sigma=0.05)
    b = sdf_train_points(scene, n - h, seed + 5000, sigma=0.005)
    return np.ascontiguousarray(np.concatenate([a, b], axis=1))


def sdf_points(n: int, seed: int) -> np.ndarray:
    """Points uniform in the object box as float32 [3, N] (SDF fitting inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.uniform(-BOX_HALF, BOX_HALF, (3, n)).astype(np.float32))


def planted_box_sdf(desc, half, seed, bias=1.0, noise=0.05):
    """SDF MLP (n_in = 3, n_out = 1, n_hidden >= 5) that computes max_i(|p_i| - half_i) exactly.

    The first 14 neurons of each layer carry the computation through ReLUs; every other
    neuron gets random weights and biases (so the products are dense) but feeds nothing
    the planted path reads.  The value is a lower bound of the distance to the box
    [-half, half] outside it, so it is a valid function to sphere trace."""
    assert desc.n_in == 3 and desc.n_out == 1 and desc.n_hidden >= 5
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal(desc.param_count()) * noise
    views = split_params(desc, p)
    B = bias
    # layer 1: relu(+p_i), relu(-p_i)
    W, b = views[0]
    W[:14, :] = 0.0; b[:14] = 0.0
    for i in range(3):
        W[2 * i, i] = 1.0; W[2 * i + 1, i] = -1.0
    # layer 2: u_i = relu(|p_i| - half_i + B)
    W, b = views[1]
    W[:14, :] = 0.0; b[:14] = 0.0
    for i in range(3):
        W[i, 2 * i] = 1.0; W[i, 2 * i + 1] = 1.0; b[i] = B - half[i]
    # layer 3: m = relu(u_y - u_x), pass u_x, u_z
    W, b = views[2]
    W[:14, :] = 0.0; b[:14] = 0.0
    W[0, 1] = 1.0; W[0, 0] = -1.0
    W[1, 0] = 1.0
    W[2, 2] = 1.0
    # layer 4: v = u_x + m = max(u_x, u_y); pass u_z
    W, b = views[3]
    W[:14, :] = 0.0; b[:14] = 0.0
    W[0, 0] = 1.0; W[0, 1] = 1.0
    W[1, 2] = 1.0
    # layer 5: w = relu(u_z - v), pass v
    W, b = views[4]
    W[:14, :] = 0.0; b[:14] = 0.0
    W[0, 1] = 1.0; W[0, 0] = -1.0
    W[1, 0] = 1.0
    # layers 6..n: s + B = v + w in neuron 0, passed through
    for l in range(5, desc.n_hidden):
        W, b = views[l]
        W[:14, :] = 0.0; b[:14] = 0.0
        if l == 5:
            W[0, 0] = 1.0; W[0, 1] = 1.0
        else:
            W[0, 0] = 1.0
    Wh, bh = views[-1]
    Wh[:] = 0.0
    if desc.n_hidden == 5:
        Wh[0, 0] = 1.0; Wh[0, 1] = 1.0
    else:
        Wh[0, 0] = 1.0
    bh[0] = -B
    return p.astype(np.float32)


# ---- the shading workload: a ground slab with objects above it, a camera and a light

@dataclasses.dataclass(frozen=True)
class View:
    """Pinhole camera: eye, look-at target, up hint, vertical field of view (radians), size."""
    eye: tuple = (0.0, 1.6, 3.2)
    target: tuple = (0.0, -0.5, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    fov_y: float = math.radians(45.0)
    width: int = 512
    height: int = 512


SHADE_LIGHT = (1.2, 2.8, 0.8)   # point light of the shading workload (outside the box)
SKY = (0.2, 1.0)                # sky radiance at the nadir and the zenith (one-bounce term)
RADIANCE_RES = 32               # vertices per axis of the surface-radiance grid
AO_RAYS = 16                    # AO rays per pixel of the shading workload


def scene_ground(n: int, seed: int) -> Scene:
    """A flat ground slab (top face at y = -1) under n spheres and ellipsoids (sizes as in
    scene_mixed) whose centres lie in [-1, 1] x [-0.8, 0.9] x [-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.concatenate([[[0.0, -1.02, 0.0]],
                        np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.9, n), rng.uniform(-1, 1, n)], 1)])
    is_sphere = rng.uniform(size=n) < 0.5
    r = rng.uniform(0.08, 0.3, n)
    a = rng.uniform(0.05, 0.25, (n, 3))
    axes = np.concatenate([[[1.45, 0.02, 1.45]], np.where(is_sphere[:, None], r[:, None], a)])
    rots = _random_rotations(rng, n)
    rots[is_sphere] = np.eye(3)
    return Scene(c, axes, np.concatenate([np.eye(3)[None], rots]))


def scene_object(n: int, seed: int) -> Scene:
    """One compound object on the ground slab of scene_ground: n spheres and ellipsoids
    (axes 0.15 .. 0.45) whose centres lie within 0.45 of (0, -0.45, 0), the way the paper's
    fields each hold one normalised object."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.array([0.0, -0.45, 0.0]) + rng.uniform(-0.45, 0.45, (n, 3))
    a = rng.uniform(0.15, 0.45, (n, 3))
    rots = _random_rotations(rng, n)
    return Scene(np.concatenate([[[0.0, -1.02, 0.0]], c]), np.concatenate([[[1.45, 0.02, 1.45]], a]),
                 np.concatenate([np.eye(3)[None], rots]))


def radiance_grid(res: int, seed: int) -> np.ndarray:
    """A smooth surface-radiance field in [0.1, 0.9] sampled at the vertices of a res^3 grid
    over the object box, float32 [res (z)][res (y)][res (x)]: the mean of four random plane
    waves of 1-3 periods across the box (a stand-in for the captured appearance)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.linspace(-BOX_HALF, BOX_HALF, res)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([x, y, z], axis=-1)
    acc = np.zeros(pts.shape[:-1])
    for _ in range(4):
        k = rng.standard_normal(3)
        k *= rng.uniform(1.0, 3.0) * 2 * np.pi / (2 * BOX_HALF) / np.linalg.norm(k)
        acc += np.cos(pts @ k + rng.uniform(0, 2 * np.pi))
    return np.ascontiguousarray((0.5 + 0.1 * acc).astype(np.float32))

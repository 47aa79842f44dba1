"""Seeded synthetic point clouds for the octree builds.

This module is shared by the CPU oracle's tests and the GPU path. It holds
no part of the method's arithmetic (no quantization, no Morton keys, no
sorting): it only draws FP32 coordinates in [0, 1)^3.

Random source: splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014). The i-th output of stream
``seed`` is mix(seed + (i + 1) * GAMMA) with the published mixing constants,
computed in wrapping uint64 numpy arithmetic, so a stream is counter-based
and any slice of it can be drawn independently.

Workloads follow the paper's synthetic distributions: uniform points in the
unit cube (Section 4.1, Table "dsTime") and points on a sphere surface
(Section 4.1, sphere experiment), plus Gaussian clusters for the nonuniform,
batched and serving workloads. All coordinates are clamped into
[0, 1 - 2^-24], which is exactly representable in FP32, so every point lies
in the half-open unit cube the paper assumes (Section 1.4).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
ONE_MINUS_ULP = np.float64(1.0 - 2.0 ** -24)
_MASK = (1 << 64) - 1

# Stream tags keep the draws of one workload independent of each other.
TAG_POINTS = 0x01
TAG_SPHERE = 0x02
TAG_CLUSTER_LABEL = 0x03
TAG_CLUSTER_NOISE = 0x04
TAG_CENTRES = 0x05
TAG_SIZES = 0x06
TAG_STEP = 0x07
TAG_ARRIVAL = 0x08
TAG_PICK = 0x09
TAG_MOVE = 0x0A


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _mix_int(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def stream_seed(*parts: int) -> int:
    """Derive a 64-bit stream seed from integers (seed, tag, index, ...):
    s <- mix(s xor (part + GAMMA)) for each part, from s = 0x243F6A8885A308D3,
    in wrapping 64-bit arithmetic (plain Python integers, masked)."""
    s = 0x243F6A8885A308D3
    for p in parts:
        s = _mix_int(s ^ (((p & _MASK) + 0x9E3779B97F4A7C15) & _MASK))
    return s


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+count-1 of the splitmix64 stream ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA)


def uniform24(seed: int, count: int) -> np.ndarray:
    """FP32 uniforms (u >> 40) * 2^-24: exactly representable, in [0, 1)."""
    u = splitmix64(seed, count) >> np.uint64(40)
    return (u.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def uniform53(seed: int, count: int, start: int = 0) -> np.ndarray:
    """FP64 uniforms (u >> 11) * 2^-53 in [0, 1)."""
    u = splitmix64(seed, count, start) >> np.uint64(11)
    return u.astype(np.float64) * 2.0 ** -53


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by the Box-Muller transform, in FP64."""
    m = (count + 1) // 2
    u = uniform53(seed, 2 * m)
    u1 = 1.0 - u[0::2]          # (0, 1]: keeps log finite
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m, dtype=np.float64)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:count]


def _to_cube_f32(p: np.ndarray) -> np.ndarray:
    p = np.clip(p, 0.0, ONE_MINUS_ULP)
    return np.ascontiguousarray(p.astype(np.float32))


def uniform_points(seed: int, n: int) -> np.ndarray:
    """n points uniform in [0,1)^3, FP32 [n, 3]; coordinate j of point i is
    draw 3i + j of the stream."""
    return uniform24(stream_seed(seed, TAG_POINTS), 3 * n).reshape(n, 3)


def sphere_points(seed: int, n: int) -> np.ndarray:
    """n points on the sphere of radius 0.5 centred at (0.5, 0.5, 0.5): the
    unit sphere scaled into the unit cube. Directions are normalized
    Gaussian triples."""
    g = normal(stream_seed(seed, TAG_SPHERE), 3 * n).reshape(n, 3)
    nrm = np.sqrt((g * g).sum(axis=1, keepdims=True))
    nrm[nrm == 0.0] = 1.0
    return _to_cube_f32(0.5 + 0.5 * g / nrm)


def cluster_centres(geometry_seed: int, k: int = 64) -> np.ndarray:
    """k cluster centres uniform in [0,1)^3 (FP64)."""
    return uniform53(stream_seed(geometry_seed, TAG_CENTRES), 3 * k).reshape(k, 3)


def cluster_points(seed: int, n: int, centres: np.ndarray,
                   sigma: float = 0.01) -> np.ndarray:
    """n points from isotropic Gaussian clusters: a label uniform over the
    centres, then centre + sigma * N(0, 1) per coordinate, clamped."""
    k = centres.shape[0]
    lab = splitmix64(stream_seed(seed, TAG_CLUSTER_LABEL), n) % np.uint64(k)
    g = normal(stream_seed(seed, TAG_CLUSTER_NOISE), 3 * n).reshape(n, 3)
    return _to_cube_f32(centres[lab.astype(np.int64)] + sigma * g)


def sphere_cluster_points(seed: int, geometry_seed: int, n: int) -> np.ndarray:
    """The nonuniform workload: the first n//2 points on the sphere, the rest
    from 64 Gaussian clusters (sigma 0.01) whose centres come from
    ``geometry_seed`` and are shared by every set built on that geometry."""
    h = n // 2
    c = cluster_centres(geometry_seed, 64)
    return np.ascontiguousarray(np.concatenate(
        [sphere_points(seed, h), cluster_points(seed, n - h, c, 0.01)], axis=0))


def moved_points(points: np.ndarray, seed: int, sigma: float) -> np.ndarray:
    """The points one time step later: each coordinate moved by
    sigma * N(0, 1) (draw 3i + j for coordinate j of point i), in FP64, then
    clamped into the cube and rounded to FP32."""
    g = normal(stream_seed(seed, TAG_MOVE), points.size).reshape(points.shape)
    return _to_cube_f32(points.astype(np.float64) + sigma * g)


def full_grid_points(level: int) -> np.ndarray:
    """One point at the centre of every box of the level-``level`` grid,
    (i + 0.5) / 2^level per axis, in x-fastest order. Every box is nonempty."""
    m = 1 << level
    ax = ((np.arange(m, dtype=np.float64) + 0.5) / m).astype(np.float32)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def level_for_size(n: int, per_leaf: int = 64, lo: int = 2) -> int:
    """Smallest L >= lo with per_leaf * 8^L >= n (ceil(log8(n / per_leaf)))."""
    L = lo
    while per_leaf * (8 ** L) < n:
        L += 1
    return L


def config_plain_small(seed: int = 1):
    """65,536 uniform points shared by sources and receivers; max level 5,
    32-bit keys, fixed depth."""
    return dict(name="uniform-65536-shared-L5-u32", src=uniform_points(seed, 65536),
                recv=None, key_bits=32, cluster_s=0, max_level=5)


def config_plain_uniform(n: int = 1 << 24, src_seed: int = 2, recv_seed: int = 3,
                         max_level: int = 8):
    """Separate uniform source and receiver sets of n points each; max level
    8, 64-bit keys, fixed depth."""
    return dict(name=f"uniform-{n}x2-L{max_level}-u64", src=uniform_points(src_seed, n),
                recv=uniform_points(recv_seed, n), key_bits=64, cluster_s=0,
                max_level=max_level)


def config_plain_nonuniform(n: int = 1 << 24, geometry_seed: int = 4, src_seed: int = 5,
                            recv_seed: int = 6, max_level: int = 10, cluster_s: int = 64):
    """Separate nonuniform sets (half sphere surface, half 64 Gaussian
    clusters) of n points each; max level 10, cluster size 64, 64-bit keys."""
    return dict(name=f"sphere+clusters-{n}x2-L{max_level}-s{cluster_s}-u64",
                src=sphere_cluster_points(src_seed, geometry_seed, n),
                recv=sphere_cluster_points(recv_seed, geometry_seed, n),
                key_bits=64, cluster_s=cluster_s, max_level=max_level)


def batch_sizes(n_sets: int = 512, seed: int = 7, lo_log2: int = 10, hi_log2: int = 20):
    """Log-uniform set sizes floor(2^(lo + (hi - lo) U)), clipped to
    [2^lo, 2^hi]."""
    u = uniform53(stream_seed(seed, TAG_SIZES), n_sets)
    n = np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    return np.clip(n, 1 << lo_log2, 1 << hi_log2)


def batch_sets(n_sets: int = 512, seed: int = 7, lo_log2: int = 10, hi_log2: int = 20):
    """The batched workload: n_sets independent shared point sets; even sets
    uniform, odd sets 64-cluster Gaussian (sigma 0.01, own centres).
    Returns (xyz concatenated [sum n, 3], offsets [n_sets + 1] uint64,
    levels [n_sets] uint8 with level = ceil(log8(n / 64)), at least 2)."""
    sizes = batch_sizes(n_sets, seed, lo_log2, hi_log2)
    parts, levels = [], []
    for i, n in enumerate(sizes):
        s = stream_seed(seed, 0x100 + i)
        if i % 2 == 0:
            parts.append(uniform_points(s, int(n)))
        else:
            parts.append(cluster_points(s, int(n), cluster_centres(s, 64), 0.01))
        levels.append(level_for_size(int(n)))
    off = np.zeros(n_sets + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes).astype(np.uint64)
    return (np.ascontiguousarray(np.concatenate(parts, axis=0)), off,
            np.asarray(levels, dtype=np.uint8))


def serving_systems(n_systems: int = 64, seed: int = 8, lo_log2: int = 14, hi_log2: int = 22):
    """Particle systems of the serving workload: sizes floor(2^(lo + (hi - lo) U)),
    64 Gaussian clusters each (sigma 0.01, own centres), level
    ceil(log8(n / 64)). Returns (list of FP32 [n, 3] arrays, levels)."""
    u = uniform53(stream_seed(seed, TAG_SIZES), n_systems)
    sizes = np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    pts, levels = [], []
    for i, n in enumerate(sizes):
        s = stream_seed(seed, 0x200 + i)
        pts.append(cluster_points(s, int(n), cluster_centres(s, 64), 0.01))
        levels.append(level_for_size(int(n)))
    return pts, levels


def poisson_trace(n_requests: int, rate: float, n_systems: int, seed: int = 8):
    """Arrival times (seconds, from 0) of a Poisson process of the given rate
    and the system each request rebuilds (uniform)."""
    u = uniform53(stream_seed(seed, TAG_ARRIVAL), n_requests)
    gaps = -np.log(1.0 - u) / rate
    pick = splitmix64(stream_seed(seed, TAG_PICK), n_requests) % np.uint64(n_systems)
    return np.cumsum(gaps), pick.astype(np.int64)


def displacement_seed(seed: int, system: int, step: int) -> int:
    """Seed of the N(0, sigma^2) displacement of one system at one step."""
    return stream_seed(seed, TAG_STEP, system, step) & 0x7FFFFFFFFFFFFFFF

"""Seeded synthetic scenes: the inputs both the rasterizer and its CPU checker consume.

This module only *makes data*: vertex positions, index buffers, instance matrices, per-vertex
attributes and cameras.  It contains none of the rasterization arithmetic (projection of vertices,
snapping, coverage, depth, keys); a camera here is just the 4x4 matrix handed to the rasterizer.

The scenes stand in for the paper's evaluation data (Table 1: Sponza, Lantern, Komainu, Venice,
Zorah), which are not available.  Each one reproduces a shape class the paper measures:
dense photogrammetry-like height fields with mostly sub-pixel triangles (Komainu/Venice/Zorah),
one dense mesh instanced thousands of times (Lantern Instances, Sec. 4.5), and a low-poly scene
with huge near-plane-crossing triangles (Sponza-like, exercising stages 2 and 3).

Noise: fBm value noise, lattice values uniform in [-1, 1) drawn from SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) of (seed, octave, i, j),
smoothstep-interpolated, 8 octaves, base frequency 8 cells, lacunarity 2, gain 0.5, normalised by
the sum of the octave gains.  All noise is evaluated in float64 and stored as float32.

The camera follows the paper's projection (Sec. 4.1, Eqs. 1-2): view space looks down -z,
x and y are scaled by f/aspect and f with f = 1/tan(fovy/2), and the homogeneous w is the
positive linear view depth.  Row 2 (clip z) of the matrix is not used by the rasterizer.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Mesh", "View", "Scene", "splitmix64", "fbm2_grid", "fbm2_points", "heightfield",
    "uv_sphere", "camera", "orbit_camera", "random_rotations", "instance_matrices",
    "scene_c1", "scene_c2", "scene_c3", "scene_c4", "scene_c5", "scene_by_name",
    "random_tiny_scene", "CHUNK_TRIS",
]

CHUNK_TRIS = 65536          # triangle-chunk size of the seeded index shuffle
NEAR = 0.01                 # near plane of every synthetic camera (scene units)
FOVY_DEG = 60.0

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------------------------
# Data containers
# --------------------------------------------------------------------------------------------
@dataclass
class Mesh:
    pos: np.ndarray                       # float32 [V, 3]
    idx: np.ndarray                       # uint32 [T, 3]
    inst: Optional[np.ndarray] = None     # float32 [N, 12] row-major 3x4 object->world, None = identity
    attrs: Optional[np.ndarray] = None    # float32 [V, C]
    bsphere: Optional[np.ndarray] = None  # float32 [4] object-space bounding sphere (cx, cy, cz, r)

    @property
    def num_instances(self) -> int:
        return 1 if self.inst is None else int(self.inst.shape[0])

    @property
    def num_triangles(self) -> int:
        return int(self.idx.shape[0])


@dataclass
class View:
    vp: np.ndarray        # float32 [4, 4] row-major view-projection (row 3 = positive view depth)
    near: float
    width: int
    height: int


@dataclass
class Scene:
    name: str
    meshes: List[Mesh]
    views: List[View]
    meta: dict = field(default_factory=dict)

    @property
    def total_tri_instances(self) -> int:
        return sum(m.num_triangles * m.num_instances for m in self.meshes)


# --------------------------------------------------------------------------------------------
# SplitMix64 and value noise
# --------------------------------------------------------------------------------------------
def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to a uint64 array (wrapping arithmetic)."""
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & _M64
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
    return z ^ (z >> np.uint64(31))


def _lattice(seed: int, octave: int, rows: int, cols: int) -> np.ndarray:
    """float64 [rows, cols] lattice values uniform in [-1, 1) from SplitMix64(seed, octave, i, j)."""
    with np.errstate(over="ignore"):
        k = splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(octave))
        i = np.arange(rows, dtype=np.uint64)[:, None]
        j = np.arange(cols, dtype=np.uint64)[None, :]
        h = splitmix64(splitmix64(k + i) + j)
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


def _axis_weights(t: np.ndarray, freq: int):
    """Cell index and smoothstep weight of coordinates t in [0, 1] on a lattice of `freq` cells."""
    s = t * freq
    i = np.minimum(np.floor(s), freq - 1).astype(np.int64)
    f = s - i
    w = f * f * (3.0 - 2.0 * f)
    return i, w


def _octaves(octaves: int, base: int, gain: float):
    gains = [gain ** o for o in range(octaves)]
    norm = sum(gains)
    return [(base * (2 ** o), gains[o] / norm) for o in range(octaves)]


def fbm2_grid(n: int, seed: int, octaves: int = 8, base: int = 8, gain: float = 0.5,
              out: Optional[np.ndarray] = None, row_chunk: int = 512) -> np.ndarray:
    """fBm on the n x n vertex grid (u = col/(n-1), v = row/(n-1)); returns float64 [n, n]
    (or writes float32 into `out` with the same shape).  Evaluated separably per octave:
    interpolate every lattice row along u, then interpolate those rows along v."""
    u = np.arange(n, dtype=np.float64) / float(n - 1)
    per_oct = []
    for o, (freq, g) in enumerate(_octaves(octaves, base, gain)):
        lat = _lattice(seed, o, freq + 1, freq + 1)          # [v-lattice, u-lattice]
        iu, wu = _axis_weights(u, freq)
        a = lat[:, iu] * (1.0 - wu) + lat[:, iu + 1] * wu     # [freq+1, n]
        iv, wv = _axis_weights(u, freq)
        per_oct.append((a, iv, wv, g))
    res = out if out is not None else np.empty((n, n), dtype=np.float64)

    def work(r0):
        r1 = min(n, r0 + row_chunk)
        acc = np.zeros((r1 - r0, n), dtype=np.float64)
        for a, iv, wv, g in per_oct:
            iv_c = iv[r0:r1]
            wv_c = wv[r0:r1, None]
            acc += g * (a[iv_c] * (1.0 - wv_c) + a[iv_c + 1] * wv_c)
        res[r0:r1] = acc
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(0, n, row_chunk)))
    return res


def fbm2_points(u: np.ndarray, v: np.ndarray, seed: int, octaves: int = 8, base: int = 8,
                gain: float = 0.5, wrap_u: bool = False) -> np.ndarray:
    """Pointwise fBm at (u, v) in [0, 1]^2 (float64), same lattice as `fbm2_grid`.
    wrap_u=True makes the last lattice column equal the first (periodic in u)."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    acc = np.zeros(np.broadcast(u, v).shape, np.float64)
    for o, (freq, g) in enumerate(_octaves(octaves, base, gain)):
        lat = _lattice(seed, o, freq + 1, freq + 1)
        if wrap_u:
            lat[:, freq] = lat[:, 0]
        iu, wu = _axis_weights(u, freq)
        iv, wv = _axis_weights(v, freq)
        top = lat[iv, iu] * (1.0 - wu) + lat[iv, iu + 1] * wu
        bot = lat[iv + 1, iu] * (1.0 - wu) + lat[iv + 1, iu + 1] * wu
        acc += g * (top * (1.0 - wv) + bot * wv)
    return acc


# --------------------------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------------------------
def _shuffle_chunks(tri_fn, T: int, seed: int, chunk: int = CHUNK_TRIS) -> np.ndarray:
    """Index buffer whose 64K-triangle chunks appear in a seeded random order.
    tri_fn(t0, t1) returns the uint32 [t1-t0, 3] triangles of the unshuffled order."""
    nch = (T + chunk - 1) // chunk
    perm = np.random.default_rng(seed).permutation(nch)
    sizes = np.array([min(chunk, T - c * chunk) for c in perm], dtype=np.int64)
    dst = np.concatenate([[0], np.cumsum(sizes)])
    idx = np.empty((T, 3), dtype=np.uint32)

    def work(k):
        c = int(perm[k])
        t0 = c * chunk
        t1 = min(T, t0 + chunk)
        idx[dst[k]:dst[k + 1]] = tri_fn(t0, t1)
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nch)))
    return idx


def heightfield(n: int, amplitude: float, seed: int, shuffle: bool = True):
    """n x n vertex grid over [0,1]^2 in (x, z) with height y = amplitude * fBm.
    Vertex (row r, col c) has index r*n + c, x = c/(n-1), z = r/(n-1).  Quad (r, c) in row-major
    order gives the two up-facing (counter-clockwise seen from +y) triangles
    (v00, v01, v10) and (v10, v01, v11).  Returns (pos f32 [n*n, 3], idx u32 [2(n-1)^2, 3])."""
    V = n * n
    pos = np.empty((n, n, 3), dtype=np.float32)
    coord = (np.arange(n, dtype=np.float64) / float(n - 1)).astype(np.float32)
    pos[:, :, 0] = coord[None, :]
    pos[:, :, 2] = coord[:, None]
    h = fbm2_grid(n, seed)
    h *= amplitude
    pos[:, :, 1] = h.astype(np.float32)
    del h
    pos = pos.reshape(V, 3)
    T = 2 * (n - 1) * (n - 1)

    def tris(t0, t1):
        t = np.arange(t0, t1, dtype=np.int64)
        q = t >> 1
        odd = (t & 1).astype(bool)
        r = q // (n - 1)
        c = q - r * (n - 1)
        v00 = r * n + c
        v10 = v00 + 1
        v01 = v00 + n
        v11 = v01 + 1
        out = np.empty((t1 - t0, 3), dtype=np.uint32)
        out[:, 0] = np.where(odd, v10, v00)
        out[:, 1] = v01
        out[:, 2] = np.where(odd, v11, v10)
        return out
    if shuffle:
        idx = _shuffle_chunks(tris, T, seed)
    else:
        idx = tris(0, T)
    return pos, idx


def uv_sphere(lat: int, lon: int, radius=1.0):
    """UV sphere with `lat` bands and `lon` segments, single pole vertices and a wrapped seam.
    Vertex 0 is the north pole (+y), ring k (1..lat-1, polar angle pi*k/lat) holds `lon`
    vertices 1+(k-1)*lon+j at azimuth 2*pi*j/lon, the south pole is last.  Each band/segment
    quad (a = ring k seg j, b = ring k seg j+1, c = ring k+1 seg j, d = ring k+1 seg j+1) gives
    the outward-facing triangles (a, b, c) and (b, d, c); the ones touching a pole are
    degenerate.  T = 2*lat*lon, V = (lat-1)*lon + 2.
    `radius` is a scalar or a callable radius(k_frac [R], j_frac [L]) -> float64 [R, L] used for
    the ring vertices, with radius(0, 0) / radius(1, 0) for the poles."""
    V = (lat - 1) * lon + 2
    theta = np.pi * np.arange(1, lat, dtype=np.float64) / lat
    phi = 2.0 * np.pi * np.arange(lon, dtype=np.float64) / lon
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    sp, cp = np.sin(phi)[None, :], np.cos(phi)[None, :]
    if callable(radius):
        rr = radius(np.arange(1, lat, dtype=np.float64) / lat, np.arange(lon, dtype=np.float64) / lon)
        r_n = float(radius(np.array([0.0]), np.array([0.0]))[0, 0])
        r_s = float(radius(np.array([1.0]), np.array([0.0]))[0, 0])
    else:
        rr = np.full((lat - 1, lon), float(radius))
        r_n = r_s = float(radius)
    pos = np.empty((V, 3), dtype=np.float32)
    pos[0] = (0.0, r_n, 0.0)
    pos[-1] = (0.0, -r_s, 0.0)
    ring = pos[1:-1].reshape(lat - 1, lon, 3)
    ring[:, :, 0] = (rr * st * cp).astype(np.float32)
    ring[:, :, 1] = (rr * ct).astype(np.float32)
    ring[:, :, 2] = (rr * st * sp).astype(np.float32)

    k = np.arange(lat, dtype=np.int64)[:, None]
    j = np.arange(lon, dtype=np.int64)[None, :]
    jn = (j + 1) % lon

    def ring_idx(kk, jj):
        kk = np.broadcast_to(kk, np.broadcast(kk, jj).shape)
        jj = np.broadcast_to(jj, kk.shape)
        out = 1 + (kk - 1) * lon + jj
        out = np.where(kk == 0, 0, out)
        out = np.where(kk == lat, V - 1, out)
        return out
    a = ring_idx(k, j)
    b = ring_idx(k, jn)
    c = ring_idx(k + 1, j)
    d = ring_idx(k + 1, jn)
    idx = np.empty((lat, lon, 2, 3), dtype=np.uint32)
    idx[:, :, 0, 0], idx[:, :, 0, 1], idx[:, :, 0, 2] = a, b, c
    idx[:, :, 1, 0], idx[:, :, 1, 1], idx[:, :, 1, 2] = b, d, c
    return pos, idx.reshape(-1, 3)


def bounding_sphere(pos: np.ndarray) -> np.ndarray:
    """Sphere around the axis-aligned bounding box (centre, half-diagonal), padded by a relative
    1e-5: it contains every vertex."""
    lo = pos.min(axis=0).astype(np.float64)
    hi = pos.max(axis=0).astype(np.float64)
    c = 0.5 * (lo + hi)
    r = 0.5 * float(np.linalg.norm(hi - lo))
    r = r * (1.0 + 1e-5) + 1e-7
    return np.array([c[0], c[1], c[2], r], dtype=np.float32)


# --------------------------------------------------------------------------------------------
# Cameras and transforms
# --------------------------------------------------------------------------------------------
def camera(eye, target, up=(0.0, 1.0, 0.0), fovy_deg: float = FOVY_DEG, aspect: float = 1.0) -> np.ndarray:
    """Row-major float32 4x4 view-projection: a right-handed look-at view (looking down -z)
    followed by the paper's projection vector [f/aspect, f, -1] (Sec. 4.1, Eqs. 1-2), so
    clip x = f/aspect * x_view, clip y = f * y_view and w = -z_view (positive linear depth).
    Row 2 is filled with the view z row; the rasterizer does not read it."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    view = np.eye(4)
    view[0, :3], view[0, 3] = right, -right @ eye
    view[1, :3], view[1, 3] = upv, -upv @ eye
    view[2, :3], view[2, 3] = -fwd, fwd @ eye
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    vp = np.zeros((4, 4))
    vp[0] = (f / aspect) * view[0]
    vp[1] = f * view[1]
    vp[2] = view[2]
    vp[3] = -view[2]
    return vp.astype(np.float32)


def orbit_camera(target, azimuth: float, elevation: float, distance: float, width: int, height: int,
                 near: float = NEAR) -> View:
    t = np.asarray(target, np.float64)
    eye = t + distance * np.array([math.cos(elevation) * math.cos(azimuth), math.sin(elevation),
                                   math.cos(elevation) * math.sin(azimuth)])
    return View(camera(eye, t, aspect=width / height), near, int(width), int(height))


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations from normalised Gaussian quaternions; float64 [n, 3, 3]."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def instance_matrices(R: np.ndarray, scale: np.ndarray, t: np.ndarray) -> np.ndarray:
    """float32 [n, 12] row-major 3x4 matrices [scale*R | t]."""
    n = R.shape[0]
    M = np.empty((n, 3, 4))
    M[:, :, :3] = R * np.asarray(scale, np.float64).reshape(n, 1, 1)
    M[:, :, 3] = t
    return M.reshape(n, 12).astype(np.float32)


# --------------------------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------------------------
def _hf_camera(width, height) -> View:
    return orbit_camera((0.5, 0.0, 0.5), math.radians(45.0), math.radians(45.0), 1.2, width, height)


# ----------------------------------------------------------------------------------------------
# Textures and texture coordinates for the textured resolve (Sec. 4.4).  The paper's scenes carry
# photographic textures; these are seeded procedural stand-ins with the same role: RGBA8, power of
# two, with detail at every scale so that mip levels differ.
# ----------------------------------------------------------------------------------------------
def texture_rgba8(width: int, height: int, seed: int, lines: int = 32) -> np.ndarray:
    """uint32 [height, width] RGBA8 (R in the low byte): fBm value noise through a colour ramp,
    darkened on grid lines every `lines` texels, alpha 255."""
    n = max(width, height, 2)
    f = fbm2_grid(n, seed, octaves=6)[:height, :width]
    f = np.clip(0.5 + 0.6 * f, 0.0, 1.0)
    r = f
    g = 0.5 + 0.5 * np.sin(6.0 * f)
    b = 1.0 - f
    jj, ii = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    dark = ((ii % lines) == 0) | ((jj % lines) == 0)
    shade = np.where(dark, 0.3, 1.0)
    to8 = lambda c: np.clip(np.rint(c * shade * 255.0), 0, 255).astype(np.uint32)
    return to8(r) | (to8(g) << 8) | (to8(b) << 16) | (np.uint32(255) << 24)


def planar_uv(pos: np.ndarray, axes=(0, 2), scale=1.0, offset=0.0) -> np.ndarray:
    """float32 [V, 2] texture coordinates (pos[:, axes[0]], pos[:, axes[1]]) * scale + offset."""
    p = np.asarray(pos, np.float64)
    uv = np.stack([p[:, axes[0]], p[:, axes[1]]], axis=1) * scale + offset
    return uv.astype(np.float32)


def scene_c1() -> Scene:
    """Plain pipeline at oracle size: jittered UV sphere 256 x 512 (r = 1, per-vertex
    N(0, 1e-3) jitter, seed 1) plus a 20 x 20 ground quad at y = -1 that crosses the near plane;
    camera at (0, 0, 3) looking at the origin, 512 x 512, per-vertex RGB uniform[0,1] (seed 11)."""
    pos, idx = uv_sphere(256, 512, 1.0)
    rng = np.random.default_rng(1)
    pos = (pos.astype(np.float64) + rng.normal(0.0, 1e-3, pos.shape)).astype(np.float32)
    gpos = np.array([[-10, -1, -10], [10, -1, -10], [-10, -1, 10], [10, -1, 10]], np.float32)
    gidx = np.array([[0, 2, 1], [1, 2, 3]], np.uint32)
    rng = np.random.default_rng(11)
    sphere = Mesh(pos, idx, attrs=rng.uniform(0, 1, (pos.shape[0], 3)).astype(np.float32),
                  bsphere=bounding_sphere(pos))
    ground = Mesh(gpos, gidx, attrs=rng.uniform(0, 1, (4, 3)).astype(np.float32),
                  bsphere=bounding_sphere(gpos))
    view = View(camera((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), aspect=1.0), NEAR, 512, 512)
    return Scene("c1_sphere_ground_512", [sphere, ground], [view])


def _hf_mesh(n, amplitude, seed, attr_seed=None, attr_normal=False) -> Mesh:
    """Height field mesh with per-vertex RGB: uniform [0, 1) by default, N(0.5, 0.1) when
    attr_normal (both drawn in float32 from numpy's default generator with attr_seed)."""
    pos, idx = heightfield(n, amplitude, seed)
    attrs = None
    if attr_seed is not None:
        rng = np.random.default_rng(attr_seed)
        if attr_normal:
            attrs = rng.standard_normal((pos.shape[0], 3), dtype=np.float32) * np.float32(0.1) + np.float32(0.5)
        else:
            attrs = rng.random((pos.shape[0], 3), dtype=np.float32)
    return Mesh(pos, idx, attrs=attrs, bsphere=bounding_sphere(pos))


def scene_c2(n: int = 4096) -> Scene:
    """Dense height field: 4096^2 vertices, amplitude 0.1 (seed 2), 1920 x 1080 camera at 45 deg
    elevation and azimuth, distance 1.2 from (0.5, 0, 0.5)."""
    hf = _hf_mesh(n, 0.1, 2, attr_seed=22)
    return Scene(f"c2_heightfield_{n}_1080p", [hf], [_hf_camera(1920, 1080)])


def _noisy_radius(base_r: float, seed: int, amp: float = 0.05, octaves: int = 4):
    """radius(k_frac, j_frac) = base_r * (1 + amp * fBm) over (polar, azimuth) fractions, with a
    lattice that wraps in the azimuth so the seam is continuous."""
    def fn(kf, jf):
        return base_r * (1.0 + amp * fbm2_points(jf[None, :], kf[:, None], seed, octaves=octaves,
                                                  base=4, wrap_u=True))
    return fn


def scene_c3(n: int = 16384, instances: int = 4096, sphere_lon: int = 1024, width: int = 3840,
             height: int = 2160) -> Scene:
    """Massive 4K frame: C3a = n^2 height field (seed 3, amplitude 0.1) and C3b = one
    noise-displaced UV sphere (lat = lon = 1024, T = 2,097,152, radius 0.004 * (1 + 0.05 fBm),
    seed 33) instanced 4096x with uniform random rotations, scale U[0.5, 2] and positions on the
    height field (seed 34); camera as C2 at 3840 x 2160."""
    hf = _hf_mesh(n, 0.1, 3, attr_seed=31)
    spos, sidx = uv_sphere(sphere_lon, sphere_lon, _noisy_radius(0.004, 33))
    rng = np.random.default_rng(34)
    R = random_rotations(rng, instances)
    scale = rng.uniform(0.5, 2.0, instances)
    xz = rng.uniform(0.02, 0.98, (instances, 2))
    y = 0.1 * fbm2_points(xz[:, 0], xz[:, 1], 3) + 0.004 * scale
    inst = instance_matrices(R, scale, np.stack([xz[:, 0], y, xz[:, 1]], axis=1))
    sattr = np.random.default_rng(35).uniform(0, 1, (spos.shape[0], 3)).astype(np.float32)
    sphere = Mesh(spos, sidx, inst=inst, attrs=sattr, bsphere=bounding_sphere(spos))
    return Scene(f"c3_heightfield_{n}_plus_{instances}x_sphere_4k", [hf, sphere],
                 [_hf_camera(width, height)])


def scene_c4(n: int = 4096, n_views: int = 64, n_spheres: int = 512, t_min: int = 1024,
             t_max: int = 4_000_000) -> Scene:
    """Batched: 64 views (seed 4) with independent W, H uniform in [256, 2048], targets uniform in
    [0.2, 0.8]^2 on the C2 height field, azimuth U[0, 2pi), elevation U[20, 70] deg, distance
    U[0.3, 1.5]; plus 512 noise-displaced UV spheres (seed 44) with T = lon^2 (lat = lon/2),
    T log-uniform in [1024, 4M], radius U[0.005, 0.05], random rotation, resting on the field."""
    hf = _hf_mesh(n, 0.1, 2, attr_seed=22)
    rng = np.random.default_rng(44)
    T = np.exp(rng.uniform(math.log(t_min), math.log(t_max), n_spheres))
    lon = np.maximum(8, 2 * np.round(np.sqrt(T) / 2.0)).astype(np.int64)
    radius = rng.uniform(0.005, 0.05, n_spheres)
    R = random_rotations(rng, n_spheres)
    xz = rng.uniform(0.05, 0.95, (n_spheres, 2))
    y = 0.1 * fbm2_points(xz[:, 0], xz[:, 1], 2) + radius
    mats = instance_matrices(R, np.ones(n_spheres), np.stack([xz[:, 0], y, xz[:, 1]], axis=1))

    def make(i):
        lo = int(lon[i])
        p, ix = uv_sphere(lo // 2, lo, _noisy_radius(float(radius[i]), 4400 + i, octaves=3))
        return Mesh(p, ix, inst=mats[i:i + 1].copy(), bsphere=bounding_sphere(p))
    with ThreadPoolExecutor(_threads()) as ex:
        spheres = list(ex.map(make, range(n_spheres)))
    vr = np.random.default_rng(4)
    views = []
    for _ in range(n_views):
        w = int(vr.integers(256, 2049))
        h = int(vr.integers(256, 2049))
        tx, tz = vr.uniform(0.2, 0.8, 2)
        ty = 0.1 * float(fbm2_points(np.array([tx]), np.array([tz]), 2)[0])
        az = vr.uniform(0.0, 2.0 * math.pi)
        el = math.radians(vr.uniform(20.0, 70.0))
        dist = vr.uniform(0.3, 1.5)
        views.append(orbit_camera((tx, ty, tz), az, el, dist, w, h))
    return Scene(f"c4_batched_{n_views}views_{n_spheres}meshes", [hf] + spheres, views)


def scene_c5(n: int = 2236) -> Scene:
    """Differentiable resolve: 2236^2 height field (seed 5, amplitude 0.1, T = 9,990,450),
    1024 x 1024 camera as C2, attributes RGB N(0.5, 0.1) (seed 55); the target image
    N(0.5, 0.1) per pixel (seed 56) is stored in meta['target']."""
    hf = _hf_mesh(n, 0.1, 5, attr_seed=55, attr_normal=True)
    view = _hf_camera(1024, 1024)
    target = np.random.default_rng(56).normal(0.5, 0.1, (1024, 1024, 3)).astype(np.float32)
    return Scene(f"c5_heightfield_{n}_1024", [hf], [view], meta={"target": target})


def scene_by_name(name: str, **kw) -> Scene:
    return {"c1": scene_c1, "c2": scene_c2, "c3": scene_c3, "c4": scene_c4, "c5": scene_c5}[name](**kw)


def random_tiny_scene(seed: int, n_tris: int = 16, width: int = 48, height: int = 40,
                      n_instances: int = 1, snap_grid: bool = False, spread: float = 1.5,
                      depth_range=(1.0, 6.0), near_crossing: bool = False) -> Scene:
    """A few random triangles in front of a camera, for brute-force comparisons.
    snap_grid=True puts vertices so that their screen positions land on pixel centres and
    pixel edges (exact ties for the fill rule); near_crossing=True spreads some vertices
    behind the camera."""
    rng = np.random.default_rng(seed)
    aspect = width / height
    vp = camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=aspect)
    pos = np.empty((3 * n_tris, 3), np.float64)
    for t in range(n_tris):
        d = rng.uniform(*depth_range)
        c = rng.uniform(-spread, spread, 2) * d * 0.5
        for k in range(3):
            dk = d * rng.uniform(0.8, 1.25)
            if near_crossing and rng.uniform() < 0.3:
                dk = rng.uniform(-2.0, 0.05)
            off = rng.normal(0.0, 0.35, 2) * max(abs(dk), 0.3)
            pos[3 * t + k] = (c[0] + off[0], c[1] + off[1], -dk)
    if snap_grid:
        # choose x, y so that the projected point lands on a multiple of half a pixel
        f = 1.0 / math.tan(math.radians(FOVY_DEG) / 2.0)
        for v in range(pos.shape[0]):
            z = -pos[v, 2]
            z = float(2.0 ** round(math.log2(max(z, 0.25))))        # exact power-of-two depth
            px = rng.integers(-2, 2 * width + 2) * 0.5
            py = rng.integers(-2, 2 * height + 2) * 0.5
            ndc_x = px / (0.5 * width) - 1.0
            ndc_y = py / (0.5 * height) - 1.0
            pos[v] = (ndc_x * z * aspect / f, ndc_y * z / f, -z)
    idx = np.arange(3 * n_tris, dtype=np.uint32).reshape(n_tris, 3)
    inst = None
    if n_instances > 1:
        R = random_rotations(rng, n_instances) * 0.0 + np.eye(3)
        t = rng.normal(0.0, 0.2, (n_instances, 3))
        inst = instance_matrices(R, rng.uniform(0.8, 1.2, n_instances), t)
    attrs = rng.uniform(0, 1, (pos.shape[0], 3)).astype(np.float32)
    m = Mesh(pos.astype(np.float32), idx, inst=inst, attrs=attrs)
    return Scene(f"tiny_{seed}", [m], [View(vp, NEAR, width, height)])

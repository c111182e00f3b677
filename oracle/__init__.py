"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
The rasterizer library never loads it; the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Mesh(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("V", C.c_uint32), ("idx", C.c_void_p), ("T", C.c_uint64),
                ("inst", C.c_void_p), ("N", C.c_uint32)]


class _View(C.Structure):
    _fields_ = [("vp", C.c_float * 16), ("near_plane", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # noqa: F401  (oracle/build.py)
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        _lib.orc_num_pairs.restype = C.c_int64
        _lib.orc_num_pairs.argtypes = [P, C.c_uint32]
        _lib.orc_texture_texels.restype = C.c_uint64
        _lib.orc_texture_texels.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        _lib.orc_sample_trilinear.restype = None
        _lib.orc_sample_trilinear.argtypes = [P, C.c_float, C.c_float, C.c_float, P]
        _lib.orc_texture_lod.restype = C.c_float
        _lib.orc_texture_lod.argtypes = [P, P, P, C.c_int]
        for name, args in {
            "orc_id_bases": [P, C.c_uint32, P],
            "orc_decode_id": [P, C.c_uint32, P, C.c_int64, P, P, P],
            "orc_rasterize": [P, C.c_uint32, P, P, C.c_int],
            "orc_rasterize_range": [P, C.c_uint32, P, C.c_int64, C.c_int64, C.c_uint64, C.c_uint64, P, C.c_int],
            "orc_coverage_counts": [P, C.c_uint32, P, P, P],
            "orc_rasterize_brute": [P, C.c_uint32, P, P],
            "orc_project": [P, C.c_uint32, P, P],
            "orc_quantize_positions": [P, C.c_uint32, P, P, P],
            "orc_decode_positions": [P, C.c_uint32, P, P, P],
            "orc_resolve": [P, C.c_uint32, P, P, P, C.c_uint32, P, C.c_int],
            "orc_build_mips": [P, C.c_uint32, C.c_uint32, C.c_uint32],
            "orc_resolve_textured": [P, C.c_uint32, P, P, P, P, P, C.c_int],
            "orc_resolve_screen": [P, C.c_int32, C.c_int32, P, C.c_uint64, C.c_int64, P, C.c_uint32, P, C.c_uint32, P],
            "orc_resolve_screen_f64": [P, C.c_int32, C.c_int32, P, C.c_uint64, C.c_int64, P, C.c_uint32, P, C.c_uint32, P],
            "orc_resolve_screen_backward_f64": [P, C.c_int32, C.c_int32, P, C.c_uint64, C.c_int64, P, C.c_uint32, P,
                                                C.c_uint32, P, P, P],
            "orc_fd_pos_grad_l2": [P, C.c_int32, C.c_int32, P, C.c_uint64, C.c_int64, P, C.c_uint32, P, C.c_uint32,
                                   P, P, C.c_uint32, C.c_double, C.c_int, P],
        }.items():
            f = getattr(_lib, name)
            f.restype = C.c_int
            f.argtypes = args
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Pack:
    """Keeps numpy arrays alive while their pointers sit in ctypes structures."""

    def __init__(self, meshes, view=None):
        self.keep = []
        arr = (_Mesh * max(1, len(meshes)))()
        for i, m in enumerate(meshes):
            pos = np.ascontiguousarray(m.pos, np.float32)
            idx = np.ascontiguousarray(m.idx, np.uint32)
            inst = None if m.inst is None else np.ascontiguousarray(m.inst, np.float32)
            self.keep += [pos, idx, inst]
            arr[i] = _Mesh(pos.ctypes.data, pos.shape[0], idx.ctypes.data, idx.shape[0],
                           None if inst is None else inst.ctypes.data, 1 if inst is None else inst.shape[0])
        self.meshes = arr
        self.M = len(meshes)
        if view is not None:
            v = _View()
            vp = np.ascontiguousarray(view.vp, np.float32).reshape(16)
            for k in range(16):
                v.vp[k] = float(vp[k])
            v.near_plane = float(view.near)
            v.width = int(view.width)
            v.height = int(view.height)
            self.view = v


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with {rc}")


def id_bases(meshes) -> np.ndarray:
    pk = _Pack(meshes)
    n = lib().orc_num_pairs(pk.meshes, pk.M)
    out = np.zeros(n + 1, np.int64)
    _check(lib().orc_id_bases(pk.meshes, pk.M, out.ctypes.data), "id_bases")
    return out


def decode_id(meshes, bases: np.ndarray, gid: int):
    pk = _Pack(meshes)
    m, i, t = C.c_uint32(), C.c_uint32(), C.c_uint64()
    rc = lib().orc_decode_id(pk.meshes, pk.M, bases.ctypes.data, int(gid), C.byref(m), C.byref(i), C.byref(t))
    return None if rc != 0 else (m.value, i.value, t.value)


def rasterize(meshes, view, threads: int = 0) -> np.ndarray:
    pk = _Pack(meshes, view)
    vis = np.empty((view.height, view.width), np.uint64)
    _check(lib().orc_rasterize(pk.meshes, pk.M, C.byref(pk.view), vis.ctypes.data, threads), "rasterize")
    return vis


def rasterize_range(meshes, view, pair_begin: int, pair_end: int, tri_begin: int, tri_end: int,
                    threads: int = 0) -> np.ndarray:
    pk = _Pack(meshes, view)
    vis = np.empty((view.height, view.width), np.uint64)
    _check(lib().orc_rasterize_range(pk.meshes, pk.M, C.byref(pk.view), pair_begin, pair_end, tri_begin,
                                     tri_end, vis.ctypes.data, threads), "rasterize_range")
    return vis


def rasterize_brute(meshes, view) -> np.ndarray:
    pk = _Pack(meshes, view)
    vis = np.empty((view.height, view.width), np.uint64)
    _check(lib().orc_rasterize_brute(pk.meshes, pk.M, C.byref(pk.view), vis.ctypes.data), "rasterize_brute")
    return vis


def coverage_counts(meshes, view):
    pk = _Pack(meshes, view)
    front = np.empty((view.height, view.width), np.uint32)
    back = np.empty((view.height, view.width), np.uint32)
    _check(lib().orc_coverage_counts(pk.meshes, pk.M, C.byref(pk.view), front.ctypes.data, back.ctypes.data),
           "coverage_counts")
    return front, back


def project(mesh, view, instance: int = 0) -> np.ndarray:
    pk = _Pack([mesh], view)
    out = np.empty((mesh.pos.shape[0], 3), np.float32)
    _check(lib().orc_project(C.byref(pk.meshes[0]), instance, C.byref(pk.view), out.ctypes.data), "project")
    return out


def resolve(meshes, view, vis: np.ndarray, attrs: Sequence[np.ndarray], threads: int = 0) -> np.ndarray:
    pk = _Pack(meshes, view)
    C_ = int(attrs[0].shape[1])
    keep = [np.ascontiguousarray(a, np.float32) for a in attrs]
    ptrs = (C.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
    vis = np.ascontiguousarray(vis, np.uint64)
    out = np.empty((view.height, view.width, C_), np.float32)
    _check(lib().orc_resolve(pk.meshes, pk.M, C.byref(pk.view), vis.ctypes.data, ptrs, C_, out.ctypes.data,
                             threads), "resolve")
    return out


# ----------------------------------------------------------------------------------------------
# compressed geometry (Sec. 4.6)
# ----------------------------------------------------------------------------------------------
def index_bits(span: int) -> int:
    """Bits per packed index for indices spanning [min, min + span]: the paper's ceil(log2(span))
    read as ceil(log2(span + 1)), the width that holds span itself; at least 1."""
    return max(1, int(span).bit_length())


def compress_indices(idx: np.ndarray):
    """(index_min, bits, packed uint32 words): index i of the flattened [T, 3] array minus
    index_min occupies bits [i bits, (i + 1) bits) of a little-endian stream, plus three zero
    words of padding.  Written bit by bit (small meshes only)."""
    flat = np.ascontiguousarray(idx, np.uint32).reshape(-1).astype(np.uint64)
    lo = int(flat.min()) if flat.size else 0
    hi = int(flat.max()) if flat.size else 0
    b = index_bits(hi - lo)
    words = np.zeros((flat.size * b + 31) // 32 + 3, np.uint64)
    vals = flat - np.uint64(lo)
    for j in range(b):
        bit = (vals >> np.uint64(j)) & np.uint64(1)
        pos = np.arange(flat.size, dtype=np.uint64) * np.uint64(b) + np.uint64(j)
        np.bitwise_or.at(words, (pos >> np.uint64(5)).astype(np.int64), bit << (pos & np.uint64(31)))
    return lo, b, words.astype(np.uint32)


def decompress_indices(words: np.ndarray, index_min: int, bits: int, T: int) -> np.ndarray:
    w = np.asarray(words, np.uint32).astype(np.uint64)
    out = np.zeros(3 * T, np.uint64)
    for j in range(bits):
        pos = np.arange(3 * T, dtype=np.uint64) * np.uint64(bits) + np.uint64(j)
        out |= ((w[(pos >> np.uint64(5)).astype(np.int64)] >> (pos & np.uint64(31))) & np.uint64(1)) << np.uint64(j)
    return (out + np.uint64(index_min)).astype(np.uint32).reshape(T, 3)


def position_box(pos: np.ndarray):
    """(lo, step) per axis: lo = the minimum, step = (float)(((double)max - (double)min) / 65535)."""
    p = np.asarray(pos, np.float32)
    lo = p.min(axis=0) if p.size else np.zeros(3, np.float32)
    hi = p.max(axis=0) if p.size else np.zeros(3, np.float32)
    step = ((hi.astype(np.float64) - lo.astype(np.float64)) / 65535.0).astype(np.float32)
    return lo.astype(np.float32), step


def quantize_positions(pos: np.ndarray, lo, step) -> np.ndarray:
    p = np.ascontiguousarray(pos, np.float32)
    out = np.empty(p.shape, np.uint16)
    lo = np.ascontiguousarray(lo, np.float32)
    step = np.ascontiguousarray(step, np.float32)
    _check(lib().orc_quantize_positions(p.ctypes.data, p.shape[0], lo.ctypes.data, step.ctypes.data,
                                        out.ctypes.data), "quantize")
    return out


def decode_positions(q: np.ndarray, lo, step) -> np.ndarray:
    q = np.ascontiguousarray(q, np.uint16)
    out = np.empty(q.shape, np.float32)
    lo = np.ascontiguousarray(lo, np.float32)
    step = np.ascontiguousarray(step, np.float32)
    _check(lib().orc_decode_positions(q.ctypes.data, q.shape[0], lo.ctypes.data, step.ctypes.data,
                                      out.ctypes.data), "decode")
    return out


def decompressed_mesh(m, words, index_min, bits, qpos, lo, step):
    """The uncompressed mesh a compressed one renders as (same instances, bounding sphere)."""
    from dataclasses import replace
    return replace(m, pos=decode_positions(qpos, lo, step),
                   idx=decompress_indices(words, index_min, bits, m.idx.shape[0]))


def box_filter(samples: np.ndarray, k: int) -> np.ndarray:
    """Mean of each k x k block of resolved samples [k H, k W, C] -> [H, W, C] (the supersampled
    resolve, Sec. 5 "Anti-Aliasing (Super Sampling)"): an fp32 sum over the block's rows, then its
    columns, in that order, times 1 / k^2 (exact)."""
    kH, kW, C_ = samples.shape
    if kH % k or kW % k:
        raise ValueError("sample grid not a multiple of k")
    samples = np.asarray(samples, np.float32)
    acc = np.zeros((kH // k, kW // k, C_), np.float32)
    for sy in range(k):
        for sx in range(k):
            acc += samples[sy::k, sx::k]
    return acc * np.float32(1.0 / (k * k))


def resolve_supersampled(meshes, view_hi, vis_hi: np.ndarray, attrs, k: int, threads: int = 0) -> np.ndarray:
    """Resolve every sample of the k-times-larger view, then box-filter k x k blocks."""
    return box_filter(resolve(meshes, view_hi, vis_hi, attrs, threads=threads), k)


# ----------------------------------------------------------------------------------------------
# textured resolve (Sec. 4.4, "Shading and Mip Mapping")
# ----------------------------------------------------------------------------------------------
class _Tex(C.Structure):
    _fields_ = [("texels", C.c_void_p), ("width", C.c_uint32), ("height", C.c_uint32), ("levels", C.c_uint32)]


def texture_texels(width: int, height: int, levels: int) -> int:
    """Words of an RGBA8 mip chain (0 for invalid sizes / level counts)."""
    return int(lib().orc_texture_texels(width, height, levels))


def level_shape(width: int, height: int, level: int):
    return max(1, height >> level), max(1, width >> level)


def build_mips(level0: np.ndarray, levels: int) -> np.ndarray:
    """The whole chain (uint32 words, levels concatenated) from level 0 [height, width] uint32."""
    h, w = level0.shape
    n = texture_texels(w, h, levels)
    if not n:
        raise ValueError("invalid texture size or level count")
    chain = np.zeros(n, np.uint32)
    chain[:w * h] = np.ascontiguousarray(level0, np.uint32).reshape(-1)
    _check(lib().orc_build_mips(chain.ctypes.data, w, h, levels), "build_mips")
    return chain


def texture_level(chain: np.ndarray, width: int, height: int, level: int) -> np.ndarray:
    off = sum(level_shape(width, height, j)[0] * level_shape(width, height, j)[1] for j in range(level))
    hl, wl = level_shape(width, height, level)
    return chain[off:off + hl * wl].reshape(hl, wl)


def _tex_struct(chain, width, height, levels):
    return _Tex(chain.ctypes.data, width, height, levels)


def sample_trilinear(chain: np.ndarray, width: int, height: int, levels: int, u: float, v: float, lod: float):
    chain = np.ascontiguousarray(chain, np.uint32)
    t = _tex_struct(chain, width, height, levels)
    out = np.zeros(4, np.float32)
    lib().orc_sample_trilinear(C.byref(t), float(u), float(v), float(lod), out.ctypes.data)
    return out


def texture_lod(width: int, height: int, levels: int, u, v, finite: bool = True) -> float:
    u = np.ascontiguousarray(u, np.float32)
    v = np.ascontiguousarray(v, np.float32)
    dummy = np.zeros(1, np.uint32)
    t = _tex_struct(dummy, width, height, levels)
    return float(lib().orc_texture_lod(C.byref(t), u.ctypes.data, v.ctypes.data, int(finite)))


def resolve_textured(meshes, view, vis: np.ndarray, uvs, textures, threads: int = 0) -> np.ndarray:
    """RGBA [H, W, 4]; uvs[m] float32 [V, 2]; textures[m] = (chain uint32, width, height, levels)."""
    pk = _Pack(meshes, view)
    keep_uv = [np.ascontiguousarray(a, np.float32) for a in uvs]
    keep_tx = [np.ascontiguousarray(t[0], np.uint32) for t in textures]
    uptr = (C.c_void_p * max(1, len(keep_uv)))(*[a.ctypes.data for a in keep_uv])
    tarr = (_Tex * max(1, len(textures)))(*[_tex_struct(c, t[1], t[2], t[3]) for c, t in zip(keep_tx, textures)])
    vis = np.ascontiguousarray(vis, np.uint64)
    out = np.empty((view.height, view.width, 4), np.float32)
    _check(lib().orc_resolve_textured(pk.meshes, pk.M, C.byref(pk.view), vis.ctypes.data, uptr, tarr,
                                      out.ctypes.data, threads), "resolve_textured")
    return out


def resolve_screen(vis, idx, id_base, pos_ss, attrs) -> np.ndarray:
    H, W = vis.shape
    vis = np.ascontiguousarray(vis, np.uint64)
    idx = np.ascontiguousarray(idx, np.uint32)
    pos_ss = np.ascontiguousarray(pos_ss, np.float32)
    attrs = np.ascontiguousarray(attrs, np.float32)
    out = np.empty((H, W, attrs.shape[1]), np.float32)
    _check(lib().orc_resolve_screen(vis.ctypes.data, W, H, idx.ctypes.data, idx.shape[0], int(id_base),
                                    pos_ss.ctypes.data, pos_ss.shape[0], attrs.ctypes.data, attrs.shape[1],
                                    out.ctypes.data), "resolve_screen")
    return out


def resolve_screen_f64(vis, idx, id_base, pos_ss, attrs) -> np.ndarray:
    H, W = vis.shape
    vis = np.ascontiguousarray(vis, np.uint64)
    idx = np.ascontiguousarray(idx, np.uint32)
    pos_ss = np.ascontiguousarray(pos_ss, np.float64)
    attrs = np.ascontiguousarray(attrs, np.float64)
    out = np.empty((H, W, attrs.shape[1]), np.float64)
    _check(lib().orc_resolve_screen_f64(vis.ctypes.data, W, H, idx.ctypes.data, idx.shape[0], int(id_base),
                                        pos_ss.ctypes.data, pos_ss.shape[0], attrs.ctypes.data, attrs.shape[1],
                                        out.ctypes.data), "resolve_screen_f64")
    return out


def resolve_screen_backward_f64(vis, idx, id_base, pos_ss, attrs, grad_out):
    H, W = vis.shape
    vis = np.ascontiguousarray(vis, np.uint64)
    idx = np.ascontiguousarray(idx, np.uint32)
    pos_ss = np.ascontiguousarray(pos_ss, np.float64)
    attrs = np.ascontiguousarray(attrs, np.float64)
    grad_out = np.ascontiguousarray(grad_out, np.float64)
    ga = np.zeros(attrs.shape, np.float64)
    gp = np.zeros(pos_ss.shape, np.float64)
    _check(lib().orc_resolve_screen_backward_f64(vis.ctypes.data, W, H, idx.ctypes.data, idx.shape[0],
                                                 int(id_base), pos_ss.ctypes.data, pos_ss.shape[0],
                                                 attrs.ctypes.data, attrs.shape[1], grad_out.ctypes.data,
                                                 ga.ctypes.data, gp.ctypes.data), "resolve_backward_f64")
    return ga, gp


def fd_pos_grad_l2(vis, idx, id_base, pos_ss, attrs, target, verts, eps=1e-3, order4=True) -> np.ndarray:
    H, W = vis.shape
    vis = np.ascontiguousarray(vis, np.uint64)
    idx = np.ascontiguousarray(idx, np.uint32)
    pos_ss = np.ascontiguousarray(pos_ss, np.float64)
    attrs = np.ascontiguousarray(attrs, np.float64)
    target = np.ascontiguousarray(target, np.float64)
    verts = np.ascontiguousarray(verts, np.uint32)
    fd = np.zeros((verts.shape[0], 3), np.float64)
    _check(lib().orc_fd_pos_grad_l2(vis.ctypes.data, W, H, idx.ctypes.data, idx.shape[0], int(id_base),
                                    pos_ss.ctypes.data, pos_ss.shape[0], attrs.ctypes.data, attrs.shape[1],
                                    target.ctypes.data, verts.ctypes.data, verts.shape[0], float(eps),
                                    1 if order4 else 0, fd.ctypes.data), "fd_pos_grad_l2")
    return fd


# ----------------------------------------------------------------------------------------------
# Key layout helpers (Sec. 4.1: 28-bit depth above a 36-bit global triangle ID)
# ----------------------------------------------------------------------------------------------
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
ID_BITS = 36


def key_id(vis: np.ndarray) -> np.ndarray:
    return vis & np.uint64((1 << ID_BITS) - 1)


def key_depth(vis: np.ndarray) -> np.ndarray:
    """float32 depth with the 3 dropped mantissa bits zeroed (valid where vis != EMPTY)."""
    d28 = (vis >> np.uint64(ID_BITS)).astype(np.uint32)
    return (d28 << np.uint32(3)).view(np.float32)

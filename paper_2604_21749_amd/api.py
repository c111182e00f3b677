"""Python binding of the C ABI in include/curast.h (ctypes; argument marshalling only).

Every step of the path runs in the HIP library libcurast.so built in this package directory; this
module only passes torch tensors' device pointers, sizes and the current HIP stream.  There is no
fallback: if the library is not built, or no GPU is present, calls raise.

Visibility buffers are torch.int64 tensors [H, W] holding the uint64 keys bit for bit (torch has
no general uint64 arithmetic); `as_uint64(t)` gives a numpy uint64 copy.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcurast.so")

OK, E_INVALID, E_ID_RANGE, E_OOM, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FLAG_NO_TINY_CULL = 0x1
FLAG_NO_EARLY_OUT = 0x2
FLAG_NO_MESH_CULL = 0x4
FLAG_STATS = 0x8
FLAG_NO_GRAPH = 0x10
FLAG_TIMING = 0x20
FLAG_S3_PER_PART = 0x40
FLAG_NO_FAST_INTERIOR = 0x80
FLAG_NO_STRIPS = 0x100
FLAG_SINGLE_STRIPS = 0x200
FLAG_S1_OVERLAP = 0x400
FLAG_EARLY_OUT_ALL = 0x800
FLAG_ZERO_QUEUES = 0x80000000

EMPTY_KEY = np.uint64(0xFFFFFFFFFFFFFFFF)


class CurastError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"curast error {status}: {message}")
        self.status = status


class Options(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in (
        "small_px", "medium_px", "s1_block", "s1_tris_per_thread", "s1_draws_per_item", "s2_waves",
        "s3_blocks", "q2_capacity", "q3_capacity", "large_capacity", "flags", "s1_mode",
        "s1_multi_tris_per_thread", "s1_blocks_per_cu")]


class CompressedStruct(C.Structure):
    _fields_ = [("indices", C.c_void_p), ("positions", C.c_void_p), ("index_min", C.c_uint32),
                ("index_bits", C.c_uint32), ("lo", C.c_float * 3), ("step", C.c_float * 3)]


class MeshStruct(C.Structure):
    _fields_ = [("vertices", C.c_void_p), ("num_vertices", C.c_uint32), ("indices", C.c_void_p),
                ("num_triangles", C.c_uint64), ("instances", C.c_void_p), ("num_instances", C.c_uint32),
                ("bsphere", C.c_float * 4), ("compressed", C.c_void_p)]


class TextureStruct(C.Structure):
    _fields_ = [("texels", C.c_void_p), ("width", C.c_uint32), ("height", C.c_uint32), ("levels", C.c_uint32)]


class ViewStruct(C.Structure):
    _fields_ = [("view_proj", C.c_float * 16), ("near_plane", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("visbuffer", C.c_void_p)]


class StatsStruct(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "tri_draws", "draws_culled", "culled_near", "culled_frustum", "culled_tiny", "culled_backface",
        "s1_rasterized", "q2_entries", "q2_overflow", "s2_rasterized", "q3_entries", "q3_overflow",
        "fragments", "atomics", "strip_draws", "strip_union_pass", "strip_sphere_pass")]


# Every entry point of include/curast.h with its ctypes signature.
_P = C.c_void_p
SIGNATURES = {
    "curast_create": (C.c_int, [C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "curast_destroy": (C.c_int, [_P]),
    "curast_set_options": (C.c_int, [_P, C.POINTER(Options)]),
    "curast_get_options": (C.c_int, [_P, C.POINTER(Options)]),
    "curast_rasterize": (C.c_int, [_P, _P, C.c_uint32, _P, C.c_uint64, _P, C.c_uint32, _P, C.c_float, C.c_int32,
                                   C.c_int32, _P, _P]),
    "curast_rasterize_noalloc": (C.c_int, [_P, _P, C.c_uint32, _P, C.c_uint64, _P, C.c_uint32, _P, C.c_float,
                                           C.c_int32, C.c_int32, _P, _P]),
    "curast_rasterize_meshes": (C.c_int, [_P, _P, C.c_uint32, _P, _P]),
    "curast_rasterize_batched": (C.c_int, [_P, _P, C.c_uint32, _P, C.c_uint32, _P]),
    "curast_project": (C.c_int, [_P, _P, C.c_uint32, _P, _P, _P]),
    "curast_resolve": (C.c_int, [_P, _P, C.c_uint32, _P, _P, C.c_uint32, _P, _P]),
    "curast_compress_prepare": (C.c_int, [_P, _P, _P, _P, _P]),
    "curast_compress": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "curast_resolve_supersampled": (C.c_int, [_P, _P, C.c_uint32, _P, C.c_uint32, _P, C.c_uint32, _P, _P]),
    "curast_texture_texels": (C.c_uint64, [C.c_uint32, C.c_uint32, C.c_uint32]),
    "curast_build_mips": (C.c_int, [_P, _P, C.c_uint32, C.c_uint32, C.c_uint32, _P]),
    "curast_resolve_textured": (C.c_int, [_P, _P, C.c_uint32, _P, _P, _P, _P, _P]),
    "curast_resolve_screen": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, C.c_uint64, C.c_uint64, _P, C.c_uint32,
                                        _P, C.c_uint32, _P, _P]),
    "curast_resolve_backward": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, C.c_uint64, C.c_uint64, _P,
                                          C.c_uint32, _P, C.c_uint32, _P, _P, _P, _P]),
    "curast_resolve_backward_meshes": (C.c_int, [_P, _P, C.c_uint32, _P, _P, C.c_uint32, _P, _P, _P, _P]),
    "curast_autotune": (C.c_int, [_P, _P, C.c_uint32, _P, C.c_uint32, C.c_char_p, C.POINTER(Options), _P]),
    "curast_get_stats": (C.c_int, [_P, C.POINTER(StatsStruct)]),
    "curast_reset_stats": (C.c_int, [_P]),
    "curast_get_stage_times": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "curast_reset_stage_times": (C.c_int, [_P]),
    "curast_id_bases": (C.c_int64, [_P, C.c_uint32, _P]),
    "curast_plan": (C.c_int, [_P, C.c_uint32, _P, C.c_uint32, C.POINTER(Options), _P, _P, _P]),
    "curast_status_string": (C.c_char_p, [C.c_int]),
    "curast_last_error": (C.c_char_p, [_P]),
    "curast_version": (C.c_int, []),
}

_lib = None


def lib():
    """Load libcurast.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_21749_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def as_uint64(vis: torch.Tensor) -> np.ndarray:
    """Host uint64 copy of a visibility buffer tensor."""
    return vis.detach().cpu().numpy().view(np.uint64)


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _check_cuda(t: torch.Tensor, dtype, name: str, shape_last=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape [N, {shape_last}]")


@dataclass
class GpuMesh:
    """A mesh whose vertices and indices live in device memory (indices as int32 bits of uint32),
    or whose geometry is compressed (pos and idx None, `compressed` set)."""
    pos: Optional[torch.Tensor]             # float32 [V, 3] (cuda)
    idx: Optional[torch.Tensor]             # int32 [T, 3] (cuda)
    inst: Optional[np.ndarray] = None       # float32 [N, 12] host, or None
    bsphere: Optional[np.ndarray] = None    # float32 [4] host, or None
    attrs: Optional[torch.Tensor] = None    # float32 [V, C] (cuda), for resolve
    compressed: Optional["CompressedGeometry"] = None

    @property
    def num_instances(self) -> int:
        return 1 if self.inst is None else int(self.inst.shape[0])

    @property
    def num_vertices(self) -> int:
        return self.compressed.num_vertices if self.compressed is not None else int(self.pos.shape[0])

    @property
    def num_triangles(self) -> int:
        return self.compressed.num_triangles if self.compressed is not None else int(self.idx.shape[0])

    @property
    def device(self):
        return self.compressed.qpos.device if self.compressed is not None else self.pos.device

    @staticmethod
    def from_host(m, device="cuda") -> "GpuMesh":
        """From a workloads.Mesh (numpy arrays)."""
        pos = torch.from_numpy(np.ascontiguousarray(m.pos, np.float32)).to(device)
        idx = torch.from_numpy(np.ascontiguousarray(m.idx, np.uint32).view(np.int32)).to(device)
        attrs = None if m.attrs is None else torch.from_numpy(np.ascontiguousarray(m.attrs, np.float32)).to(device)
        inst = None if m.inst is None else np.ascontiguousarray(m.inst, np.float32)
        bs = None if m.bsphere is None else np.ascontiguousarray(m.bsphere, np.float32)
        return GpuMesh(pos, idx, inst, bs, attrs)


def texture_texels(width: int, height: int, levels: int) -> int:
    """curast_texture_texels: words of an RGBA8 mip chain (0 for invalid sizes or level counts)."""
    return int(lib().curast_texture_texels(width, height, levels))


@dataclass
class Texture:
    """A mip-mapped RGBA8 texture in device memory (curast_texture): `texels` holds every level,
    level 0 first, as int32 bits of the RGBA8 words."""
    texels: torch.Tensor                    # int32 [curast_texture_texels(width, height, levels)] (cuda)
    width: int
    height: int
    levels: int

    def struct(self) -> TextureStruct:
        return TextureStruct(self.texels.data_ptr(), self.width, self.height, self.levels)


@dataclass
class CompressedGeometry:
    """Device buffers and parameters of a compressed mesh (curast_compressed, Sec. 4.6)."""
    packed: torch.Tensor                    # int32 [words] bits of the packed index stream (cuda)
    qpos: torch.Tensor                      # int16 [3 V + 1] bits of the uint16 positions, then one
                                            # padding element (cuda)
    index_min: int
    index_bits: int
    lo: np.ndarray                          # float32 [3]
    step: np.ndarray                        # float32 [3]
    num_vertices: int
    num_triangles: int

    def struct(self) -> CompressedStruct:
        c = CompressedStruct()
        c.indices = self.packed.data_ptr() if self.packed.numel() else None
        c.positions = self.qpos.data_ptr() if self.qpos.numel() else None
        c.index_min = self.index_min
        c.index_bits = self.index_bits
        for k in range(3):
            c.lo[k] = float(self.lo[k])
            c.step[k] = float(self.step[k])
        return c


def _mesh_struct(m: GpuMesh, keep: list, check: bool = True) -> MeshStruct:
    s = MeshStruct()
    if m.compressed is not None:
        if check:
            _check_cuda(m.compressed.packed, torch.int32, "packed indices")
            _check_cuda(m.compressed.qpos, torch.int16, "quantized positions")
            if m.compressed.qpos.numel() != 3 * m.compressed.num_vertices + 1:
                raise ValueError("quantized positions must hold 3 V + 1 elements")
        cs = m.compressed.struct()
        keep.append(cs)
        s.compressed = C.addressof(cs)
        s.vertices = None
        s.indices = None
        s.num_vertices = m.compressed.num_vertices
        s.num_triangles = m.compressed.num_triangles
    else:
        if check:
            _check_cuda(m.pos, torch.float32, "vertices", 3)
            _check_cuda(m.idx, torch.int32, "indices", 3)
        s.compressed = None
        s.vertices = m.pos.data_ptr() if m.pos.numel() else None
        s.num_vertices = m.pos.shape[0]
        s.indices = m.idx.data_ptr() if m.idx.numel() else None
        s.num_triangles = m.idx.shape[0]
    if m.inst is not None:
        inst = np.ascontiguousarray(m.inst, np.float32).reshape(-1, 12)
        keep.append(inst)
        s.instances = inst.ctypes.data
        s.num_instances = inst.shape[0]
    else:
        s.instances = None
        s.num_instances = 1
    bs = np.zeros(4, np.float32) if m.bsphere is None else np.asarray(m.bsphere, np.float32)
    for k in range(4):
        s.bsphere[k] = float(bs[k])
    return s


def _view_struct(vp, near, width, height, vis: Optional[torch.Tensor]) -> ViewStruct:
    v = ViewStruct()
    vp = np.ascontiguousarray(vp, np.float32).reshape(16)
    for k in range(16):
        v.view_proj[k] = float(vp[k])
    v.near_plane = float(near)
    v.width = int(width)
    v.height = int(height)
    if vis is not None:
        _check_cuda(vis, torch.int64, "visbuffer")
        if tuple(vis.shape) != (int(height), int(width)):
            raise ValueError("visbuffer must have shape [height, width]")
        v.visbuffer = vis.data_ptr()
    else:
        v.visbuffer = None
    return v


class Context:
    """A rasterizer context on the current HIP device (wraps curast_create / curast_destroy)."""

    def __init__(self, **options):
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self._h = C.c_void_p()
        opt = self._options(options)
        self._check(L.curast_create(C.byref(opt), C.byref(self._h)), owner=False)

    @staticmethod
    def _options(kw) -> Options:
        o = Options()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise ValueError(f"unknown option {k}")
            setattr(o, k, int(v))
        return o

    def _check(self, rc: int, owner: bool = True):
        if rc != OK:
            msg = lib().curast_last_error(self._h).decode() if owner and self._h else ""
            if not msg:
                msg = lib().curast_status_string(rc).decode()
            raise CurastError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            lib().curast_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- options -------------------------------------------------------------------------------
    def set_options(self, **options):
        self._check(lib().curast_set_options(self._h, C.byref(self._options(options))))

    def options(self) -> dict:
        o = Options()
        self._check(lib().curast_get_options(self._h, C.byref(o)))
        return {n: getattr(o, n) for n, _ in Options._fields_}

    # -- rasterization ---------------------------------------------------------------------------
    def rasterize(self, vertices: torch.Tensor, indices: torch.Tensor, view_proj, near: float, width: int,
                  height: int, instances: Optional[np.ndarray] = None, out: Optional[torch.Tensor] = None):
        """curast_rasterize: one mesh (optionally instanced) into one view -> int64 [H, W] keys."""
        _check_cuda(vertices, torch.float32, "vertices", 3)
        _check_cuda(indices, torch.int32, "indices", 3)
        if out is None:
            out = torch.empty((int(height), int(width)), dtype=torch.int64, device=vertices.device)
        _check_cuda(out, torch.int64, "out")
        vp = np.ascontiguousarray(view_proj, np.float32).reshape(16)
        inst = None if instances is None else np.ascontiguousarray(instances, np.float32).reshape(-1, 12)
        self._check(lib().curast_rasterize(
            self._h, vertices.data_ptr(), vertices.shape[0], indices.data_ptr(), indices.shape[0],
            None if inst is None else inst.ctypes.data, 0 if inst is None else inst.shape[0], vp.ctypes.data,
            float(near), int(width), int(height), out.data_ptr(), _stream(vertices.device)))
        return out

    def rasterize_noalloc(self, vertices: torch.Tensor, indices: torch.Tensor, view_proj, near: float, width: int,
                          height: int, out: torch.Tensor, instances: Optional[np.ndarray] = None):
        """curast_rasterize_noalloc: curast_rasterize through the library's static scratch (the
        caller passes the output buffer; at most 32 instances)."""
        _check_cuda(vertices, torch.float32, "vertices", 3)
        _check_cuda(indices, torch.int32, "indices", 3)
        _check_cuda(out, torch.int64, "out")
        if tuple(out.shape) != (int(height), int(width)):
            raise ValueError("out must have shape [height, width]")
        vp = np.ascontiguousarray(view_proj, np.float32).reshape(16)
        inst = None if instances is None else np.ascontiguousarray(instances, np.float32).reshape(-1, 12)
        self._check(lib().curast_rasterize_noalloc(
            self._h, vertices.data_ptr(), vertices.shape[0], indices.data_ptr(), indices.shape[0],
            None if inst is None else inst.ctypes.data, 0 if inst is None else inst.shape[0], vp.ctypes.data,
            float(near), int(width), int(height), out.data_ptr(), _stream(vertices.device)))
        return out

    def rasterize_meshes(self, meshes: Sequence[GpuMesh], view, out: Optional[torch.Tensor] = None):
        """curast_rasterize_meshes: a mesh list into one view (view: workloads.View-like)."""
        keep = []
        arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep) for m in meshes])
        dev = meshes[0].device if meshes else torch.device("cuda")
        if out is None:
            out = torch.empty((view.height, view.width), dtype=torch.int64, device=dev)
        vs = _view_struct(view.vp, view.near, view.width, view.height, out)
        self._check(lib().curast_rasterize_meshes(self._h, arr, len(meshes), C.byref(vs), _stream(dev)))
        return out

    def rasterize_batched(self, meshes: Sequence[GpuMesh], views, outs: Optional[List[torch.Tensor]] = None):
        """curast_rasterize_batched: the same meshes into many views in one graph launch."""
        keep = []
        arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep) for m in meshes])
        dev = meshes[0].device if meshes else torch.device("cuda")
        if outs is None:
            outs = [torch.empty((v.height, v.width), dtype=torch.int64, device=dev) for v in views]
        vs = (ViewStruct * len(views))(*[_view_struct(v.vp, v.near, v.width, v.height, o) for v, o in zip(views, outs)])
        self._check(lib().curast_rasterize_batched(self._h, arr, len(meshes), vs, len(views), _stream(dev)))
        return outs

    def project(self, mesh: GpuMesh, view, instance: int = 0, out: Optional[torch.Tensor] = None):
        """curast_project: unsnapped window positions (sx, sy, w) per vertex, float32 [V, 3]."""
        keep = []
        ms = _mesh_struct(mesh, keep)
        if out is None:
            out = torch.empty((mesh.num_vertices, 3), dtype=torch.float32, device=mesh.device)
        _check_cuda(out, torch.float32, "pos_ss", 3)
        vs = _view_struct(view.vp, view.near, view.width, view.height, None)
        self._check(lib().curast_project(self._h, C.byref(ms), int(instance), C.byref(vs), out.data_ptr(),
                                         _stream(mesh.device)))
        return out

    def compress(self, mesh: GpuMesh) -> GpuMesh:
        """curast_compress_prepare + curast_compress: the same mesh with compressed geometry
        (bit-packed indices, 16-bit positions; Sec. 4.6).  Instances, bounding sphere and
        attributes are kept."""
        keep = []
        ms = _mesh_struct(mesh, keep)
        info = CompressedStruct()
        words = C.c_uint64()
        stream = _stream(mesh.device)
        self._check(lib().curast_compress_prepare(self._h, C.byref(ms), C.byref(info), C.byref(words), stream))
        packed = torch.empty(int(words.value), dtype=torch.int32, device=mesh.device)
        qpos = torch.empty(3 * mesh.num_vertices + 1, dtype=torch.int16, device=mesh.device)
        self._check(lib().curast_compress(self._h, C.byref(ms), C.byref(info),
                                          packed.data_ptr(), qpos.data_ptr(), stream))
        geo = CompressedGeometry(packed, qpos, int(info.index_min), int(info.index_bits),
                                 np.array(info.lo[:], np.float32), np.array(info.step[:], np.float32),
                                 mesh.num_vertices, mesh.num_triangles)
        return GpuMesh(None, None, mesh.inst, mesh.bsphere, mesh.attrs, geo)

    def resolve(self, meshes: Sequence[GpuMesh], view, vis: torch.Tensor, attrs: Sequence[torch.Tensor],
                out: Optional[torch.Tensor] = None, samples_per_axis: int = 1):
        """curast_resolve: interpolated attributes float32 [H, W, C] of a visibility buffer.  With
        samples_per_axis = s > 1 (curast_resolve_supersampled) `view` and `vis` are at s times the
        output size and the result is [H / s, W / s, C], the mean of each pixel's s x s samples."""
        keep = []
        ss = int(samples_per_axis)
        arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep) for m in meshes])
        Cn = int(attrs[0].shape[1])
        for a in attrs:
            _check_cuda(a, torch.float32, "attrs", Cn)
        ptrs = (C.c_void_p * max(1, len(attrs)))(*[a.data_ptr() for a in attrs])
        if ss < 1 or view.width % ss or view.height % ss:
            raise ValueError("view size must be a multiple of samples_per_axis")
        shape = (view.height // ss, view.width // ss, Cn)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=vis.device)
        _check_cuda(out, torch.float32, "out")
        if tuple(out.shape) != shape:
            raise ValueError(f"out must have shape {list(shape)}")
        for m, a in zip(meshes, attrs):
            if a.shape[0] != m.num_vertices:
                raise ValueError("attrs[m] must have one row per vertex of mesh m")
        vs = _view_struct(view.vp, view.near, view.width, view.height, vis)
        if ss == 1:
            rc = lib().curast_resolve(self._h, arr, len(meshes), C.byref(vs), ptrs, Cn, out.data_ptr(),
                                      _stream(vis.device))
        else:
            rc = lib().curast_resolve_supersampled(self._h, arr, len(meshes), C.byref(vs), ss, ptrs, Cn,
                                                   out.data_ptr(), _stream(vis.device))
        self._check(rc)
        return out

    def texture(self, level0: torch.Tensor, levels: Optional[int] = None) -> Texture:
        """A texture from its level 0 (int32 [height, width] RGBA8 words, cuda) with the full chain
        (or `levels` levels) filled by curast_build_mips."""
        _check_cuda(level0, torch.int32, "level 0")
        if level0.dim() != 2:
            raise ValueError("level 0 must be [height, width]")
        h, w = int(level0.shape[0]), int(level0.shape[1])
        if levels is None:
            levels = max(w, h).bit_length()
        n = texture_texels(w, h, levels)
        if not n:
            raise ValueError("texture sizes must be powers of two in [1, 16384] with 1 .. 1 + log2(max) levels")
        texels = torch.empty(n, dtype=torch.int32, device=level0.device)
        texels[:w * h].copy_(level0.reshape(-1))
        self.build_mips(texels, w, h, levels)
        return Texture(texels, w, h, levels)

    def build_mips(self, texels: torch.Tensor, width: int, height: int, levels: int):
        """curast_build_mips: fills levels 1 .. levels - 1 of `texels` from its level 0."""
        _check_cuda(texels, torch.int32, "texels")
        if texels.numel() < texture_texels(width, height, levels):
            raise ValueError("texels is smaller than the mip chain")
        self._check(lib().curast_build_mips(self._h, texels.data_ptr(), width, height, levels,
                                            _stream(texels.device)))

    def resolve_textured(self, meshes: Sequence[GpuMesh], view, vis: torch.Tensor, uvs: Sequence[torch.Tensor],
                         textures: Sequence[Texture], out: Optional[torch.Tensor] = None):
        """curast_resolve_textured: RGBA float32 [H, W, 4], trilinear texture samples with the mip
        level from four ray-plane hits per pixel (Sec. 4.4)."""
        if not (len(meshes) == len(uvs) == len(textures)):
            raise ValueError("one UV array and one texture per mesh")
        keep = []
        arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep) for m in meshes])
        for m, uv in zip(meshes, uvs):
            _check_cuda(uv, torch.float32, "uvs", 2)
            if uv.shape[0] != m.num_vertices:
                raise ValueError("uvs[m] must have one row per vertex of mesh m")
        for t in textures:
            _check_cuda(t.texels, torch.int32, "texels")
            if not texture_texels(t.width, t.height, t.levels):
                raise ValueError("texture sizes must be powers of two in [1, 16384] with 1 .. 1 + log2(max) levels")
            if t.texels.numel() < texture_texels(t.width, t.height, t.levels):
                raise ValueError("texture texels smaller than its mip chain")
        ptrs = (C.c_void_p * max(1, len(uvs)))(*[u.data_ptr() for u in uvs])
        tex = (TextureStruct * max(1, len(textures)))(*[t.struct() for t in textures])
        shape = (view.height, view.width, 4)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=vis.device)
        _check_cuda(out, torch.float32, "out")
        if tuple(out.shape) != shape:
            raise ValueError(f"out must have shape {list(shape)}")
        vs = _view_struct(view.vp, view.near, view.width, view.height, vis)
        self._check(lib().curast_resolve_textured(self._h, arr, len(meshes), C.byref(vs), ptrs, tex, out.data_ptr(),
                                                  _stream(vis.device)))
        return out

    def resolve_screen(self, vis: torch.Tensor, indices: torch.Tensor, pos_ss: torch.Tensor, attrs: torch.Tensor,
                       id_base: int = 0, out: Optional[torch.Tensor] = None):
        """curast_resolve_screen: the differentiable resolve of one mesh from pos_ss."""
        _check_cuda(vis, torch.int64, "visbuffer")
        _check_cuda(indices, torch.int32, "indices", 3)
        _check_cuda(pos_ss, torch.float32, "pos_ss", 3)
        Cn = int(attrs.shape[1])
        _check_cuda(attrs, torch.float32, "attrs", Cn)
        if attrs.shape[0] != pos_ss.shape[0]:
            raise ValueError("attrs and pos_ss must have one row per vertex")
        H, W = vis.shape
        if out is None:
            out = torch.empty((H, W, Cn), dtype=torch.float32, device=vis.device)
        _check_cuda(out, torch.float32, "out")
        if tuple(out.shape) != (H, W, Cn):
            raise ValueError("out must have shape [H, W, C]")
        self._check(lib().curast_resolve_screen(self._h, vis.data_ptr(), W, H, indices.data_ptr(), indices.shape[0],
                                                int(id_base), pos_ss.data_ptr(), pos_ss.shape[0], attrs.data_ptr(), Cn,
                                                out.data_ptr(), _stream(vis.device)))
        return out

    def resolve_backward(self, vis: torch.Tensor, indices: torch.Tensor, pos_ss: torch.Tensor, attrs: torch.Tensor,
                         grad_out: torch.Tensor, grad_attr: torch.Tensor, grad_pos: Optional[torch.Tensor] = None,
                         id_base: int = 0):
        """curast_resolve_backward: accumulates into grad_attr [V, C] and grad_pos [V, 3]."""
        _check_cuda(vis, torch.int64, "visbuffer")
        _check_cuda(indices, torch.int32, "indices", 3)
        _check_cuda(pos_ss, torch.float32, "pos_ss", 3)
        Cn = int(attrs.shape[1])
        _check_cuda(attrs, torch.float32, "attrs", Cn)
        _check_cuda(grad_out, torch.float32, "grad_out")
        _check_cuda(grad_attr, torch.float32, "grad_attr", Cn)
        if grad_pos is not None:
            _check_cuda(grad_pos, torch.float32, "grad_pos", 3)
        if attrs.shape[0] != pos_ss.shape[0] or grad_attr.shape != attrs.shape or (
                grad_pos is not None and grad_pos.shape != pos_ss.shape):
            raise ValueError("attrs, pos_ss, grad_attr and grad_pos must have one row per vertex")
        H, W = vis.shape
        if tuple(grad_out.shape) != (H, W, Cn):
            raise ValueError("grad_out must have shape [H, W, C]")
        self._check(lib().curast_resolve_backward(
            self._h, vis.data_ptr(), W, H, indices.data_ptr(), indices.shape[0], int(id_base), pos_ss.data_ptr(),
            pos_ss.shape[0], attrs.data_ptr(), Cn, grad_out.data_ptr(), grad_attr.data_ptr(), _ptr(grad_pos),
            _stream(vis.device)))

    def resolve_backward_meshes(self, meshes: Sequence[GpuMesh], view, vis: torch.Tensor,
                                attrs: Sequence[torch.Tensor], grad_out: torch.Tensor,
                                grad_attrs: Sequence[Optional[torch.Tensor]],
                                grad_pos: Optional[Sequence[Optional[torch.Tensor]]] = None):
        """curast_resolve_backward_meshes: backward of resolve() over every (mesh, instance);
        accumulates into grad_attrs[m] [V_m, C] and, for one-instance meshes, grad_pos[m] [V_m, 3]
        (gradients to the window positions project() gives)."""
        keep = []
        arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep) for m in meshes])
        Cn = int(attrs[0].shape[1])
        for m, a in zip(meshes, attrs):
            _check_cuda(a, torch.float32, "attrs", Cn)
            if a.shape[0] != m.num_vertices:
                raise ValueError("attrs[m] must have one row per vertex of mesh m")
        _check_cuda(vis, torch.int64, "visbuffer")
        _check_cuda(grad_out, torch.float32, "grad_out")
        if tuple(grad_out.shape) != (view.height, view.width, Cn) or tuple(vis.shape) != (view.height, view.width):
            raise ValueError("vis must be [H, W] and grad_out [H, W, C] of the view")
        if len(attrs) != len(meshes) or len(grad_attrs) != len(meshes) or (
                grad_pos is not None and len(grad_pos) != len(meshes)):
            raise ValueError("one attrs, grad_attrs (and grad_pos) entry per mesh")
        for m, g in zip(meshes, grad_attrs):
            if g is not None:
                _check_cuda(g, torch.float32, "grad_attrs", Cn)
                if g.shape[0] != m.num_vertices:
                    raise ValueError("grad_attrs[m] must have one row per vertex of mesh m")
        if grad_pos is not None:
            for m, g in zip(meshes, grad_pos):
                if g is not None:
                    _check_cuda(g, torch.float32, "grad_pos", 3)
                    if g.shape[0] != m.num_vertices:
                        raise ValueError("grad_pos[m] must have one row per vertex of mesh m")
        n = max(1, len(meshes))
        aptr = (C.c_void_p * n)(*[a.data_ptr() for a in attrs])
        gaptr = (C.c_void_p * n)(*[_ptr(g) for g in grad_attrs])
        gpptr = None if grad_pos is None else (C.c_void_p * n)(*[_ptr(g) for g in grad_pos])
        vs = _view_struct(view.vp, view.near, view.width, view.height, vis)
        self._check(lib().curast_resolve_backward_meshes(
            self._h, arr, len(meshes), C.byref(vs), aptr, Cn, grad_out.data_ptr(), gaptr, gpptr,
            _stream(vis.device)))

    # -- tuning, statistics, timing ---------------------------------------------------------------
    def autotune(self, meshes: Sequence[GpuMesh], views, outs: Sequence[torch.Tensor],
                 cache_path: Optional[str] = None) -> dict:
        keep = []
        arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep) for m in meshes])
        vs = (ViewStruct * len(views))(*[_view_struct(v.vp, v.near, v.width, v.height, o) for v, o in zip(views, outs)])
        chosen = Options()
        dev = outs[0].device
        self._check(lib().curast_autotune(self._h, arr, len(meshes), vs, len(views),
                                          None if cache_path is None else cache_path.encode(), C.byref(chosen),
                                          _stream(dev)))
        return {n: getattr(chosen, n) for n, _ in Options._fields_}

    def stats(self) -> dict:
        s = StatsStruct()
        self._check(lib().curast_get_stats(self._h, C.byref(s)))
        return {n: int(getattr(s, n)) for n, _ in StatsStruct._fields_}

    def reset_stats(self):
        self._check(lib().curast_reset_stats(self._h))

    def stage_times(self) -> dict:
        ms = (C.c_double * 9)()
        frames = C.c_uint64()
        self._check(lib().curast_get_stage_times(self._h, ms, C.byref(frames)))
        names = ["clear", "stage1_multi", "stage1_single", "stage1_overflow", "stage2", "stage3", "resolve",
                 "resolve_backward", "frame"]
        d = {n: ms[i] for i, n in enumerate(names)}
        d["stage1"] = d["stage1_multi"] + d["stage1_single"]
        d["frames"] = int(frames.value)
        return d

    def reset_stage_times(self):
        self._check(lib().curast_reset_stage_times(self._h))


def id_bases(meshes: Sequence[GpuMesh]) -> np.ndarray:
    """curast_id_bases (host only): exclusive prefix of triangle counts over (mesh, instance)."""
    keep = []
    arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep, check=False) for m in meshes])
    n = lib().curast_id_bases(arr, len(meshes), None)
    if n < 0:
        raise CurastError(int(n), lib().curast_status_string(int(n)).decode())
    out = np.zeros(n + 1, np.int64)
    lib().curast_id_bases(arr, len(meshes), out.ctypes.data)
    return out


def plan(meshes: Sequence[GpuMesh], views, **options):
    """curast_plan (host only): (visible [pairs, n_views] uint8: 0 culled, 1 drawn, 2 drawn and
    interior; bases [pairs + 1]; counts dict)."""
    keep = []
    arr = (MeshStruct * max(1, len(meshes)))(*[_mesh_struct(m, keep, check=False) for m in meshes])
    dummy = (C.c_uint64 * max(1, len(views)))()     # distinct non-NULL buffers, never touched
    vs = (ViewStruct * len(views))()
    for i, v in enumerate(views):
        vs[i] = _view_struct(v.vp, v.near, v.width, v.height, None)
        vs[i].visbuffer = C.addressof(dummy) + 8 * i
    pairs = sum(m.num_instances for m in meshes)
    visible = np.zeros((pairs, len(views)), np.uint8)
    bases = np.zeros(pairs + 1, np.int64)
    counts = np.zeros(4, np.uint64)
    opt = Context._options(options)
    rc = lib().curast_plan(arr, len(meshes), vs, len(views), C.byref(opt), visible.ctypes.data, bases.ctypes.data,
                           counts.ctypes.data)
    if rc != OK:
        raise CurastError(rc, lib().curast_status_string(rc).decode())
    return visible, bases, dict(zip(("draws", "culled", "work_items", "tri_draws"), map(int, counts)))


class ResolveFn(torch.autograd.Function):
    """Differentiable resolve of one mesh: out = resolve(attrs, pos_ss | visibility, indices).

    forward(attrs [V, C], pos_ss [V, 3], vis [H, W] int64, indices [T, 3] int32, id_base, ctx)
    returns float32 [H, W, C]; backward returns gradients for attrs and pos_ss (visibility held
    fixed), computed by the curast_resolve_backward kernel.
    """

    @staticmethod
    def forward(fctx, attrs, pos_ss, vis, indices, id_base: int, rctx: Context):
        attrs = attrs.contiguous()
        pos_ss = pos_ss.contiguous()
        out = rctx.resolve_screen(vis, indices, pos_ss, attrs, id_base=id_base)
        fctx.save_for_backward(attrs, pos_ss, vis, indices)
        fctx.id_base = id_base
        fctx.rctx = rctx
        return out

    @staticmethod
    def backward(fctx, grad_out):
        attrs, pos_ss, vis, indices = fctx.saved_tensors
        grad_attr = torch.zeros_like(attrs)
        need_pos = fctx.needs_input_grad[1]
        grad_pos = torch.zeros_like(pos_ss) if need_pos else None
        fctx.rctx.resolve_backward(vis, indices, pos_ss, attrs, grad_out.contiguous().float(), grad_attr, grad_pos,
                                   id_base=fctx.id_base)
        return grad_attr, grad_pos, None, None, None, None

"""MI355X-native brute-force visibility-buffer rasterizer (after CuRast, arXiv 2604.21749).

The compute path is the HIP library libcurast.so (C ABI in include/curast.h); `api` is its thin
Python binding and `workloads` makes the seeded synthetic scenes.  Attributes of `api` are
re-exported lazily so that importing `workloads` alone needs neither torch nor the library.
"""
_API_NAMES = {"Context", "GpuMesh", "ResolveFn", "CurastError", "as_uint64", "id_bases", "lib", "EMPTY_KEY",
              "FLAG_NO_TINY_CULL", "FLAG_NO_EARLY_OUT", "FLAG_NO_MESH_CULL", "FLAG_STATS", "FLAG_NO_GRAPH",
              "FLAG_TIMING", "FLAG_ZERO_QUEUES"}


def __getattr__(name):
    if name in _API_NAMES:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)


__all__ = sorted(_API_NAMES)

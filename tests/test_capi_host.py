"""C-ABI library checks that need no GPU: symbols, struct layouts, host-only logic, error paths.

The host planning step (curast_plan: draw matrices, int64 ID prefix, bounding-sphere frustum cull)
is pinned against the CPU oracle: a draw the host culls must produce no fragment at all.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from paper_2604_21749_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "curast.h")


@pytest.fixture(scope="module")
def api():
    from paper_2604_21749_amd import api as A
    A.lib()
    return A


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(curast_\w+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("curast_create", "curast_rasterize", "curast_resolve", "curast_resolve_backward"):
        assert n in names


def test_library_exports_every_declared_symbol(api):
    L = api.lib()
    for name in declared_functions():
        assert hasattr(L, name), f"libcurast.so does not export {name}"
    # and the binding knows the signature of each
    assert set(declared_functions()) <= set(api.SIGNATURES), set(declared_functions()) - set(api.SIGNATURES)


def test_struct_layouts_match_the_binding(api):
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "curast.h"
#define P(t) printf(#t " %zu\n", sizeof(t))
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f))
int main(void) {
  P(curast_options); O(curast_options, flags); O(curast_options, s1_mode);
  P(curast_mesh); O(curast_mesh, num_triangles); O(curast_mesh, instances); O(curast_mesh, bsphere);
  O(curast_mesh, compressed);
  P(curast_compressed); O(curast_compressed, index_min); O(curast_compressed, lo); O(curast_compressed, step);
  P(curast_view); O(curast_view, near_plane); O(curast_view, visbuffer);
  P(curast_texture); O(curast_texture, width); O(curast_texture, levels);
  P(curast_stats); O(curast_stats, atomics); O(curast_stats, strip_union_pass);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    got = {k: int(v) for k, v in got.items()}
    assert got["curast_options"] == C.sizeof(api.Options)
    assert got["curast_options.flags"] == api.Options.flags.offset
    assert got["curast_options.s1_mode"] == api.Options.s1_mode.offset
    assert got["curast_mesh"] == C.sizeof(api.MeshStruct)
    assert got["curast_mesh.num_triangles"] == api.MeshStruct.num_triangles.offset
    assert got["curast_mesh.instances"] == api.MeshStruct.instances.offset
    assert got["curast_mesh.bsphere"] == api.MeshStruct.bsphere.offset
    assert got["curast_mesh.compressed"] == api.MeshStruct.compressed.offset
    assert got["curast_compressed"] == C.sizeof(api.CompressedStruct)
    for f in ("index_min", "lo", "step"):
        assert got[f"curast_compressed.{f}"] == getattr(api.CompressedStruct, f).offset
    assert got["curast_view"] == C.sizeof(api.ViewStruct)
    assert got["curast_view.near_plane"] == api.ViewStruct.near_plane.offset
    assert got["curast_view.visbuffer"] == api.ViewStruct.visbuffer.offset
    assert got["curast_texture"] == C.sizeof(api.TextureStruct)
    assert got["curast_texture.width"] == api.TextureStruct.width.offset
    assert got["curast_texture.levels"] == api.TextureStruct.levels.offset
    assert got["curast_stats"] == C.sizeof(api.StatsStruct)
    assert got["curast_stats.atomics"] == api.StatsStruct.atomics.offset
    assert got["curast_stats.strip_union_pass"] == api.StatsStruct.strip_union_pass.offset


def test_status_strings_and_version(api):
    L = api.lib()
    assert L.curast_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5):
        assert L.curast_status_string(code)
    assert L.curast_status_string(-99) == b"unknown status"
    assert L.curast_last_error(None) == b"no context"


def test_null_context_is_rejected_without_a_gpu(api):
    L = api.lib()
    vp = (C.c_float * 16)()
    assert L.curast_create(None, None) == api.E_INVALID
    assert L.curast_destroy(None) == api.OK
    assert L.curast_rasterize(None, None, 0, None, 0, None, 0, vp, 0.1, 8, 8, None, None) == api.E_INVALID
    assert L.curast_rasterize_meshes(None, None, 0, None, None) == api.E_INVALID
    assert L.curast_rasterize_batched(None, None, 0, None, 0, None) == api.E_INVALID
    assert L.curast_project(None, None, 0, None, None, None) == api.E_INVALID
    assert L.curast_resolve(None, None, 0, None, None, 3, None, None) == api.E_INVALID
    assert L.curast_resolve_supersampled(None, None, 0, None, 2, None, 3, None, None) == api.E_INVALID
    assert L.curast_compress_prepare(None, None, None, None, None) == api.E_INVALID
    assert L.curast_compress(None, None, None, None, None, None) == api.E_INVALID
    assert L.curast_build_mips(None, None, 8, 8, 4, None) == api.E_INVALID
    assert L.curast_resolve_textured(None, None, 0, None, None, None, None, None) == api.E_INVALID
    assert L.curast_resolve_screen(None, None, 8, 8, None, 0, 0, None, 1, None, 3, None, None) == api.E_INVALID
    assert L.curast_resolve_backward(None, None, 8, 8, None, 0, 0, None, 1, None, 3, None, None, None,
                                     None) == api.E_INVALID
    assert L.curast_autotune(None, None, 0, None, 0, None, None, None) == api.E_INVALID
    assert L.curast_get_stats(None, None) == api.E_INVALID
    assert L.curast_set_options(None, None) == api.E_INVALID


def test_texture_chain_sizes_match_the_oracle(api):
    """curast_texture_texels (host only) against the oracle's chain sizes, including invalid sizes
    and level counts (0)."""
    import oracle as O
    for w in (1, 2, 3, 8, 64, 100, 1024, 16384, 32768):
        for h in (1, 4, 6, 256, 16384):
            for levels in (0, 1, 2, 5, 11, 15, 16):
                assert api.texture_texels(w, h, levels) == O.texture_texels(w, h, levels), (w, h, levels)
    assert api.texture_texels(16384, 16384, 15) == sum((16384 >> l) ** 2 for l in range(15))
    assert api.texture_texels(4, 1, 3) == 4 + 2 + 1 and api.texture_texels(4, 1, 4) == 0


def _cpu_mesh(api, m):
    import torch
    return api.GpuMesh(torch.from_numpy(m.pos), torch.from_numpy(m.idx.view(np.int32)), m.inst, m.bsphere)


def test_id_bases_match_the_oracle(api):
    rng = np.random.default_rng(0)
    for trial in range(20):
        meshes = []
        for _ in range(int(rng.integers(1, 6))):
            T = int(rng.integers(0, 50))
            N = int(rng.integers(1, 5))
            pos = rng.normal(size=(5, 3)).astype(np.float32)
            idx = rng.integers(0, 5, (T, 3)).astype(np.uint32)
            inst = None if N == 1 and rng.uniform() < 0.5 else np.tile(
                np.eye(3, 4, dtype=np.float32).reshape(1, 12), (N, 1))
            meshes.append(W.Mesh(pos, idx, inst=inst))
        assert np.array_equal(api.id_bases([_cpu_mesh(api, m) for m in meshes]), O.id_bases(meshes))


def test_id_range_limit(api):
    """Sum of triangle instances above 2^36 is refused (the 36-bit ID field, Sec. 4.1)."""
    m = api.MeshStruct()
    m.vertices = 1
    m.num_vertices = 3
    m.indices = 1
    m.num_triangles = 1 << 32
    m.instances = None
    arr = (api.MeshStruct * 17)(*([m] * 17))
    assert api.lib().curast_id_bases(arr, 16, None) == 16       # exactly 2^36
    assert api.lib().curast_id_bases(arr, 17, None) == api.E_ID_RANGE


def test_plan_rejects_bad_views(api):
    s = W.random_tiny_scene(0)
    m = _cpu_mesh(api, s.meshes[0])
    bad = [W.View(s.views[0].vp, 0.0, 8, 8), W.View(s.views[0].vp, 0.1, 0, 8), W.View(s.views[0].vp, 0.1, 8, 20000)]
    for v in bad:
        with pytest.raises(api.CurastError):
            api.plan([m], [v])


@pytest.mark.parametrize("seed", range(6))
def test_host_cull_is_conservative(api, seed):
    """Every (mesh, instance, view) draw the host culls by bounding sphere covers no pixel in the
    oracle, and a good share of off-screen instances is culled."""
    rng = np.random.default_rng(50 + seed)
    pos, idx = W.uv_sphere(6, 12, 1.0)
    n_inst = 40
    R = W.random_rotations(rng, n_inst)
    t = rng.uniform(-12, 12, (n_inst, 3))
    t[:, 2] -= 8.0
    inst = W.instance_matrices(R, rng.uniform(0.3, 2.0, n_inst), t)
    mesh = W.Mesh(pos, idx, inst=inst, bsphere=W.bounding_sphere(pos))
    views = [W.View(W.camera((0, 0, 0), rng.normal(size=3) + np.array([0, 0, -3]), aspect=1.3), 0.05, 52, 40)
             for _ in range(3)]
    visible, bases, counts = api.plan([_cpu_mesh(api, mesh)], views)
    assert counts["culled"] + counts["draws"] == n_inst * len(views)
    assert counts["culled"] > 10
    for v, view in enumerate(views):
        for i in range(n_inst):
            one = W.Mesh(pos, idx, inst=inst[i:i + 1])
            covered = bool((O.rasterize([one], view) != O.EMPTY).any())
            if covered:
                assert visible[i, v] > 0, (i, v)
            if visible[i, v] == 2:
                # interior draws skip the per-vertex near / guard-band tests in the fast stage-1
                # path: every vertex must pass them
                ss = O.project(one, view)
                A = view.vp.astype(np.float64)
                X = np.concatenate([inst[i].reshape(3, 4).astype(np.float64), [[0, 0, 0, 1]]])
                P = np.concatenate([pos.astype(np.float64), np.ones((pos.shape[0], 1))], 1) @ (A @ X).T
                assert np.all(P[:, 3] >= view.near) and np.all(ss[:, 2] >= view.near)
                assert np.all(np.abs(P[:, 0]) <= 2 * P[:, 3]) and np.all(np.abs(P[:, 1]) <= 2 * P[:, 3])
    assert (visible == 2).sum() > 0


def test_prescaled_interior_needs_a_small_error_bound(api):
    """Interior draws take prescaled window rows only when the host's error bound for them is
    below the fast margin: the same object and camera, with the mesh's coordinates far from its
    own origin (large matrix terms against a small depth; the sphere stays well inside the
    frustum), fall back to the general fast path."""
    pos, idx = W.uv_sphere(6, 12, 1.0)
    for origin, expect in ((0.0, 2), (100.0, 2), (1e3, 1)):
        o = np.array([origin, 0.0, origin])
        p = (pos.astype(np.float64) + o + [0.0, 0.0, -6.0]).astype(np.float32)
        m = W.Mesh(p, idx, bsphere=W.bounding_sphere(p))
        view = W.View(W.camera(o, o + [0.0, 0.0, -1.0], aspect=1.0), 0.05, 640, 640)
        visible, _, _ = api.plan([_cpu_mesh(api, m)], [view])
        assert visible[0, 0] == expect, (origin, visible)
        visible, _, _ = api.plan([_cpu_mesh(api, m)], [view], flags=api.FLAG_NO_FAST_INTERIOR)
        assert visible[0, 0] == 1


def test_host_log_lines(api):
    """CURAST_LOG=1 prints the plan of a frame and every error to stderr (host only; a separate
    process, since the setting is read once)."""
    code = r'''
import numpy as np, torch
from paper_2604_21749_amd import api, workloads as W
s = W.random_tiny_scene(1)
m = api.GpuMesh(torch.from_numpy(s.meshes[0].pos), torch.from_numpy(s.meshes[0].idx.view(np.int32)),
                s.meshes[0].inst, s.meshes[0].bsphere)
api.plan([m], [s.views[0]])
try:
    api.plan([m], [W.View(s.views[0].vp, 0.0, 8, 8)])
except api.CurastError:
    pass
'''
    env = dict(os.environ, CURAST_LOG="1", PYTHONPATH=ROOT)
    r = subprocess.run([os.sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    assert re.search(r"^\[curast\] plan: 1 meshes, 1 views, \d+ draws", r.stderr, flags=re.M), r.stderr
    assert "[curast] error -1: near plane must be finite and > 0" in r.stderr, r.stderr
    env["CURAST_LOG"] = "0"
    r = subprocess.run([os.sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0 and "[curast]" not in r.stderr

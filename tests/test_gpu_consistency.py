"""GPU self-consistency (needs an MI355X): triangles with out-of-range indices produce nothing
(they never reach a vertex load), and the result does not depend on the order of the triangles:
a seeded permutation of a mesh's triangles, with the IDs mapped back, gives the same buffer."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import assert_vis_equal
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu


def _break_indices(m, seed, frac=0.01, values=None):
    """A copy of mesh m with about frac of its triangles given one index >= V (V, V + 5 or
    2^32 - 1); returns the copy and the sorted list of broken triangles."""
    rng = np.random.default_rng(seed)
    idx = m.idx.copy()
    V = m.pos.shape[0]
    bad = np.sort(rng.choice(len(idx), max(1, int(len(idx) * frac)), replace=False))
    vals = np.array(values if values is not None else [V, V + 5, 0xFFFFFFFF], np.uint64)
    idx[bad, rng.integers(0, 3, len(bad))] = vals[rng.integers(0, len(vals), len(bad))].astype(np.uint32)
    return W.Mesh(m.pos, idx, inst=m.inst, attrs=m.attrs, bsphere=m.bsphere), bad


def _instanced_sphere(n_inst=6, seed=3):
    """A UV sphere instanced side by side above the C1 sphere (in view of the C1 camera):
    centres 8 / n_inst apart in x and radii below a third of that, so no two instances intersect
    (no depth ties between them)."""
    rng = np.random.default_rng(seed)
    pos, idx = W.uv_sphere(32, 64, 1.0)
    R = W.random_rotations(rng, n_inst)
    gap = 8.0 / n_inst
    t = np.stack([-4.0 + gap * (np.arange(n_inst) + 0.5), rng.uniform(2.4, 3.6, n_inst),
                  -rng.uniform(4.0, 6.0, n_inst)], 1)
    inst = W.instance_matrices(R, rng.uniform(0.15, 0.33, n_inst) * gap, t)
    return W.Mesh(pos, idx, inst=inst, attrs=np.zeros_like(pos), bsphere=W.bounding_sphere(pos))


@pytest.mark.parametrize("opts", [{}, dict(s1_mode=1), dict(s1_multi_tris_per_thread=8),
                                  dict(s1_multi_tris_per_thread=2, flags=api.FLAG_SINGLE_STRIPS),
                                  dict(s1_mode=3), dict(flags=api.FLAG_ZERO_QUEUES),
                                  dict(flags=api.FLAG_S1_OVERLAP), dict(s1_mode=1, flags=api.FLAG_S1_OVERLAP),
                                  dict(flags=api.FLAG_EARLY_OUT_ALL)])
def test_out_of_range_indices_produce_nothing(opts):
    """R14 on every stage-1 kernel: the single-draw launch (C1 sphere and ground quad), the
    multi-draw launch with strips (an instanced sphere: broken indices split strips), the
    vertex-sharing kernel and the overflow pass."""
    c1 = W.scene_c1()
    view = c1.views[0]
    sphere, bad0 = _break_indices(c1.meshes[0], 1)
    inst, bad1 = _break_indices(_instanced_sphere(), 2, frac=0.02)
    meshes = [sphere, c1.meshes[1], inst]
    with api.Context(**opts) as c:
        vis = api.as_uint64(c.rasterize_meshes([api.GpuMesh.from_host(m) for m in meshes], view))
    ref = O.rasterize(meshes, view)
    assert_vis_equal(vis, ref, f"out-of-range indices {opts}")
    ids = O.key_id(vis[vis != O.EMPTY]).astype(np.int64)
    bases = O.id_bases(meshes)
    broken = [bad0 + bases[0]] + [bad1 + bases[2 + i] for i in range(inst.num_instances)]
    assert not np.isin(ids, np.concatenate(broken)).any(), "a broken triangle produced a fragment"
    assert (ids >= bases[2]).sum() > 1000          # the instanced spheres are drawn


def test_out_of_range_indices_compressed():
    """A compressed mesh whose index span reaches V + 5: the decoded indices are range-checked
    like plain ones."""
    c1 = W.scene_c1()
    m, _ = _break_indices(c1.meshes[0], 4, values=[c1.meshes[0].pos.shape[0] + 5])
    lo_i, bits, words = O.compress_indices(m.idx)
    lo, step = O.position_box(m.pos)
    dm = O.decompressed_mesh(m, words, lo_i, bits, O.quantize_positions(m.pos, lo, step), lo, step)
    with api.Context() as c:
        vis = api.as_uint64(c.rasterize_meshes([c.compress(api.GpuMesh.from_host(m))], c1.views[0]))
    assert_vis_equal(vis, O.rasterize([dm], c1.views[0]), "compressed, out-of-range indices")


def _permuted(m, seed):
    perm = np.random.default_rng(seed).permutation(m.num_triangles)
    return W.Mesh(m.pos, m.idx[perm], inst=m.inst, attrs=m.attrs, bsphere=m.bsphere), perm


def _remap(vis, meshes, perms):
    """Map the IDs of a buffer rendered from permuted meshes back to the original triangle
    numbers (triangle j of a permuted mesh is triangle perm[j] of the original)."""
    out = vis.copy()
    cov = vis != O.EMPTY
    ids = O.key_id(vis[cov]).astype(np.int64)
    bases = O.id_bases(meshes)
    new = ids.copy()
    pair = 0
    for m, perm in zip(meshes, perms):
        for _ in range(m.num_instances):
            lo, hi = bases[pair], bases[pair + 1]
            sel = (ids >= lo) & (ids < hi)
            new[sel] = lo + perm[ids[sel] - lo]
            pair += 1
    depth = vis[cov] >> np.uint64(36)
    out[cov] = (depth << np.uint64(36)) | new.astype(np.uint64)
    return out


@pytest.mark.parametrize("opts", [{}, dict(s1_multi_tris_per_thread=8), dict(s1_mode=3)])
def test_triangle_order_does_not_change_the_result(opts):
    """A closed jittered sphere (every covered pixel has exactly one front-facing triangle, so
    no depth ties) and an instanced sphere, both rendered with their triangles in a seeded random
    order: after mapping the IDs back the buffer equals the unpermuted one bit for bit."""
    c1 = W.scene_c1()
    view = c1.views[0]
    meshes = [c1.meshes[0], _instanced_sphere(4, seed=9)]
    permuted = [_permuted(m, 20 + i) for i, m in enumerate(meshes)]
    with api.Context(**opts) as c:
        a = api.as_uint64(c.rasterize_meshes([api.GpuMesh.from_host(m) for m in meshes], view))
        b = api.as_uint64(c.rasterize_meshes([api.GpuMesh.from_host(p) for p, _ in permuted], view))
    assert_vis_equal(a, O.rasterize(meshes, view), f"unpermuted {opts}")
    assert (a != O.EMPTY).sum() > 50000
    assert_vis_equal(_remap(b, meshes, [p for _, p in permuted]), a, f"permuted, IDs mapped back {opts}")


def test_triangle_order_heightfield_ties_only_by_id():
    """A shuffled height field in a seeded random order: depths are identical at every pixel;
    an ID may differ only where two triangles reach the same 28-bit depth (the smaller ID wins, and
    the permutation changes which is smaller), which the oracle confirms triangle by triangle."""
    hpos, hidx = W.heightfield(257, 0.1, 6)
    m = W.Mesh(hpos, hidx, bsphere=W.bounding_sphere(hpos))
    view = W.orbit_camera((0.5, 0.0, 0.5), 0.8, 0.7, 1.1, 640, 480)
    p, perm = _permuted(m, 33)
    with api.Context() as c:
        a = api.as_uint64(c.rasterize_meshes([api.GpuMesh.from_host(m)], view))
        b = api.as_uint64(c.rasterize_meshes([api.GpuMesh.from_host(p)], view))
    back = _remap(b, [m], [perm])
    assert np.array_equal(a >> np.uint64(36), back >> np.uint64(36)), "depths depend on the triangle order"
    diff = np.argwhere(a != back)
    assert len(diff) <= 50, f"{len(diff)} pixels differ by ID"
    for y, x in diff:
        ta, tb = int(O.key_id(a[y, x])), int(O.key_id(back[y, x]))
        keys = [O.rasterize([W.Mesh(hpos, hidx[[t]])], view)[y, x] for t in (ta, tb)]
        assert keys[0] >> np.uint64(36) == keys[1] >> np.uint64(36) == a[y, x] >> np.uint64(36), (y, x, ta, tb)

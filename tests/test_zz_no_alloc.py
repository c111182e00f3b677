"""GPU test of the allocation-free entry point (curast_rasterize_noalloc, needs an MI355X): its
visibility buffer must equal curast_rasterize's bit for bit (and the oracle's) on two calls in a
row, the second with a smaller input, for plain, instanced and near-clipped meshes and under
options that route triangles through every stage and through the overflow paths."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import assert_vis_equal
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu


def _instanced(n_inst, seed):
    rng = np.random.default_rng(seed)
    pos, idx = W.uv_sphere(24, 48, 1.0)
    R = W.random_rotations(rng, n_inst)
    t = np.stack([rng.uniform(-4, 4, n_inst), rng.uniform(-3, 3, n_inst), -rng.uniform(4, 20, n_inst)], 1)
    t[0] = (0.0, 0.0, -0.5)                       # crosses the near plane
    inst = W.instance_matrices(R, rng.uniform(0.5, 2.0, n_inst), t)
    return W.Mesh(pos, idx, inst=inst, bsphere=W.bounding_sphere(pos))


def _cases():
    """(mesh, view) pairs: each entry's second input is smaller than its first."""
    c1 = W.scene_c1()
    tiny = W.random_tiny_scene(5, n_tris=24, near_crossing=True, spread=6.0)
    vp = W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=300 / 200)
    return [
        [(c1.meshes[0], c1.views[0]), (tiny.meshes[0], tiny.views[0])],
        [(c1.meshes[1], c1.views[0]), (W.Mesh(c1.meshes[1].pos, c1.meshes[1].idx[:1]), W.View(c1.views[0].vp, 0.01, 97, 61))],
        [(_instanced(32, 1), W.View(vp, 0.05, 300, 200)), (_instanced(3, 2), W.View(vp, 0.05, 150, 100))],
    ]


def _run(c, mesh, view, noalloc):
    pos = torch.from_numpy(mesh.pos).cuda()
    idx = torch.from_numpy(mesh.idx.view(np.int32)).cuda()
    out = torch.full((view.height, view.width), 7, dtype=torch.int64, device="cuda")
    if noalloc:
        c.rasterize_noalloc(pos, idx, view.vp, view.near, view.width, view.height, out, instances=mesh.inst)
    else:
        c.rasterize(pos, idx, view.vp, view.near, view.width, view.height, instances=mesh.inst, out=out)
    torch.cuda.synchronize()
    return api.as_uint64(out)


@pytest.mark.parametrize("opts", [{}, dict(small_px=1, medium_px=1), dict(flags=api.FLAG_ZERO_QUEUES),
                                  dict(q2_capacity=1 << 26, q3_capacity=1 << 24, large_capacity=1 << 22),
                                  dict(s1_multi_tris_per_thread=8, flags=api.FLAG_STATS | api.FLAG_TIMING),
                                  dict(s1_mode=3), dict(flags=api.FLAG_S3_PER_PART, small_px=1)])
def test_noalloc_matches_rasterize(opts):
    with api.Context(**opts) as c:
        for pair in _cases():
            for k, (mesh, view) in enumerate(pair):          # two calls in a row, the second smaller
                got = _run(c, mesh, view, noalloc=True)
                ref = _run(c, mesh, view, noalloc=False)
                assert_vis_equal(got, ref, f"call {k} {view.width}x{view.height} {opts}")
                assert_vis_equal(got, O.rasterize([mesh], view), f"call {k} vs oracle {opts}")


def test_noalloc_rejects_more_than_32_instances():
    mesh = _instanced(33, 3)
    view = W.View(W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0)), 0.05, 64, 64)
    with api.Context() as c:
        with pytest.raises(api.CurastError):
            _run(c, mesh, view, noalloc=True)
        got = _run(c, _instanced(32, 3), view, noalloc=True)      # the context still works
        assert_vis_equal(got, O.rasterize([_instanced(32, 3)], view), "32 instances")

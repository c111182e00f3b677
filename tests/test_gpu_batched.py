"""GPU parity of the batched launch (curast_rasterize_batched: one captured hipGraph over every
(mesh, instance, view) draw; needs an MI355X).  Every view of every call is compared with the
oracle bit for bit, under the option sweep of the plain path, with compressed meshes, with queue
capacities of zero and with the per-part stage 3, on scenes that cross the near plane and hold
meshes without triangles, and over several replays of the same captured graph with eager work
between them."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import assert_vis_equal
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W
from test_gpu_parity import OPTION_SWEEP

pytestmark = pytest.mark.gpu

# uneven view sizes: square, wide, tall, a ragged 1-pixel column and a view of one tile
SIZES = [(96, 80), (257, 64), (33, 190), (1, 77), (64, 64), (150, 149)]


def _empty_mesh(n_instances=1):
    inst = None
    if n_instances > 1:
        inst = np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (n_instances, 1))
    return W.Mesh(np.zeros((3, 3), np.float32), np.zeros((0, 3), np.uint32), inst=inst,
                  attrs=np.zeros((3, 3), np.float32))


def _views(seed, n, target=(0.0, 0.0, -3.0), dist=(2.0, 6.0)):
    """n orbit cameras of uneven size around `target`; some of them sit close enough for the
    scene to cross their near plane."""
    rng = np.random.default_rng(seed)
    views = []
    for i in range(n):
        w, h = SIZES[(seed + i) % len(SIZES)]
        views.append(W.orbit_camera(target, rng.uniform(0, 2 * np.pi), rng.uniform(-0.6, 0.9),
                                    rng.uniform(*dist), w, h))
    return views


def _scene(seed):
    """Tiny random meshes (one instanced, one crossing the near plane of the first camera),
    two meshes without triangles between them, and a shuffled height-field patch."""
    a = W.random_tiny_scene(seed, n_instances=4, n_tris=30, spread=3.0)
    b = W.random_tiny_scene(seed + 50, n_tris=24, near_crossing=True, spread=6.0)
    hpos, hidx = W.heightfield(17, 0.2, seed)
    hpos = (hpos - np.array([0.5, 0.0, 0.5], np.float32)) * 4.0 + np.array([0.0, -1.0, -3.0], np.float32)
    hf = W.Mesh(hpos, hidx, attrs=np.zeros((hpos.shape[0], 3), np.float32), bsphere=W.bounding_sphere(hpos))
    meshes = [_empty_mesh(), a.meshes[0], _empty_mesh(3), b.meshes[0], hf]
    views = [b.views[0]] + _views(seed, 4)
    return meshes, views


def _check_views(c, gm, meshes, views, what):
    outs = c.rasterize_batched(gm, views)
    torch.cuda.synchronize()
    for i, (v, o) in enumerate(zip(views, outs)):
        assert_vis_equal(api.as_uint64(o), O.rasterize(meshes, v), f"{what} view {i} ({v.width}x{v.height})")
    return outs


@pytest.mark.parametrize("opts", OPTION_SWEEP)
def test_batched_under_the_option_sweep(opts):
    meshes, views = _scene(3)
    with api.Context(**opts) as c:
        gm = [api.GpuMesh.from_host(m) for m in meshes]
        _check_views(c, gm, meshes, views, f"batched {opts}")


@pytest.mark.parametrize("opts", [{}, dict(flags=api.FLAG_ZERO_QUEUES), dict(flags=api.FLAG_S3_PER_PART),
                                  dict(flags=api.FLAG_ZERO_QUEUES | api.FLAG_S3_PER_PART, small_px=1, medium_px=1),
                                  dict(s1_multi_tris_per_thread=8, s1_draws_per_item=3),
                                  dict(flags=api.FLAG_S1_OVERLAP), dict(flags=api.FLAG_EARLY_OUT_ALL)])
def test_batched_graph_replays(opts):
    """Three replays of one captured graph per scene, with new cameras (same structure) and eager
    work (fills, a plain frame) between them: every replay equals the oracle."""
    for seed in range(3):
        meshes, views = _scene(10 + seed)
        with api.Context(**opts) as c:
            gm = [api.GpuMesh.from_host(m) for m in meshes]
            outs = [torch.empty((v.height, v.width), dtype=torch.int64, device="cuda") for v in views]
            for replay in range(3):
                moved = _views(100 * seed + replay, len(views) - 1)
                cams = [views[0]] + [W.View(m.vp, m.near, v.width, v.height) for m, v in zip(moved, views[1:])]
                for o in outs:
                    o.fill_(replay)
                c.rasterize_meshes(gm, cams[0])              # eager frame between replays
                c.rasterize_batched(gm, cams, outs)
                torch.cuda.synchronize()
                for i, (v, o) in enumerate(zip(cams, outs)):
                    assert_vis_equal(api.as_uint64(o), O.rasterize(meshes, v),
                                     f"seed {seed} replay {replay} view {i} {opts}")


@pytest.mark.parametrize("opts", [{}, dict(flags=api.FLAG_ZERO_QUEUES), dict(s1_multi_tris_per_thread=2, s1_block=256)])
def test_batched_compressed_meshes(opts):
    """Compressed meshes in the batched launch render as the oracle's decompressed meshes, mixed
    with plain ones."""
    meshes, views = _scene(21)
    dec = []
    with api.Context(**opts) as c:
        gm = []
        for i, m in enumerate(meshes):
            g = api.GpuMesh.from_host(m)
            if i in (1, 4):
                g = c.compress(g)
                lo_i, bits, words = O.compress_indices(m.idx)
                lo, step = O.position_box(m.pos)
                dec.append(O.decompressed_mesh(m, words, lo_i, bits, O.quantize_positions(m.pos, lo, step), lo, step))
            else:
                dec.append(m)
            gm.append(g)
        _check_views(c, gm, dec, views, f"batched compressed {opts}")


def test_batched_one_view_and_meshes_without_triangles():
    """One view takes the graph path as well; a scene of meshes without triangles clears every
    view."""
    meshes, views = _scene(30)
    with api.Context() as c:
        gm = [api.GpuMesh.from_host(m) for m in meshes]
        for _ in range(2):
            _check_views(c, gm, meshes, views[:1], "batched single view")
        empty = [_empty_mesh(), _empty_mesh(2)]
        outs = c.rasterize_batched([api.GpuMesh.from_host(m) for m in empty], views)
        torch.cuda.synchronize()
        for o in outs:
            assert np.all(api.as_uint64(o) == O.EMPTY)

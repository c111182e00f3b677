"""GPU parity of the strip-sphere test of the multi-draw stage-1 launch (needs an MI355X): many
small instances, the regime the test is built for, and flat grids whose vertices fall exactly on
pixel centres and pixel edges (exact ties for the fill rule, boxes that just reach a centre).  A
rejected strip must cover no pixel centre, so every buffer equals the oracle's bit for bit."""
import numpy as np
import pytest

import oracle as O
from helpers import assert_vis_equal
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = [dict(s1_mode=2, s1_multi_tris_per_thread=8, s1_draws_per_item=128),
         dict(s1_mode=2, s1_multi_tris_per_thread=4, s1_draws_per_item=3),
         dict(s1_mode=2, s1_multi_tris_per_thread=2, s1_draws_per_item=37, s1_block=256),
         dict(s1_mode=0, s1_multi_tris_per_thread=8, s1_draws_per_item=1, s1_block=512),
         dict(s1_mode=2, s1_multi_tris_per_thread=8, flags=api.FLAG_ZERO_QUEUES),
         dict(s1_mode=2, s1_multi_tris_per_thread=8, flags=api.FLAG_NO_TINY_CULL),
         dict(s1_mode=4, s1_multi_tris_per_thread=8)]


def _tiny_instances(seed, n=300, width=320, height=240):
    """A noisy UV sphere instanced n times at 2 to 40 pixels across, most of it inside the view,
    some of it across the view's sides and close to the camera."""
    rng = np.random.default_rng(seed)
    pos, idx = W.uv_sphere(32, 64, 1.0)
    pos = pos * (1.0 + 0.02 * rng.standard_normal((pos.shape[0], 1))).astype(np.float32)
    R = W.random_rotations(rng, n)
    depth = rng.uniform(1.0, 12.0, n)
    xy = rng.uniform(-1.1, 1.1, (n, 2)) * depth[:, None] * np.array([width / height, 1.0]) * 0.577
    t = np.stack([xy[:, 0], xy[:, 1], -depth], 1)
    scale = rng.uniform(0.01, 0.15, n) * depth / 6.0
    inst = W.instance_matrices(R, scale, t)
    vp = W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=width / height)
    m = W.Mesh(pos.astype(np.float32), idx, inst=inst, bsphere=W.bounding_sphere(pos.astype(np.float32)))
    return [m], W.View(vp, 0.05, width, height)


def _tie_grid(seed, width=128, height=128):
    """A flat n x n grid facing the camera at depth 2 (fovy 90: view (x, y, -2) -> window
    (32 x + 64, 32 y + 64)), rows of quads in strip order, instanced with scales 1/2, 1 and 2 and
    translations of whole and half pixels, so that every vertex lands on a pixel centre or a pixel
    edge."""
    rng = np.random.default_rng(seed)
    n = 24
    step = 0.5 / 32.0                                   # half a pixel
    g = np.arange(n + 1, dtype=np.float64) * step
    vx, vy = np.meshgrid(g, g)
    pos = np.stack([vx.ravel(), vy.ravel(), np.full(vx.size, 0.0)], 1).astype(np.float32)
    tris = []
    for r in range(n):
        for c in range(n):
            a, b, cc, d = r * (n + 1) + c, r * (n + 1) + c + 1, (r + 1) * (n + 1) + c, (r + 1) * (n + 1) + c + 1
            tris += [(a, b, cc), (b, d, cc)]
    k = 40
    inst = np.zeros((k, 12), np.float32)
    for i in range(k):
        s = float(rng.choice([0.5, 1.0, 2.0]))
        tx = (int(rng.integers(-140, 120)) * 0.5 + 0.5 * int(rng.integers(0, 2))) / 32.0
        ty = (int(rng.integers(-140, 120)) * 0.5) / 32.0
        inst[i] = [s, 0, 0, tx, 0, s, 0, ty, 0, 0, s, -2.0]
    vp = W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), fovy_deg=90.0, aspect=width / height)
    m = W.Mesh(pos, np.array(tris, np.uint32), inst=inst, bsphere=W.bounding_sphere(pos))
    return [m], W.View(vp, 0.05, width, height)


@pytest.mark.parametrize("opts", MODES)
def test_sphere_strips_tiny_instances(opts):
    with api.Context(**opts) as c:
        for seed in range(3):
            meshes, view = _tiny_instances(seed)
            vis = c.rasterize_meshes([api.GpuMesh.from_host(m) for m in meshes], view)
            ref = O.rasterize(meshes, view)
            assert (ref != O.EMPTY).sum() > 2000
            assert_vis_equal(api.as_uint64(vis), ref, f"tiny instances seed {seed} {opts}")


@pytest.mark.parametrize("opts", MODES)
def test_sphere_strips_exact_ties(opts):
    flags = opts.get("flags", 0)
    rest = {k: v for k, v in opts.items() if k != "flags"}
    for seed in range(3):
        meshes, view = _tie_grid(seed)
        ref = O.rasterize(meshes, view)
        assert (ref != O.EMPTY).sum() > 1000
        # the timed kernel, then the statistics variant (which also counts the sphere passes)
        for stats in (False, True):
            with api.Context(flags=flags | (api.FLAG_STATS if stats else 0), **rest) as c:
                gm = [api.GpuMesh.from_host(m) for m in meshes]
                visible, _, _ = api.plan(gm, [view])
                assert (visible == 2).sum() > 10, "the grid instances should be interior draws"
                vis = c.rasterize_meshes(gm, view)
                assert_vis_equal(api.as_uint64(vis), ref, f"tie grid seed {seed} stats {stats} {opts}")
                if stats and rest.get("s1_mode") in (0, 2):
                    st = c.stats()
                    assert 0 < st["strip_sphere_pass"] < st["strip_draws"], st

"""GPU parity: the HIP path through the C ABI against the CPU oracle (needs an MI355X).

Visibility buffers must be bit-identical to the oracle's; resolved fp32 attributes must agree
within 1e-5 relative (floor 0.1 on the reference magnitude); every option combination and every
stage routing must give the same bytes.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu

RESOLVE_RTOL = 1e-5
RESOLVE_FLOOR = 0.1


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = api.Context()
    yield c
    c.close()


def gpu_meshes(scene):
    return [api.GpuMesh.from_host(m) for m in scene.meshes]


def assert_vis_equal(got: np.ndarray, ref: np.ndarray, what: str):
    if np.array_equal(got, ref):
        return
    bad = np.argwhere(got != ref)
    y, x = bad[0]
    raise AssertionError(f"{what}: {len(bad)} of {ref.size} pixels differ; first at (x={x}, y={y}) "
                         f"gpu={int(got[y, x]):#018x} oracle={int(ref[y, x]):#018x}")


def assert_resolve_close(got: np.ndarray, ref: np.ndarray, what: str):
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    lim = RESOLVE_RTOL * np.maximum(np.abs(ref.astype(np.float64)), RESOLVE_FLOOR)
    assert np.all(err <= lim), f"{what}: max err {err.max()} (limit {lim[np.argmax(err - lim)]})"


def test_c1_visibility_and_resolve(ctx):
    s = W.scene_c1()
    gm = gpu_meshes(s)
    view = s.views[0]
    vis = ctx.rasterize_meshes(gm, view)
    torch.cuda.synchronize()
    ref = O.rasterize(s.meshes, view)
    assert_vis_equal(api.as_uint64(vis), ref, "C1")
    out = ctx.resolve(gm, view, vis, [m.attrs for m in gm])
    ref_out = O.resolve(s.meshes, view, ref, [m.attrs for m in s.meshes])
    assert_resolve_close(out.cpu().numpy(), ref_out, "C1 resolve")
    # the ground quad crosses the near plane and covers large areas: stages 2 and 3 ran
    ids = O.key_id(ref[ref != O.EMPTY])
    assert (ids >= 262144).sum() > 50000


@pytest.mark.parametrize("variant", [
    {}, {"snap_grid": True}, {"near_crossing": True}, {"n_instances": 3}, {"spread": 8.0},
    {"near_crossing": True, "spread": 6.0, "n_tris": 24},
])
def test_random_tiny_scenes(ctx, variant):
    for seed in range(12):
        s = W.random_tiny_scene(seed, **variant)
        gm = gpu_meshes(s)
        vis = ctx.rasterize_meshes(gm, s.views[0])
        ref = O.rasterize(s.meshes, s.views[0])
        assert_vis_equal(api.as_uint64(vis), ref, f"tiny seed {seed} {variant}")


OPTION_SWEEP = [
    dict(small_px=1), dict(small_px=4096), dict(medium_px=1), dict(medium_px=1 << 20),
    dict(s1_block=64), dict(s1_block=512, s1_tris_per_thread=4), dict(s1_block=128, s1_tris_per_thread=2),
    dict(flags=api.FLAG_ZERO_QUEUES), dict(flags=api.FLAG_ZERO_QUEUES, small_px=1, medium_px=1),
    dict(flags=api.FLAG_NO_TINY_CULL | api.FLAG_NO_EARLY_OUT | api.FLAG_NO_MESH_CULL),
    dict(small_px=1, medium_px=1, s3_blocks=1, s2_waves=4), dict(q2_capacity=3, q3_capacity=5, large_capacity=2),
    dict(flags=api.FLAG_STATS | api.FLAG_TIMING),
    dict(s1_mode=1), dict(s1_mode=2), dict(s1_mode=3), dict(s1_mode=3, s1_block=64),
    dict(s1_mode=2, s1_block=512), dict(s1_mode=3, s1_block=128, s1_draws_per_item=2),
    dict(s1_mode=3, flags=api.FLAG_NO_TINY_CULL), dict(s1_mode=2, flags=api.FLAG_ZERO_QUEUES),
    dict(s1_mode=0, s1_tris_per_thread=2), dict(s1_mode=2, s1_tris_per_thread=4, s1_block=128),
    dict(s1_mode=0, s1_tris_per_thread=4, s1_block=64, small_px=2),
    dict(s1_mode=3, s1_tris_per_thread=1), dict(s1_mode=3, s1_tris_per_thread=4, flags=api.FLAG_ZERO_QUEUES),
    dict(flags=api.FLAG_S3_PER_PART), dict(flags=api.FLAG_S3_PER_PART, medium_px=1),
    dict(medium_px=1, s3_blocks=3), dict(medium_px=64, q3_capacity=7),
    dict(s1_multi_tris_per_thread=4, s1_tris_per_thread=1), dict(s1_multi_tris_per_thread=1, s1_block=512),
    dict(flags=api.FLAG_SINGLE_STRIPS), dict(flags=api.FLAG_SINGLE_STRIPS, s1_tris_per_thread=2, s1_block=64),
    dict(flags=api.FLAG_SINGLE_STRIPS | api.FLAG_NO_TINY_CULL, small_px=1),
    dict(s1_tris_per_thread=8), dict(s1_tris_per_thread=8, s1_block=512, s1_mode=1),
    dict(s1_tris_per_thread=8, s1_block=64, flags=api.FLAG_SINGLE_STRIPS),
    dict(s1_multi_tris_per_thread=8), dict(s1_multi_tris_per_thread=8, s1_block=64, flags=api.FLAG_NO_FAST_INTERIOR),
    dict(s1_multi_tris_per_thread=8, s1_block=512, s1_draws_per_item=3, flags=api.FLAG_STATS),
    dict(s1_blocks_per_cu=1), dict(s1_blocks_per_cu=1, s1_mode=1, s1_block=512),
    dict(flags=api.FLAG_S1_OVERLAP), dict(flags=api.FLAG_S1_OVERLAP | api.FLAG_ZERO_QUEUES, s1_mode=4),
    dict(flags=api.FLAG_S1_OVERLAP | api.FLAG_STATS | api.FLAG_TIMING, s1_mode=3),
    dict(s1_blocks_per_cu=3, s1_mode=3), dict(s1_blocks_per_cu=65536),
    dict(flags=api.FLAG_EARLY_OUT_ALL), dict(flags=api.FLAG_EARLY_OUT_ALL | api.FLAG_NO_EARLY_OUT, s1_mode=3),
    dict(flags=api.FLAG_EARLY_OUT_ALL | api.FLAG_ZERO_QUEUES, s1_multi_tris_per_thread=8),
    dict(s1_mode=4), dict(s1_mode=4, s1_multi_tris_per_thread=8), dict(s1_mode=2, s1_multi_tris_per_thread=8, s1_block=256),
    dict(s1_mode=4, flags=api.FLAG_ZERO_QUEUES, s1_multi_tris_per_thread=2),
]


@pytest.mark.parametrize("opts", OPTION_SWEEP)
def test_options_do_not_change_results(opts):
    s = W.scene_c1()
    ref = O.rasterize(s.meshes, s.views[0])
    with api.Context(**opts) as c:
        gm = gpu_meshes(s)
        vis = c.rasterize_meshes(gm, s.views[0])
        assert_vis_equal(api.as_uint64(vis), ref, f"C1 with {opts}")
        for seed in range(4):
            t = W.random_tiny_scene(seed, near_crossing=True, spread=6.0, n_tris=24)
            v2 = c.rasterize_meshes(gpu_meshes(t), t.views[0])
            assert_vis_equal(api.as_uint64(v2), O.rasterize(t.meshes, t.views[0]), f"tiny {seed} with {opts}")


@pytest.mark.parametrize("mode,tpt", [(0, 2), (0, 1), (0, 4), (1, 2), (2, 4), (3, 1), (3, 2), (3, 4), (2, 8), (4, 2),
                                      (4, 8)])
def test_instanced_stage1_modes(mode, tpt):
    """Instanced meshes take the first stage-1 launch (the vertex-sharing kernel with LDS
    deduplication in mode 3), at every multi-draw batch size."""
    with api.Context(s1_mode=mode, s1_draws_per_item=8, s1_multi_tris_per_thread=tpt) as c:
        for seed in range(6):
            s = W.random_tiny_scene(seed, n_instances=13, n_tris=40, spread=3.0)
            # shared vertices: rebuild the index buffer over a small vertex pool
            rng = np.random.default_rng(seed)
            m = s.meshes[0]
            m.idx = rng.integers(0, 17, m.idx.shape).astype(np.uint32)
            vis = c.rasterize_meshes(gpu_meshes(s), s.views[0])
            assert_vis_equal(api.as_uint64(vis), O.rasterize(s.meshes, s.views[0]), f"instanced seed {seed} mode {mode}")


def test_single_mesh_entry_point_matches_mesh_list(ctx):
    s = W.scene_c1()
    m = s.meshes[0]
    g = api.GpuMesh.from_host(m)
    v = s.views[0]
    vis = ctx.rasterize(g.pos, g.idx, v.vp, v.near, v.width, v.height)
    ref = O.rasterize([m], v)
    assert_vis_equal(api.as_uint64(vis), ref, "curast_rasterize")


def test_autotune_keeps_results_and_caches(tmp_path):
    s = W.scene_c1()
    view = s.views[0]
    ref = O.rasterize(s.meshes, view)
    cache = str(tmp_path / "tune.jsonl")
    with api.Context() as c:
        gm = gpu_meshes(s)
        vis = torch.empty((view.height, view.width), dtype=torch.int64, device="cuda")
        chosen = c.autotune(gm, [view], [vis], cache_path=cache)
        assert chosen["s1_block"] in (64, 128, 256, 512) and chosen["s1_mode"] in (0, 1, 2, 3)
        assert_vis_equal(api.as_uint64(c.rasterize_meshes(gm, view)), ref, f"C1 with tuned {chosen}")
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"key": "gfx950/' in lines[0]
    with api.Context() as c:                     # second context: loads the entry, no re-measuring
        again = c.autotune(gpu_meshes(s), [view], [vis], cache_path=cache)
        assert again == chosen
    assert len(open(cache).read().strip().splitlines()) == 1


@pytest.mark.parametrize("mode", [1, 2])
def test_stats_account_for_every_triangle(mode):
    """Every (triangle, draw) ends in exactly one of: a cull reason, stage-1 raster, stage 2."""
    s = W.scene_c1()
    with api.Context(flags=api.FLAG_STATS, s1_mode=mode) as c:
        gm = gpu_meshes(s)
        c.rasterize_meshes(gm, s.views[0])
        st = c.stats()
    done = (st["culled_near"] + st["culled_frustum"] + st["culled_tiny"] + st["culled_backface"] +
            st["s1_rasterized"] + st["q2_entries"])
    assert st["tri_draws"] == 262146
    assert done == st["tri_draws"], st
    assert st["q2_entries"] >= 2 and st["q3_entries"] > 0 and st["fragments"] > 0


def _strip_scene(seed):
    """Instanced meshes whose consecutive triangles form strips (UV sphere bands, unshuffled
    height-field rows), a copy with a few triangles moved out of order, degenerate duplicates and
    an odd count, drawn near and far, inside the frustum and across its sides and near plane."""
    rng = np.random.default_rng(seed)
    pos, idx = W.uv_sphere(24, 48, 1.0)
    hpos, hidx = W.heightfield(33, 0.15, 5 + seed, shuffle=False)
    hpos = hpos - np.array([0.5, 0.0, 0.5], np.float32)
    broken = idx.copy()
    moved = rng.choice(len(broken), len(broken) // 30, replace=False)
    broken[np.sort(moved)] = broken[moved]
    broken[rng.choice(len(broken), 7, replace=False), 1] = broken[rng.choice(len(broken), 7, replace=False), 0]
    broken = broken[:-1]
    n = 14
    R = W.random_rotations(rng, n)
    t = np.stack([rng.uniform(-6, 6, n), rng.uniform(-4, 4, n), -rng.uniform(2.5, 30, n)], 1)
    t[0] = (0.0, 0.0, -0.6)          # straddles the near plane
    t[1] = (9.0, 0.0, -8.0)          # straddles the frustum side
    inst = W.instance_matrices(R, rng.uniform(0.5, 2.0, n), t)
    meshes = [W.Mesh(pos, idx, inst=inst, bsphere=W.bounding_sphere(pos)),
              W.Mesh(hpos, hidx, inst=inst[::-1].copy(), bsphere=W.bounding_sphere(hpos)),
              W.Mesh(pos, broken, inst=inst[3:].copy(), bsphere=W.bounding_sphere(pos))]
    vp = W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=256 / 192)
    return W.Scene(f"strips_{seed}", meshes, [W.View(vp, 0.05, 256, 192)])


@pytest.mark.parametrize("opts", [
    {}, dict(flags=api.FLAG_NO_STRIPS), dict(flags=api.FLAG_NO_FAST_INTERIOR),
    dict(flags=api.FLAG_NO_STRIPS | api.FLAG_NO_FAST_INTERIOR), dict(s1_multi_tris_per_thread=4),
    dict(s1_multi_tris_per_thread=4, s1_block=64), dict(s1_multi_tris_per_thread=2, s1_block=512),
    dict(flags=api.FLAG_NO_TINY_CULL), dict(s1_mode=2, small_px=1, medium_px=1),
    dict(flags=api.FLAG_SINGLE_STRIPS, s1_draws_per_item=3), dict(s1_multi_tris_per_thread=8),
    dict(s1_multi_tris_per_thread=8, s1_block=64, s1_draws_per_item=5),
    dict(s1_multi_tris_per_thread=8, flags=api.FLAG_SINGLE_STRIPS, s1_tris_per_thread=8),
    dict(s1_mode=4), dict(s1_mode=4, s1_multi_tris_per_thread=8), dict(s1_mode=4, flags=api.FLAG_NO_FAST_INTERIOR),
    dict(s1_multi_tris_per_thread=8, s1_block=512, s1_draws_per_item=1),
    dict(s1_multi_tris_per_thread=2, s1_draws_per_item=200, flags=api.FLAG_ZERO_QUEUES),
])
def test_strips_and_interior_draws(opts):
    """The strip path (shared window positions and one union-box test per strip of 2, 4 or 8
    triangles) and the prescaled interior rows reject only what the exact path would:
    bit-identical to the oracle."""
    with api.Context(**opts) as c:
        for seed in range(3):
            s = _strip_scene(seed)
            gm = gpu_meshes(s)
            visible, _, counts = api.plan(gm, s.views)
            if not (opts.get("flags", 0) & api.FLAG_NO_FAST_INTERIOR):
                assert (visible == 2).sum() > 5, counts
            vis = c.rasterize_meshes(gm, s.views[0])
            assert_vis_equal(api.as_uint64(vis), O.rasterize(s.meshes, s.views[0]), f"strips seed {seed} {opts}")


@pytest.mark.parametrize("opts", [dict(s1_block=96), dict(s1_tris_per_thread=3), dict(s1_multi_tris_per_thread=16),
                                  dict(s1_mode=3, s1_multi_tris_per_thread=8), dict(s1_mode=5),
                                  dict(s1_blocks_per_cu=65537), dict(small_px=65537),
                                  dict(q2_capacity=(1 << 30) + 1)])
def test_invalid_options_are_rejected(opts):
    """curast_create / curast_set_options refuse options outside their documented ranges, and a
    refused set_options leaves the context's options as they were."""
    with pytest.raises(api.CurastError):
        api.Context(**opts).close()
    with api.Context() as c:
        before = c.options()
        with pytest.raises(api.CurastError):
            c.set_options(**opts)
        assert c.options() == before

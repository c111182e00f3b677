"""GPU edge cases of the rasterizer and resolve against the oracle (needs an MI355X): no meshes,
meshes without triangles between others (ID bases), and views of 1 x 1, ragged sizes and the
maximum width and height."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import assert_resolve_close, assert_vis_equal
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context()
    yield c
    c.close()


def _empty_mesh(n_instances=1):
    inst = None
    if n_instances > 1:
        inst = np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (n_instances, 1))
    return W.Mesh(np.zeros((3, 3), np.float32), np.zeros((0, 3), np.uint32), inst=inst,
                  attrs=np.zeros((3, 3), np.float32))


def test_no_meshes_clears_the_view(ctx):
    s = W.random_tiny_scene(1)
    vis = ctx.rasterize_meshes([], s.views[0])
    assert np.all(api.as_uint64(vis) == O.EMPTY)


@pytest.mark.parametrize("graph", [True, False])
def test_meshes_without_triangles_keep_the_id_bases(graph):
    """[empty, tiny instanced, empty x 3 instances, tiny, empty]: IDs skip nothing and the
    resolve finds the right mesh.  graph=True renders through curast_rasterize_batched (the
    captured graph, replayed on the second frame) into two views; graph=False through
    curast_rasterize_meshes (eager launches)."""
    a = W.random_tiny_scene(7, n_instances=3, n_tris=20, spread=3.0)
    b = W.random_tiny_scene(8, n_tris=12, near_crossing=True)
    meshes = [_empty_mesh(), a.meshes[0], _empty_mesh(3), b.meshes[0], _empty_mesh()]
    view = a.views[0]
    second = W.View(b.views[0].vp, b.views[0].near, 31, 45)
    with api.Context() as c:
        gm = [api.GpuMesh.from_host(m) for m in meshes]
        for _ in range(2):     # with graph=True the second frame replays the captured graph
            if graph:
                vis, vis2 = c.rasterize_batched(gm, [view, second])
                assert_vis_equal(api.as_uint64(vis2), O.rasterize(meshes, second), "second view")
            else:
                vis = c.rasterize_meshes(gm, view)
            ref = O.rasterize(meshes, view)
            assert_vis_equal(api.as_uint64(vis), ref, "meshes without triangles")
        out = c.resolve(gm, view, vis, [g.attrs for g in gm]).cpu().numpy()
        assert_resolve_close(out, O.resolve(meshes, view, ref, [m.attrs for m in meshes]), "resolve")


@pytest.mark.parametrize("w,h", [(1, 1), (1, 37), (37, 1), (65, 65), (127, 3), (16384, 40), (40, 16384)])
def test_view_sizes(ctx, w, h):
    """Ragged tiles, single rows and columns, and the maximum width and height (16384)."""
    for seed in range(3):
        s = W.random_tiny_scene(100 + seed, n_tris=10, width=w, height=h, near_crossing=seed == 2, spread=2.0)
        gm = [api.GpuMesh.from_host(m) for m in s.meshes]
        vis = ctx.rasterize_meshes(gm, s.views[0])
        ref = O.rasterize(s.meshes, s.views[0])
        assert_vis_equal(api.as_uint64(vis), ref, f"{w}x{h} seed {seed}")
        out = ctx.resolve(gm, s.views[0], vis, [g.attrs for g in gm]).cpu().numpy()
        assert_resolve_close(out, O.resolve(s.meshes, s.views[0], ref, [m.attrs for m in s.meshes]), f"{w}x{h}")


def test_maximum_view_16384_squared(ctx):
    """A 16384 x 16384 view (2 GiB visibility buffer): few triangles, most of them large, so
    stages 2 and 3 cover millions of pixels each."""
    s = W.random_tiny_scene(200, n_tris=8, width=16384, height=16384, spread=1.0)
    gm = [api.GpuMesh.from_host(m) for m in s.meshes]
    vis = ctx.rasterize_meshes(gm, s.views[0])
    ref = O.rasterize(s.meshes, s.views[0])
    got = api.as_uint64(vis)
    del vis
    torch.cuda.empty_cache()
    assert (ref != O.EMPTY).sum() > 10_000_000
    assert_vis_equal(got, ref, "16384^2")


def test_empty_compressed_mesh_renders_nothing(ctx):
    a = W.random_tiny_scene(9, n_tris=16)
    meshes = [_empty_mesh(), a.meshes[0]]
    gm = [ctx.compress(api.GpuMesh.from_host(m)) for m in meshes]
    vis = ctx.rasterize_meshes(gm, a.views[0])
    lo_i, bits, words = O.compress_indices(a.meshes[0].idx)
    lo, step = O.position_box(a.meshes[0].pos)
    dm = O.decompressed_mesh(a.meshes[0], words, lo_i, bits, O.quantize_positions(a.meshes[0].pos, lo, step), lo,
                             step)
    assert_vis_equal(api.as_uint64(vis), O.rasterize([meshes[0], dm], a.views[0]), "empty compressed mesh")


def _sliver_scene(seed, n=60, width=300, height=200):
    """Long thin triangles in every orientation (slivers, near-horizontal and near-vertical
    needles, wide flat ones) at depth 2..4, both windings."""
    rng = np.random.default_rng(seed)
    vp = W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=width / height)
    pos = []
    for t in range(n):
        z = -rng.uniform(2.0, 4.0)
        c = rng.uniform(-1.2, 1.2, 2) * (-z) * 0.5
        ang = rng.uniform(0, np.pi)
        length = rng.uniform(0.1, 1.5) * (-z) * 0.5
        width_w = rng.choice([1e-4, 1e-3, 5e-3, 0.05]) * (-z) * 0.5
        d = np.array([np.cos(ang), np.sin(ang)]) * length
        nrm = np.array([-np.sin(ang), np.cos(ang)]) * width_w
        a, b, m = c - d, c + d, c + nrm * rng.uniform(-1, 1) + d * rng.uniform(-0.9, 0.9)
        tri = [(a[0], a[1], z), (b[0], b[1], z), (m[0], m[1], z)]
        if rng.uniform() < 0.5:
            tri = tri[::-1]
        pos.extend(tri)
    pos = np.array(pos, np.float32)
    idx = np.arange(len(pos), dtype=np.uint32).reshape(-1, 3)
    m = W.Mesh(pos, idx, attrs=rng.uniform(0, 1, (len(pos), 3)).astype(np.float32))
    return W.Scene(f"slivers_{seed}", [m], [W.View(vp, 0.05, width, height)])


@pytest.mark.parametrize("opts", [dict(small_px=1, medium_px=1 << 20), dict(small_px=1),
                                  dict(small_px=1, medium_px=1 << 20, s2_waves=4)])
def test_stage2_slivers_every_orientation(opts):
    """Slivers forced through stage 2: the block traversal tests each 64-pixel block at each
    edge's maximizing corner and must never skip a covered pixel (bit-identical to the oracle),
    for narrow, flat and square block shapes."""
    with api.Context(flags=api.FLAG_STATS, **opts) as c:
        total_s2 = 0
        for seed in range(6):
            s = _sliver_scene(seed)
            gm = [api.GpuMesh.from_host(m) for m in s.meshes]
            c.reset_stats()
            vis = c.rasterize_meshes(gm, s.views[0])
            total_s2 += c.stats()["s2_rasterized"]
            assert_vis_equal(api.as_uint64(vis), O.rasterize(s.meshes, s.views[0]), f"slivers seed {seed} {opts}")
        assert total_s2 > 50


def _outside_scene():
    """A 9 x 9 grid (128 triangles, consecutive ones forming strips) seen from a camera at the
    origin looking down -z: instances wholly beyond each side of the view (|x| or |y| > 2w, so
    the fast stage-1 tests have no window position for them), wholly behind the camera, in
    front of it, crossing a side, and crossing the near plane; plus a one-instance copy beyond
    the right side (the single-draw launch)."""
    pos, idx = W.heightfield(9, 0.0, 1, shuffle=False)
    # grid plane (x, z) -> (x, -z): facing the camera, x in [0, 1], y in [-1, 0] before the offset
    face = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], np.float64)
    flat = np.eye(3)
    rows = [(face, (-0.5, 0.5, -3.0)),                  # in view
            (face, (30.0, 0.5, -3.0)), (face, (-31.0, 0.5, -3.0)),      # beyond right / left
            (face, (-0.5, 31.0, -3.0)), (face, (-0.5, -30.0, -3.0)),    # beyond top / bottom
            (face, (-0.5, 0.5, 3.0)), (face, (-0.5, 0.5, -0.05)),       # behind, before the near plane
            (face, (3.2, 0.5, -3.0)),                   # beyond the right side within 2w
            (face, (1.8, 0.5, -3.0)),                   # across the right side
            (flat, (-0.5, -0.05, -0.5))]                # across the near plane and w = 0
    R = np.stack([r for r, _ in rows])
    inst = W.instance_matrices(R, np.ones(len(rows)), np.array([t for _, t in rows]))
    attrs = np.zeros((pos.shape[0], 3), np.float32)
    multi = W.Mesh(pos, idx, inst=inst, attrs=attrs, bsphere=W.bounding_sphere(pos))
    single = W.Mesh(pos, idx, inst=W.instance_matrices(face[None], np.ones(1), np.array([[40.0, 0.5, -3.0]])),
                    attrs=attrs, bsphere=W.bounding_sphere(pos))
    view = W.View(W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=64 / 48), 0.1, 64, 48)
    return [multi, single], view


@pytest.mark.parametrize("mode", [1, 2, 3, 4])
def test_triangles_beyond_a_clip_plane(mode):
    """Triangles wholly beyond a side or the near plane, with vertices outside the fast stage-1
    range, next to triangles across a side and across the near plane (rasterized, or clipped in
    stage 2): every stage-1 mode's image equals the oracle's.  The exact-only mode culls the
    former in the classification (near and side culls counted)."""
    meshes, view = _outside_scene()
    ref = O.rasterize(meshes, view)
    assert (ref != O.EMPTY).sum() > 100
    with api.Context(flags=api.FLAG_STATS, s1_mode=mode, s1_multi_tris_per_thread=4) as c:
        gm = [api.GpuMesh.from_host(m) for m in meshes]
        vis = c.rasterize_meshes(gm, view)
        assert_vis_equal(api.as_uint64(vis), ref, f"s1_mode {mode}")
        st = c.stats()
    if mode == 1:
        assert st["culled_frustum"] > 0 and st["culled_near"] > 0, st


def test_clip_plane_bits_reject_strips_before_the_exact_path():
    """Union-box strips (s1_mode 4) whose vertices all lie beyond one clip plane are rejected from
    the clip-plane bits of their vertices, so that few near and side culls are left for the
    classification, against all of them with the exact path alone (s1_mode 1)."""
    meshes, view = _outside_scene()
    left = {}
    for mode in (1, 4):
        with api.Context(flags=api.FLAG_STATS, s1_mode=mode, s1_multi_tris_per_thread=4) as c:
            c.rasterize_meshes([api.GpuMesh.from_host(m) for m in meshes], view)
            st = c.stats()
        left[mode] = st["culled_frustum"] + st["culled_near"]
    assert left[1] >= 128 and 10 * left[4] < left[1], left

"""GPU parity of compressed geometry (Sec. 4.6; needs an MI355X): the library's compression
against the oracle's, bit for bit, and rendering / resolving / projecting a compressed mesh against
the oracle on the decompressed mesh it stands for."""
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


def oracle_compress(m):
    lo_i, bits, words = O.compress_indices(m.idx)
    lo, step = O.position_box(m.pos)
    return lo_i, bits, words, O.quantize_positions(m.pos, lo, step), lo, step


def decompressed(m):
    """The mesh the compressed form of m renders as, from the oracle's own compression."""
    lo_i, bits, words, q, lo, step = oracle_compress(m)
    return O.decompressed_mesh(m, words, lo_i, bits, q, lo, step)


def _meshes():
    s = W.scene_c1()
    hpos, hidx = W.heightfield(33, 0.15, 5, shuffle=False)
    t = W.random_tiny_scene(4, n_instances=5, n_tris=40, spread=3.0)
    return s, [s.meshes[0], s.meshes[1], W.Mesh(hpos, hidx, bsphere=W.bounding_sphere(hpos)), t.meshes[0]]


def _edge_meshes():
    """Degenerate inputs: no geometry at all, one repeated index (span 0: 1 bit), a flat axis
    (step 0), and indices spanning a 2^20-vertex buffer (20 bits, values across word boundaries)."""
    rng = np.random.default_rng(11)
    flat = rng.uniform(-1, 1, size=(50, 3)).astype(np.float32)
    flat[:, 2] = 0.25
    big = rng.uniform(-2, 2, size=(1 << 20, 3)).astype(np.float32)
    big_idx = rng.integers(0, 1 << 20, size=(700, 3)).astype(np.uint32)
    big_idx[0] = (0, (1 << 20) - 1, 5)
    return [W.Mesh(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.uint32)),
            W.Mesh(flat, np.full((7, 3), 13, np.uint32)),
            W.Mesh(flat, rng.integers(0, 50, size=(33, 3)).astype(np.uint32)),
            W.Mesh(big, big_idx)]


def test_compression_matches_the_oracle_bit_for_bit(ctx):
    _, meshes = _meshes()
    for m in meshes + _edge_meshes():
        g = ctx.compress(api.GpuMesh.from_host(m))
        lo_i, bits, words, q, lo, step = oracle_compress(m)
        c = g.compressed
        assert (c.index_min, c.index_bits) == (lo_i, bits)
        assert np.array_equal(c.lo, lo) and np.array_equal(c.step, step)
        assert np.array_equal(c.packed.cpu().numpy().view(np.uint32), words)
        qp = c.qpos.cpu().numpy().view(np.uint16)
        assert qp.shape == (3 * len(m.pos) + 1,) and qp[-1] == 0
        assert np.array_equal(qp[:-1].reshape(-1, 3), q)
        assert np.array_equal(decompressed(m).idx, m.idx)


@pytest.mark.parametrize("opts", [{}, dict(s1_mode=1), dict(s1_mode=3), dict(flags=api.FLAG_NO_STRIPS),
                                  dict(flags=api.FLAG_SINGLE_STRIPS), dict(small_px=1, medium_px=1),
                                  dict(s1_tris_per_thread=8)])
def test_compressed_meshes_render_as_their_decompressed_form(ctx, opts):
    s, meshes = _meshes()
    with api.Context(**opts) as c:
        plain = [api.GpuMesh.from_host(m) for m in meshes]
        comp = [c.compress(g) for g in plain]
        # C1 (sphere + ground quad crossing the near plane) fully compressed, then mixed
        for gm, hm in ((comp[:2], [decompressed(m) for m in meshes[:2]]),
                       ([comp[0], plain[1]], [decompressed(meshes[0]), meshes[1]])):
            vis = c.rasterize_meshes(gm, s.views[0])
            assert_vis_equal(api.as_uint64(vis), O.rasterize(hm, s.views[0]), f"compressed C1 {opts}")
        # instanced tiny scene and a height-field patch
        t = W.random_tiny_scene(4, n_instances=5, n_tris=40, spread=3.0)
        hm = [decompressed(meshes[3])]
        vis = c.rasterize_meshes([comp[3]], t.views[0])
        assert_vis_equal(api.as_uint64(vis), O.rasterize(hm, t.views[0]), f"compressed instanced {opts}")


def test_compressed_resolve_and_project(ctx):
    s, meshes = _meshes()
    comp = [ctx.compress(api.GpuMesh.from_host(m)) for m in meshes[:2]]
    hm = [decompressed(m) for m in meshes[:2]]
    view = s.views[0]
    vis = ctx.rasterize_meshes(comp, view)
    out = ctx.resolve(comp, view, vis, [g.attrs for g in comp]).cpu().numpy()
    ref_vis = O.rasterize(hm, view)
    assert_resolve_close(out, O.resolve(hm, view, ref_vis, [m.attrs for m in meshes[:2]]), "compressed resolve")
    for g, m in zip(comp, hm):
        assert np.array_equal(ctx.project(g, view).cpu().numpy(), O.project(m, view))

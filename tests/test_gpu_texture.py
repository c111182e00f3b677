"""GPU parity of the textured resolve (Sec. 4.4, "Shading and Mip Mapping"; needs an MI355X):
mip chains bit for bit, and textured resolves of plain, compressed and instanced meshes against
the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu

# The two sides run the same binary32 steps in the same order; they may differ only where the
# level of detail goes through log2 (an ulp of the level moves the blend by ~1e-7).
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = api.Context()
    yield c
    c.close()


def _as_i32(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("w,h,levels", [(1, 1, 1), (8, 2, 4), (64, 64, 7), (256, 128, 9), (1024, 1024, 11),
                                        (2048, 16, 12)])
def test_mip_chain_bit_exact(ctx, w, h, levels):
    rng = np.random.default_rng(w * 7 + h)
    level0 = rng.integers(0, 1 << 32, size=(h, w), dtype=np.uint64).astype(np.uint32)
    tex = ctx.texture(_as_i32(level0), levels)
    assert tex.texels.numel() == api.texture_texels(w, h, levels) == O.texture_texels(w, h, levels)
    assert np.array_equal(tex.texels.cpu().numpy().view(np.uint32), O.build_mips(level0, levels))


def _textured_c1():
    s = W.scene_c1()
    sphere, ground = s.meshes
    uvs = [W.planar_uv(sphere.pos, (0, 1), 0.5, 0.5), W.planar_uv(ground.pos, (0, 2), 0.4, 0.0)]
    texs = [W.texture_rgba8(256, 256, 71), W.texture_rgba8(512, 128, 72, lines=16)]
    return s, uvs, texs


def _check(got: np.ndarray, ref: np.ndarray, what: str):
    err = np.abs(got.astype(np.float64) - ref)
    assert err.max() <= TOL, f"{what}: max |err| {err.max()} at {np.unravel_index(err.argmax(), err.shape)}"


@pytest.mark.parametrize("compressed", [False, True])
def test_textured_resolve_c1(ctx, compressed):
    """C1: the jittered sphere and the ground quad that crosses the near plane, one texture each."""
    s, uvs, texs = _textured_c1()
    view = s.views[0]
    gm = [api.GpuMesh.from_host(m) for m in s.meshes]
    hm = list(s.meshes)
    if compressed:
        # the library's compression equals the oracle's bit for bit (test_gpu_compress); the
        # expected meshes come from the oracle's own
        gm = [ctx.compress(g) for g in gm]
        hm = []
        for m in s.meshes:
            lo_i, bits, words = O.compress_indices(m.idx)
            lo, step = O.position_box(m.pos)
            hm.append(O.decompressed_mesh(m, words, lo_i, bits, O.quantize_positions(m.pos, lo, step), lo, step))
    vis = ctx.rasterize_meshes(gm, view)
    ref_vis = O.rasterize(hm, view)
    assert np.array_equal(api.as_uint64(vis), ref_vis)
    gt = [ctx.texture(_as_i32(t)) for t in texs]
    out = ctx.resolve_textured(gm, view, vis, [torch.from_numpy(u).cuda() for u in uvs], gt).cpu().numpy()
    chains = [(O.build_mips(t, g.levels), g.width, g.height, g.levels) for t, g in zip(texs, gt)]
    ref = O.resolve_textured(hm, view, ref_vis, uvs, chains)
    _check(out, ref, f"C1 textured (compressed={compressed})")
    covered = ref_vis != O.EMPTY
    assert np.all(out[~covered] == 0) and np.all(out[covered][:, 3] > 0.99)


def test_textured_resolve_instanced_and_shared_texture(ctx):
    """Instanced tiny meshes and a second mesh sharing one texture; levels fewer than the maximum."""
    t = W.random_tiny_scene(5, n_instances=6, n_tris=40, spread=3.0)
    u = W.random_tiny_scene(105, n_tris=20, near_crossing=True)
    meshes = [t.meshes[0], u.meshes[0]]
    view = t.views[0]
    gm = [api.GpuMesh.from_host(m) for m in meshes]
    vis = ctx.rasterize_meshes(gm, view)
    ref_vis = O.rasterize(meshes, view)
    assert np.array_equal(api.as_uint64(vis), ref_vis)
    uvs = [W.planar_uv(m.pos, (0, 1), 3.0, 0.25) for m in meshes]
    tex = W.texture_rgba8(128, 64, 73, lines=8)
    g = ctx.texture(_as_i32(tex), 5)
    out = ctx.resolve_textured(gm, view, vis, [torch.from_numpy(x).cuda() for x in uvs], [g, g]).cpu().numpy()
    chain = (O.build_mips(tex, 5), 128, 64, 5)
    _check(out, O.resolve_textured(meshes, view, ref_vis, uvs, [chain, chain]), "instanced textured")


def test_textured_resolve_level_of_detail_readback(ctx):
    """The ground quad alone with a level-constant chain: the output is the level of detail (x20);
    GPU and oracle agree at every covered pixel."""
    s = W.scene_c1()
    ground = s.meshes[1]
    view = s.views[0]
    g = api.GpuMesh.from_host(ground)
    vis = ctx.rasterize_meshes([g], view)
    ref_vis = O.rasterize([ground], view)
    assert np.array_equal(api.as_uint64(vis), ref_vis)
    uv = W.planar_uv(ground.pos, (0, 2), 0.4, 0.5)
    L = 9
    chain = np.zeros(O.texture_texels(256, 256, L), np.uint32)
    off = 0
    for lv in range(L):
        hl, wl = O.level_shape(256, 256, lv)
        chain[off:off + hl * wl] = np.uint32(20 * lv * 0x01010101)
        off += hl * wl
    tex = api.Texture(_as_i32(chain), 256, 256, L)
    out = ctx.resolve_textured([g], view, vis, [torch.from_numpy(uv).cuda()], [tex]).cpu().numpy()
    ref = O.resolve_textured([ground], view, ref_vis, [uv], [(chain, 256, 256, L)])
    _check(out, ref, "level readback")
    lod = out[..., 0][ref_vis != O.EMPTY] * 255 / 20
    assert lod.max() > 4.0 and lod.min() < 1.0


def test_textured_resolve_rejects_bad_textures(ctx):
    s = W.scene_c1()
    g = api.GpuMesh.from_host(s.meshes[1])
    vis = ctx.rasterize_meshes([g], s.views[0])
    uv = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    bad = api.Texture(torch.zeros(100, dtype=torch.int32, device="cuda"), 6, 4, 1)
    with pytest.raises(ValueError):
        ctx.resolve_textured([g], s.views[0], vis, [uv], [bad])
    with pytest.raises(ValueError):
        ctx.texture(torch.zeros((3, 4), dtype=torch.int32, device="cuda"))

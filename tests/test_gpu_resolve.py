"""GPU parity of the resolve family (needs an MI355X): project, resolve, screen resolve, backward."""
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


def test_project_is_bit_exact(ctx):
    s = W.scene_c1()
    for m in s.meshes:
        g = api.GpuMesh.from_host(m)
        got = ctx.project(g, s.views[0]).cpu().numpy()
        assert np.array_equal(got, O.project(m, s.views[0]))
    t = W.random_tiny_scene(3, n_instances=5)
    g = api.GpuMesh.from_host(t.meshes[0])
    for i in range(5):
        assert np.array_equal(ctx.project(g, t.views[0], instance=i).cpu().numpy(),
                              O.project(t.meshes[0], t.views[0], instance=i))


@pytest.mark.parametrize("seed", range(4))
def test_resolve_instanced_multimesh(ctx, seed):
    scenes = [W.random_tiny_scene(seed, n_instances=4, n_tris=30, spread=3.0),
              W.random_tiny_scene(seed + 100, n_tris=20, near_crossing=True)]
    meshes = [scenes[0].meshes[0], scenes[1].meshes[0]]
    view = scenes[0].views[0]
    gm = [api.GpuMesh.from_host(m) for m in meshes]
    vis = ctx.rasterize_meshes(gm, view)
    ref = O.rasterize(meshes, view)
    assert_vis_equal(api.as_uint64(vis), ref, f"multi-mesh seed {seed}")
    out = ctx.resolve(gm, view, vis, [g.attrs for g in gm]).cpu().numpy()
    assert_resolve_close(out, O.resolve(meshes, view, ref, [m.attrs for m in meshes]), "multi-mesh resolve")


def test_screen_resolve_equals_resolve_and_ignores_other_meshes(ctx):
    s = W.scene_c1()
    view = s.views[0]
    gm = [api.GpuMesh.from_host(m) for m in s.meshes]
    vis = ctx.rasterize_meshes(gm, view)
    full = ctx.resolve(gm, view, vis, [g.attrs for g in gm]).cpu().numpy()
    ids = O.key_id(api.as_uint64(vis))
    covered = api.as_uint64(vis) != O.EMPTY
    # the ground quad alone, as mesh 1 with id_base = T_sphere
    g = gm[1]
    pss = ctx.project(g, view)
    out = ctx.resolve_screen(vis, g.idx, pss, g.attrs, id_base=262144).cpu().numpy()
    ground = covered & (ids >= 262144)
    assert ground.sum() > 50000
    assert np.array_equal(out[ground], full[ground])
    assert np.all(out[~ground] == 0)
    ref = O.resolve_screen(api.as_uint64(vis), s.meshes[1].idx, 262144, pss.cpu().numpy(), s.meshes[1].attrs)
    assert np.array_equal(out, ref)


def test_backward_small_scene_vs_fp64(ctx):
    s = W.scene_c5(n=256)
    m = s.meshes[0]
    view = W.View(s.views[0].vp, s.views[0].near, 200, 160)
    g = api.GpuMesh.from_host(m)
    vis = ctx.rasterize_meshes([g], view)
    pss = ctx.project(g, view)
    rng = np.random.default_rng(4)
    gout = rng.normal(size=(view.height, view.width, 3)).astype(np.float32)
    ga = torch.zeros_like(g.attrs)
    gp = torch.zeros_like(pss)
    ctx.resolve_backward(vis, g.idx, pss, g.attrs, torch.from_numpy(gout).cuda(), ga, gp)
    ra, rp = O.resolve_screen_backward_f64(api.as_uint64(vis), m.idx, 0, pss.cpu().numpy(), m.attrs,
                                           gout.astype(np.float64))
    for got, ref, what in ((ga.cpu().numpy(), ra, "attrs"), (gp.cpu().numpy(), rp, "positions")):
        scale = np.maximum(np.abs(ref), 1e-3 * np.sqrt(np.mean(ref ** 2)))
        err = np.abs(got.astype(np.float64) - ref) / scale
        assert err.max() <= 1e-3, f"{what}: {err.max()}"
    # pixels of other meshes (id_base shifted past every ID) contribute nothing
    ga2 = torch.zeros_like(g.attrs)
    ctx.resolve_backward(vis, g.idx, pss, g.attrs, torch.from_numpy(gout).cuda(), ga2, None, id_base=1 << 30)
    assert float(ga2.abs().sum()) == 0.0


@pytest.mark.parametrize("k,size", [(1, 256), (2, 256), (4, 96)])
def test_supersampled_resolve(ctx, k, size):
    """curast_resolve_supersampled against the oracle's per-sample resolve and box filter, on the
    C1 scene rasterized at k times the output size."""
    s = W.scene_c1()
    hi = W.View(s.views[0].vp, s.views[0].near, size * k, size * k)
    gm = [api.GpuMesh.from_host(m) for m in s.meshes]
    vis = ctx.rasterize_meshes(gm, hi)
    ref_vis = O.rasterize(s.meshes, hi)
    assert_vis_equal(api.as_uint64(vis), ref_vis, f"C1 at {k}x")
    out = ctx.resolve(gm, hi, vis, [g.attrs for g in gm], samples_per_axis=k).cpu().numpy()
    assert out.shape == (size, size, 3)
    ref = O.resolve_supersampled(s.meshes, hi, ref_vis, [m.attrs for m in s.meshes], k)
    assert_resolve_close(out, ref, f"supersampled resolve {k}x{k}")
    if k == 1:
        assert np.array_equal(out, ctx.resolve(gm, hi, vis, [g.attrs for g in gm]).cpu().numpy())


def _empty_mesh(n_instances=1):
    inst = None if n_instances == 1 else np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (n_instances, 1))
    return W.Mesh(np.zeros((3, 3), np.float32), np.zeros((0, 3), np.uint32), inst=inst,
                  attrs=np.zeros((3, 3), np.float32))


def _backward_meshes_reference(meshes, view, vis, attrs, gout):
    """fp64 reference from oracle values only: for every (mesh, instance), the oracle's window
    positions and its one-mesh backward at that instance's ID range, attribute gradients summed
    over the instances of a mesh; position gradients for one-instance meshes."""
    bases = O.id_bases(meshes)
    ga, gp, pair = [], [], 0
    for m, a in zip(meshes, attrs):
        acc_a = np.zeros(a.shape, np.float64)
        acc_p = np.zeros((m.pos.shape[0], 3), np.float64)
        for i in range(m.num_instances):
            if m.num_triangles:
                pss = O.project(m, view, instance=i)
                ra, rp = O.resolve_screen_backward_f64(vis, m.idx, int(bases[pair]), pss, a, gout)
                acc_a += ra
                acc_p += rp
            pair += 1
        ga.append(acc_a)
        gp.append(acc_p if m.num_instances == 1 else None)
    return ga, gp


def _assert_grads(got, ref, what):
    scale = np.maximum(np.abs(ref), 1e-3 * np.sqrt(np.mean(ref ** 2)) + 1e-30)
    err = np.abs(got.astype(np.float64) - ref) / scale
    assert err.max() <= 1e-3, f"{what}: {err.max()}"


@pytest.mark.parametrize("seed,C", [(0, 3), (1, 3), (2, 5), (3, 1)])
def test_backward_meshes_matches_the_oracle(ctx, seed, C):
    """curast_resolve_backward_meshes on a multi-mesh scene with an instanced mesh, a mesh crossing
    the near plane and meshes without triangles (one of them instanced), every input (visibility,
    attributes, upstream gradient) from the oracle or the seeded generator."""
    a = W.random_tiny_scene(seed, n_instances=4, n_tris=30, spread=3.0)
    b = W.random_tiny_scene(seed + 100, n_tris=20, near_crossing=True)
    meshes = [_empty_mesh(), a.meshes[0], _empty_mesh(3), b.meshes[0]]
    view = a.views[0]
    rng = np.random.default_rng(40 + seed)
    attrs = [rng.normal(size=(m.pos.shape[0], C)).astype(np.float32) for m in meshes]
    vis = O.rasterize(meshes, view)
    assert (vis != O.EMPTY).sum() > 200
    gout = rng.normal(size=(view.height, view.width, C)).astype(np.float32)
    gm = [api.GpuMesh.from_host(m) for m in meshes]
    ta = [torch.from_numpy(x).cuda() for x in attrs]
    ga = [torch.zeros_like(x) for x in ta]
    gp = [torch.zeros((m.pos.shape[0], 3), dtype=torch.float32, device="cuda") if m.num_instances == 1 else None
          for m in meshes]
    tvis = torch.from_numpy(vis.view(np.int64)).cuda()
    ctx.resolve_backward_meshes(gm, view, tvis, ta, torch.from_numpy(gout).cuda(), ga, gp)
    ra, rp = _backward_meshes_reference(meshes, view, vis, attrs, gout.astype(np.float64))
    for m in range(len(meshes)):
        _assert_grads(ga[m].cpu().numpy(), ra[m], f"attrs of mesh {m}")
        if gp[m] is not None:
            _assert_grads(gp[m].cpu().numpy(), rp[m], f"positions of mesh {m}")
    assert float(ga[1].abs().sum()) > 0 and float(ga[3].abs().sum()) > 0
    # the one-mesh form on the one-instance mesh gives the same position gradients
    g3 = gm[3]
    ga1 = torch.zeros_like(ta[3])
    gp1 = torch.zeros_like(gp[3])
    base = int(O.id_bases(meshes)[1 + 4 + 3])
    ctx.resolve_backward(tvis, g3.idx, ctx.project(g3, view), ta[3], torch.from_numpy(gout).cuda(), ga1, gp1,
                         id_base=base)
    _assert_grads(gp1.cpu().numpy(), rp[3], "one-mesh form, positions")
    _assert_grads(ga1.cpu().numpy(), ra[3], "one-mesh form, attrs")


def test_backward_meshes_rejects_position_gradients_of_instanced_meshes(ctx):
    a = W.random_tiny_scene(5, n_instances=3, n_tris=10)
    m = a.meshes[0]
    view = a.views[0]
    g = api.GpuMesh.from_host(m)
    vis = ctx.rasterize_meshes([g], view)
    attrs = torch.zeros((m.pos.shape[0], 3), dtype=torch.float32, device="cuda")
    gout = torch.zeros((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(api.CurastError):
        ctx.resolve_backward_meshes([g], view, vis, [attrs], gout, [torch.zeros_like(attrs)],
                                    [torch.zeros((m.pos.shape[0], 3), dtype=torch.float32, device="cuda")])
    ctx.resolve_backward_meshes([g], view, vis, [attrs], gout, [torch.zeros_like(attrs)], [None])

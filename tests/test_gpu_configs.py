"""GPU parity at the full sizes of the five workloads, in the launch configuration bench.py times.

C2 and C3 compare the whole visibility buffer with the full oracle (C3: 9.1G triangle instances,
about a minute of CPU time on 16 cores).  C4 checks the batched graph launch view by view against
plain launches over several graph replays, and every view against the oracle.  C5 checks the
differentiable resolve: forward, fp64 reference gradients under an upstream gradient formed from
oracle values only, the autograd wrapper, and central differences.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import assert_resolve_close, assert_vis_equal, oracle_threads
from paper_2604_21749_amd import api
from paper_2604_21749_amd import workloads as W

pytestmark = pytest.mark.gpu


def gpu_meshes(scene):
    return [api.GpuMesh.from_host(m) for m in scene.meshes]


def test_c2_full_parity():
    s = W.scene_c2()
    view = s.views[0]
    with api.Context() as c:
        gm = gpu_meshes(s)
        vis = c.rasterize_meshes(gm, view)
        out = c.resolve(gm, view, vis, [m.attrs for m in gm])
        got = api.as_uint64(vis)
        got_out = out.cpu().numpy()
    ref = O.rasterize(s.meshes, view, threads=oracle_threads())
    assert_vis_equal(got, ref, "C2")
    assert (ref != O.EMPTY).sum() > 400000
    assert_resolve_close(got_out, O.resolve(s.meshes, view, ref, [m.attrs for m in s.meshes],
                                            threads=oracle_threads()), "C2 resolve")


@pytest.mark.timeout(900)
def test_c3_full_parity():
    s = W.scene_c3()
    view = s.views[0]
    # the library defaults, then the options the autotuner picks (what the benchmark times)
    frames = []
    with api.Context() as c:
        gm = gpu_meshes(s)
        for label in ("defaults", "autotuned"):
            if label == "autotuned":
                tuned = c.autotune(gm, [view], [torch.empty((view.height, view.width), dtype=torch.int64,
                                                            device="cuda")])
                print(f"[c3] autotuned options {tuned}", flush=True)
            vis = c.rasterize_meshes(gm, view)
            out = c.resolve(gm, view, vis, [m.attrs for m in gm])
            frames.append((label, api.as_uint64(vis), out.cpu().numpy()))
            del vis, out
        del gm
    torch.cuda.empty_cache()
    print(f"[c3] GPU frames done, running the oracle on {oracle_threads()} threads", flush=True)
    ref = O.rasterize(s.meshes, view, threads=oracle_threads())
    ids = O.key_id(ref[ref != O.EMPTY]).astype(np.int64)
    assert (ids >= s.meshes[0].num_triangles).sum() > 1000      # instanced spheres are visible
    ref_out = O.resolve(s.meshes, view, ref, [m.attrs for m in s.meshes], threads=oracle_threads())
    for label, got, got_out in frames:
        assert_vis_equal(got, ref, f"C3 ({label})")
        assert_resolve_close(got_out, ref_out, f"C3 resolve ({label})")


@pytest.mark.timeout(900)
def test_c4_batched_graph_matches_plain_and_oracle():
    s = W.scene_c4()
    views = s.views
    with api.Context() as c:
        gm = gpu_meshes(s)
        plain = [c.rasterize_meshes(gm, v) for v in views]
        torch.cuda.synchronize()
        plain_h = [api.as_uint64(p) for p in plain]
        outs = [torch.empty_like(p) for p in plain]
        rng = np.random.default_rng(7)
        for replay in range(3):
            for o in outs:
                o.fill_(0)                        # eager work between replays
            torch.cuda.synchronize()
            c.rasterize_batched(gm, views, outs)
            torch.cuda.synchronize()
            for i, o in enumerate(outs):
                assert_vis_equal(api.as_uint64(o), plain_h[i], f"C4 replay {replay} view {i}")
        # a replay with different cameras (same structure): the graph is reused with new descriptors
        moved = [W.orbit_camera((0.5, 0.0, 0.5), rng.uniform(0, 6.28), rng.uniform(0.4, 1.1), rng.uniform(0.4, 1.4),
                                v.width, v.height) for v in views]
        c.rasterize_batched(gm, moved, outs)
        torch.cuda.synchronize()
        for i in (0, 17, 63):
            ref_plain = api.as_uint64(c.rasterize_meshes(gm, moved[i]))
            assert_vis_equal(api.as_uint64(outs[i]), ref_plain, f"C4 moved view {i}")
        # the options the autotuner picks for the batched frame (what the benchmark times)
        tuned = c.autotune(gm, views, outs)
        print(f"[c4] autotuned options {tuned}", flush=True)
        c.rasterize_batched(gm, views, outs)
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert_vis_equal(api.as_uint64(o), plain_h[i], f"C4 autotuned view {i}")
    # every view against the oracle (the batched frames equal these view by view, above)
    for i, v in enumerate(views):
        ref = O.rasterize(s.meshes, v, threads=oracle_threads())
        assert_vis_equal(plain_h[i], ref, f"C4 view {i} ({v.width}x{v.height}) vs oracle")


def _c5_oracle():
    """C5 from the oracle alone: visibility buffer, screen positions, fp32 image and the upstream
    gradient of L = sum over covered pixels of (out - target)^2, g = 2 (out - target) formed in
    fp32 from the oracle's fp32 image (0 on empty pixels)."""
    s = W.scene_c5()
    m = s.meshes[0]
    view = s.views[0]
    vis = O.rasterize([m], view, threads=oracle_threads())
    pss = O.project(m, view)
    out = O.resolve_screen(vis, m.idx, 0, pss, m.attrs)
    cov = vis != O.EMPTY
    g = np.where(cov[..., None], np.float32(2.0) * (out - s.meta["target"].astype(np.float32)),
                 np.float32(0.0)).astype(np.float32)
    return s, m, view, vis, pss, out, g


def _assert_grad_close(got, ref, what):
    """|got - ref| <= 1e-3 max(|ref|, 1e-3 rms(ref)) element by element (acceptance of the
    differentiable resolve)."""
    scale = np.maximum(np.abs(ref), 1e-3 * np.sqrt(np.mean(ref ** 2)))
    rel = np.abs(got - ref) / scale
    assert np.all(rel <= 1e-3), f"{what}: worst relative error {rel.max()}"


def test_c5_resolve_forward_and_backward():
    """Forward (visibility, screen positions, resolve) against the oracle; the backward kernel
    called through the C ABI on inputs that all come from the oracle (visibility buffer, screen
    positions, attributes, upstream gradient) against the fp64 reference gradients under the
    same upstream gradient; position gradients against central differences of the L2 loss."""
    s, m, view, ref_vis, pss_ref, out_ref, g = _c5_oracle()
    with api.Context() as c:
        gmesh = api.GpuMesh.from_host(m)
        vis = c.rasterize_meshes([gmesh], view)
        pos_ss = c.project(gmesh, view)
        out = c.resolve_screen(vis, gmesh.idx, pos_ss, gmesh.attrs)
        torch.cuda.synchronize()
        assert_vis_equal(api.as_uint64(vis), ref_vis, "C5")
        assert np.array_equal(pos_ss.cpu().numpy(), pss_ref), "screen positions differ from the oracle"
        assert_resolve_close(out.cpu().numpy(), out_ref, "C5 resolve")
        # backward on oracle inputs only
        vis_o = torch.from_numpy(ref_vis.view(np.int64)).cuda()
        pss_o = torch.from_numpy(pss_ref).cuda()
        g_o = torch.from_numpy(g).cuda()
        ga = torch.zeros_like(gmesh.attrs)
        gp = torch.zeros_like(pss_o)
        c.resolve_backward(vis_o, gmesh.idx, pss_o, gmesh.attrs, g_o, ga, gp)
        torch.cuda.synchronize()
        ga = ga.cpu().numpy().astype(np.float64)
        gp = gp.cpu().numpy().astype(np.float64)
    ra, rp = O.resolve_screen_backward_f64(ref_vis, m.idx, 0, pss_ref, m.attrs, g.astype(np.float64))
    _assert_grad_close(ga, ra, "attribute gradient")
    _assert_grad_close(gp, rp, "position gradient")
    # central finite differences (eps 1e-3, fourth-order stencil) on 256 seeded visible vertices
    cov = ref_vis != O.EMPTY
    used = np.unique(m.idx[O.key_id(ref_vis[cov]).astype(np.int64)])
    verts = np.random.default_rng(57).choice(used, 256, replace=False).astype(np.uint32)
    fd = O.fd_pos_grad_l2(ref_vis, m.idx, 0, pss_ref, m.attrs, s.meta["target"], verts, eps=1e-3, order4=True)
    _assert_grad_close(gp[verts], fd, "FD check")


def test_c5_autograd_wrapper():
    """ResolveFn (torch.autograd.Function) on the GPU's own forward: with L = sum(img * G) for the
    oracle's upstream gradient G, autograd hands the backward exactly G, so its gradients must
    match the fp64 reference gradients under G."""
    s, m, view, ref_vis, pss_ref, out_ref, g = _c5_oracle()
    with api.Context() as c:
        gmesh = api.GpuMesh.from_host(m)
        vis = c.rasterize_meshes([gmesh], view)
        pos_ss = c.project(gmesh, view)
        attrs = gmesh.attrs.clone().requires_grad_(True)
        pss = pos_ss.clone().requires_grad_(True)
        img = api.ResolveFn.apply(attrs, pss, vis, gmesh.idx, 0, c)
        (img * torch.from_numpy(g).cuda()).sum().backward()
        ga = attrs.grad.cpu().numpy().astype(np.float64)
        gp = pss.grad.cpu().numpy().astype(np.float64)
        assert_resolve_close(img.detach().cpu().numpy(), out_ref, "C5 autograd forward")
    ra, rp = O.resolve_screen_backward_f64(ref_vis, m.idx, 0, pss_ref, m.attrs, g.astype(np.float64))
    _assert_grad_close(ga, ra, "autograd attribute gradient")
    _assert_grad_close(gp, rp, "autograd position gradient")

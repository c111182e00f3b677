"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (CPU only).

Each test is chosen so that a plausible mistake in the oracle (a dropped term, a wrong sign or
index, a transposed operand, a wrong tie rule, an off-by-one bound) fails at least one of them:

  * brute force vs bounding-box traversal (two independent transcriptions, bit for bit)
  * hand-derived golden triangle: exact covered set, exact key (Sec. 4.1 layout), exact resolve
  * projection closed form (Sec. 4.1 Eqs. 1-2)
  * watertightness: closed sphere winding invariant, camera inside a closed box (clip path),
    planar grid covers its rectangle exactly once
  * depth: exact powers of two for fronto-parallel triangles, fp64 closed form for tilted ones
  * tie-break by triangle ID, key layout, ID prefix-sum decode
  * clip path vs an fp64 analytic coverage of the visible part
  * resolve vs the paper's world-space ray/plane formulation (Sec. 4.4) and constant attributes
  * backward: partition of unity, linearity in the attributes, fp64 analytic vs central FD
  * supersampling: identity at k = 1, covered fractions, symmetric sample grid
  * compressed geometry: the paper's 9-bit example, bit layout, quantization bounds
  * textured resolve: mip chain by hand, bilinear ramps and wrap, trilinear blend, the level of
    detail in closed form, and the uv / level of detail of a near-plane-crossing ground plane
    against fp64 world-space ray casting (Sec. 4.4)
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2604_21749_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _view_cam(width, height, fovy=90.0, near=0.01, eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, -1.0)):
    return W.View(W.camera(eye, target, fovy_deg=fovy, aspect=width / height), near, width, height)


def _ids(vis):
    return O.key_id(vis)


# ----------------------------------------------------------------------------------------------
# brute force
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("variant", [
    {}, {"snap_grid": True}, {"near_crossing": True}, {"n_instances": 3}, {"spread": 8.0},
    {"near_crossing": True, "spread": 6.0, "n_tris": 24},
])
def test_brute_force_matches_bbox_traversal(variant):
    for seed in range(25):
        s = W.random_tiny_scene(seed, **variant)
        a = O.rasterize(s.meshes, s.views[0], threads=3)
        b = O.rasterize_brute(s.meshes, s.views[0])
        assert np.array_equal(a, b), (seed, variant)


def test_brute_force_scenes_exercise_ties_and_clipping():
    """The brute-force comparison is only a pin if its inputs reach the tie and clip cases."""
    ties = 0
    for seed in range(25):
        s = W.random_tiny_scene(seed, snap_grid=True)
        ss = O.project(s.meshes[0], s.views[0])
        frac = ss[:, :2] * 2.0
        ties += int(np.sum(frac == np.round(frac)))
    assert ties > 100
    behind = 0
    for seed in range(25):
        s = W.random_tiny_scene(seed, near_crossing=True)
        ss = O.project(s.meshes[0], s.views[0])
        behind += int(np.sum(ss[:, 2] < s.views[0].near))
    assert behind > 20


# ----------------------------------------------------------------------------------------------
# golden fixtures
# ----------------------------------------------------------------------------------------------
def _golden_triangle_scene(g, pad=True):
    verts = np.array(g["vertices"], np.float32)
    npad = g["pad_triangles_before"] if pad else 0
    far = np.array([[0, 0, -5], [0.01, 0, -5], [0, 0.01, -5]], np.float32)  # tiny, covers nothing
    pos = np.concatenate([far] * npad + [verts]) if npad else verts
    idx = np.arange(pos.shape[0], dtype=np.uint32).reshape(-1, 3)
    attrs = np.zeros((pos.shape[0], 3), np.float32)
    attrs[-3:] = np.array(g["resolve_attrs"], np.float32)
    mesh = W.Mesh(pos, idx, attrs=attrs)
    view = _view_cam(g["width"], g["height"], fovy=g["fovy_deg"], near=g["near"])
    return mesh, view


def test_golden_single_triangle():
    g = json.load(open(os.path.join(GOLDEN, "single_triangle.json")))
    mesh, view = _golden_triangle_scene(g)
    vis = O.rasterize([mesh], view)
    py, px = np.mgrid[0:g["height"], 0:g["width"]]
    expect = (px >= 2) & (py >= 2) & (px + py <= 10)
    assert int(expect.sum()) == g["expected_covered_count"]
    assert np.array_equal(vis != O.EMPTY, expect)
    assert np.all(vis[expect] == np.uint64(int(g["expected_key_hex"], 16)))
    out = O.resolve([mesh], view, vis, [mesh.attrs])
    x, y = g["resolve_pixel"]
    assert out[y, x].tolist() == g["resolve_expected"]


def test_golden_projection_cases():
    g = json.load(open(os.path.join(GOLDEN, "projection_cases.json")))
    for case in g["cases"]:
        view = _view_cam(case["width"], case["height"], fovy=case["fovy_deg"])
        mesh = W.Mesh(np.array([case["view_point"]], np.float32), np.zeros((0, 3), np.uint32))
        ss = O.project(mesh, view)
        assert ss[0].tolist() == case["expected"], case


def test_projection_matches_paper_closed_form():
    """Sec. 4.1: x_ndc = x f/(aspect d), y_ndc = y f/d, depth = d for view point (x, y, -d)."""
    rng = np.random.default_rng(5)
    for fovy, Wd, Hd in [(60.0, 640, 480), (45.0, 333, 517), (100.0, 1920, 1080)]:
        view = _view_cam(Wd, Hd, fovy=fovy)
        d = rng.uniform(0.05, 50.0, 200)
        p = np.stack([rng.uniform(-1, 1, 200) * d, rng.uniform(-1, 1, 200) * d, -d], 1).astype(np.float32)
        mesh = W.Mesh(p, np.zeros((0, 3), np.uint32))
        ss = O.project(mesh, view).astype(np.float64)
        f = 1.0 / math.tan(math.radians(fovy) / 2)
        a = Wd / Hd
        P = p.astype(np.float64)
        ex = (P[:, 0] * f / (a * -P[:, 2]) + 1.0) * Wd / 2
        ey = (P[:, 1] * f / -P[:, 2] + 1.0) * Hd / 2
        # a few binary32 roundings of values of magnitude up to ~2 * size
        assert np.all(np.abs(ss[:, 0] - ex) <= 8 * 2.0 ** -23 * 2 * Wd)
        assert np.all(np.abs(ss[:, 1] - ey) <= 8 * 2.0 ** -23 * 2 * Hd)
        assert np.all(np.abs(ss[:, 2] + P[:, 2]) <= 4 * 2.0 ** -23 * d)


# ----------------------------------------------------------------------------------------------
# watertightness
# ----------------------------------------------------------------------------------------------
def _jittered_sphere(lat, lon, seed, sigma):
    pos, idx = W.uv_sphere(lat, lon, 1.0)
    rng = np.random.default_rng(seed)
    pos = (pos.astype(np.float64) + rng.normal(0, sigma, pos.shape)).astype(np.float32)
    return W.Mesh(pos, idx)


@pytest.mark.parametrize("seed", range(6))
def test_closed_sphere_front_equals_back(seed):
    """For a closed surface seen from outside, every pixel centre is entered as often as it is
    left: #front == #back exactly, under any consistent fill rule of exact integer edges."""
    rng = np.random.default_rng(100 + seed)
    sphere = _jittered_sphere(24, 48, seed, 4e-3)
    d = rng.uniform(2.2, 6.0)
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    Wd, Hd = int(rng.integers(40, 90)), int(rng.integers(40, 90))
    view = W.View(W.camera(direction * d, (0, 0, 0), aspect=Wd / Hd), 0.01, Wd, Hd)
    front, back = O.coverage_counts([sphere], view)
    assert np.array_equal(front, back)
    # the silhouette is (nearly) the disk of angular radius asin(1/d)
    f = 1.0 / math.tan(math.radians(60.0) / 2)
    r_px = f * math.tan(math.asin(1.0 / d)) * Hd / 2
    area = math.pi * r_px ** 2
    assert abs(int((front > 0).sum()) - area) < 0.1 * area + 2 * math.pi * r_px


def _box(half=1.0):
    p = np.array([[x, y, z] for x in (-half, half) for y in (-half, half) for z in (-half, half)], np.float32)
    # outward-facing, counter-clockwise seen from outside
    q = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    tris = []
    for a, b, c, d in q:
        tris += [(a, b, c), (a, c, d)]
    return p, np.array(tris, np.uint32)


@pytest.mark.parametrize("seed", range(8))
def test_camera_inside_closed_box_sees_each_pixel_once(seed):
    """Clip path pin: from inside a closed box every view ray leaves through exactly one face,
    so after near-plane and guard-band clipping every pixel centre is covered exactly once, by a
    back-facing fragment.  Fails on any crack or overlap along clipped shared edges."""
    rng = np.random.default_rng(200 + seed)
    p, t = _box(1.0)
    X = W.instance_matrices(W.random_rotations(rng, 1), np.array([rng.uniform(0.5, 4.0)]),
                            rng.uniform(-0.2, 0.2, (1, 3)))
    mesh = W.Mesh(p, t, inst=X)
    Wd, Hd = int(rng.integers(30, 80)), int(rng.integers(30, 80))
    target = rng.normal(size=3)
    view = W.View(W.camera((0, 0, 0), target, fovy_deg=float(rng.uniform(40, 120)), aspect=Wd / Hd),
                  float(rng.uniform(0.001, 0.2)), Wd, Hd)
    front, back = O.coverage_counts([mesh], view)
    assert np.all(front == 0)
    assert np.all(back == 1)


def test_planar_grid_covers_rectangle_exactly_once():
    """A flat grid facing the camera at depth 2 covers every pixel centre of its window
    rectangle [x0, x1) x (y0, y1] exactly once (left and top borders are top-left edges)."""
    Wd = Hd = 64
    view = _view_cam(Wd, Hd)       # fovy 90: view (x, y, -2) -> window (16x + 32, 16y + 32)
    x0, x1, y0, y1 = 5.5, 52.25, 9.0, 50.5           # window rectangle, exact in binary32
    n = 7
    gx = np.linspace(x0, x1, n + 1)
    gy = np.linspace(y0, y1, n + 1)
    gx = np.round(gx * 256) / 256
    gy = np.round(gy * 256) / 256
    vx, vy = np.meshgrid((gx - 32) / 16, (gy - 32) / 16)
    pos = np.stack([vx.ravel(), vy.ravel(), np.full(vx.size, -2.0)], 1).astype(np.float32)
    tris = []
    for r in range(n):
        for c in range(n):
            a, b, cc, d = r * (n + 1) + c, r * (n + 1) + c + 1, (r + 1) * (n + 1) + c, (r + 1) * (n + 1) + c + 1
            tris += [(a, b, d), (a, d, cc)] if (r + c) % 2 else [(a, b, cc), (b, d, cc)]
    mesh = W.Mesh(pos, np.array(tris, np.uint32))
    front, back = O.coverage_counts([mesh], view)
    cy, cx = np.mgrid[0:Hd, 0:Wd] + 0.5
    expect = (cx >= x0) & (cx < x1) & (cy > y0) & (cy <= y1)
    assert np.array_equal(front, expect.astype(np.uint32))
    assert np.all(back == 0)
    vis = O.rasterize([mesh], view)
    assert np.array_equal(vis != O.EMPTY, expect)
    assert np.all(O.key_depth(vis[expect]) == 2.0)


# ----------------------------------------------------------------------------------------------
# depth
# ----------------------------------------------------------------------------------------------
def test_fronto_parallel_depth_is_exact():
    """Equal 1/w at the three vertices: every partial sum of the depth denominator is exact when
    area < 2^24, so the depth is exactly the plane depth (here powers of two)."""
    rng = np.random.default_rng(7)
    view = _view_cam(96, 64, fovy=70.0)
    for k in range(-3, 6):
        d = 2.0 ** k
        pos = []
        for _ in range(20):
            c = rng.uniform(-0.5, 0.5, 2) * d
            for _v in range(3):
                pos.append([c[0] + rng.uniform(-0.12, 0.12) * d, c[1] + rng.uniform(-0.12, 0.12) * d, -d])
        pos = np.array(pos, np.float32)
        idx = np.arange(pos.shape[0], dtype=np.uint32).reshape(-1, 3)
        idx = np.concatenate([idx, idx[:, [0, 2, 1]]])          # both windings, one of them visible
        vis = O.rasterize([W.Mesh(pos, idx)], view)
        cov = vis != O.EMPTY
        assert cov.sum() > 20
        assert np.all(O.key_depth(vis[cov]) == np.float32(d)), k


def test_tilted_plane_depth_matches_fp64():
    """Depth of a tilted triangle at each covered pixel centre vs the fp64 perspective-correct
    depth over the snapped window triangle (interpolated 1/w): agreement to the 3 dropped
    mantissa bits plus a few roundings."""
    view = _view_cam(64, 64)               # view (x, y, -z) -> window (32x/z + 32, 32y/z + 32)
    # window positions on the 1/256 grid and power-of-two depths make the snapped inputs exact
    win = np.array([[3.25, 4.0], [60.5, 10.75], [20.0, 58.5]])
    z = np.array([1.0, 4.0, 2.0])
    pos = np.stack([(win[:, 0] - 32) / 32 * z, (win[:, 1] - 32) / 32 * z, -z], 1).astype(np.float32)
    vis = O.rasterize([W.Mesh(pos, np.array([[0, 1, 2]], np.uint32))], view)
    cov = vis != O.EMPTY
    assert cov.sum() > 500
    py, px = np.nonzero(cov)
    cx, cy = px + 0.5, py + 0.5
    (x0, y0), (x1, y1), (x2, y2) = win
    area = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0)
    e0 = (x2 - x1) * (cy - y1) - (y2 - y1) * (cx - x1)
    e1 = (x0 - x2) * (cy - y2) - (y0 - y2) * (cx - x2)
    e2 = (x1 - x0) * (cy - y0) - (y1 - y0) * (cx - x0)
    depth = area / (e0 / z[0] + e1 / z[1] + e2 / z[2])
    got = O.key_depth(vis[cov]).astype(np.float64)
    rel = (depth - got) / depth
    assert np.all(rel >= -4 * 2.0 ** -24)            # truncation only lowers the value
    assert np.all(rel <= 2.0 ** -20 + 4 * 2.0 ** -24)


# ----------------------------------------------------------------------------------------------
# key, tie-break, IDs
# ----------------------------------------------------------------------------------------------
def test_tie_break_prefers_smaller_id_and_key_layout():
    s = W.random_tiny_scene(11, n_tris=12)
    m = s.meshes[0]
    dup = W.Mesh(m.pos, np.concatenate([m.idx, m.idx]))           # IDs t and t + 12 coincide
    vis = O.rasterize([dup], s.views[0])
    cov = vis != O.EMPTY
    assert cov.sum() > 100
    assert np.all(_ids(vis[cov]) < 12)
    # same via two identical instances: instance 0's IDs win
    ident = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]] * 2, np.float32)
    vis2 = O.rasterize([W.Mesh(m.pos, m.idx, inst=ident)], s.views[0])
    assert np.array_equal(vis2, O.rasterize([m], s.views[0]))
    # layout: depth in bits 36..63 (28 bits: float bits without the sign bit and the 3 lowest
    # mantissa bits), a finite positive depth, never the clear value
    d = O.key_depth(vis[cov])
    assert np.all(d > 0) and np.all(np.isfinite(d))
    assert np.all((vis[cov] >> np.uint64(36)) <= np.uint64(0x0FEFFFFF))
    assert not np.any(vis[cov] == O.EMPTY)


def test_id_prefix_and_binary_search_round_trip():
    rng = np.random.default_rng(3)
    meshes = []
    for T, N in [(5, 1), (0, 3), (7, 4), (1, 1), (0, 1), (13, 2)]:
        pos = rng.normal(size=(4, 3)).astype(np.float32)
        idx = rng.integers(0, 4, (T, 3)).astype(np.uint32)
        inst = None if N == 1 else np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (N, 1))
        meshes.append(W.Mesh(pos, idx, inst=inst))
    bases = O.id_bases(meshes)
    expect = []
    for mi, m in enumerate(meshes):
        for i in range(m.num_instances):
            for t in range(m.num_triangles):
                expect.append((mi, i, t))
    assert bases[-1] == len(expect)
    for gid, e in enumerate(expect):
        assert O.decode_id(meshes, bases, gid) == e
    assert O.decode_id(meshes, bases, len(expect)) is None


# ----------------------------------------------------------------------------------------------
# clip path vs fp64 analytic coverage
# ----------------------------------------------------------------------------------------------
def _analytic_cover(tri_view, width, height, fovy, near, margin_px):
    """fp64: clip the view-space triangle to depth >= near, project, test pixel centres against
    the resulting convex polygon; returns (covered, decided) where decided excludes centres
    within margin_px of an edge."""
    f = 1.0 / math.tan(math.radians(fovy) / 2)
    a = width / height
    poly = [np.array(v, np.float64) for v in tri_view]
    out = []
    for i in range(len(poly)):
        p, q = poly[i], poly[(i + 1) % len(poly)]
        dp, dq = -p[2] - near, -q[2] - near
        if dp >= 0:
            out.append(p)
        if (dp >= 0) != (dq >= 0):
            t = dp / (dp - dq)
            out.append(p + t * (q - p))
    win = np.array([[(v[0] * f / (a * -v[2]) + 1) * width / 2, (v[1] * f / -v[2] + 1) * height / 2] for v in out])
    cy, cx = np.mgrid[0:height, 0:width] + 0.5
    inside = np.ones((height, width), bool)
    mind = np.full((height, width), np.inf)
    n = len(win)
    orient = 0.0
    for i in range(n):
        orient += win[i][0] * win[(i + 1) % n][1] - win[(i + 1) % n][0] * win[i][1]
    sgn = 1.0 if orient > 0 else -1.0
    for i in range(n):
        p, q = win[i], win[(i + 1) % n]
        e = q - p
        L = math.hypot(*e)
        if L == 0:
            continue
        dist = sgn * (e[0] * (cy - p[1]) - e[1] * (cx - p[0])) / L
        inside &= dist > 0
        mind = np.minimum(mind, np.abs(dist))
    return inside & (orient > 0), mind > margin_px


@pytest.mark.parametrize("seed", range(12))
def test_clipped_triangle_matches_fp64_coverage(seed):
    rng = np.random.default_rng(300 + seed)
    Wd, Hd, fovy, near = 64, 48, 75.0, 0.05
    view = _view_cam(Wd, Hd, fovy=fovy, near=near)
    while True:
        tri = np.stack([rng.uniform(-3, 3, 3), rng.uniform(-3, 3, 3), -rng.uniform(-2.0, 4.0, 3)], 1)
        if np.sum(-tri[:, 2] < near) in (1, 2):
            break
    tri32 = tri.astype(np.float32)
    tri = tri32.astype(np.float64)
    for order in ([0, 1, 2], [0, 2, 1]):
        mesh = W.Mesh(tri32, np.array([order], np.uint32))
        front, back = O.coverage_counts([mesh], view)
        cov, decided = _analytic_cover(tri[order], Wd, Hd, fovy, near, 0.02)
        vis = O.rasterize([mesh], view)
        assert np.array_equal((vis != O.EMPTY), front > 0)
        assert np.array_equal(front[decided] > 0, cov[decided]), order
        assert np.all(front + back <= 1)


# ----------------------------------------------------------------------------------------------
# resolve
# ----------------------------------------------------------------------------------------------
def test_resolve_constant_attribute():
    s = W.scene_c1()
    vis = O.rasterize(s.meshes, s.views[0])
    consts = [np.full_like(m.attrs, 0.37) for m in s.meshes]
    out = O.resolve(s.meshes, s.views[0], vis, consts)
    cov = vis != O.EMPTY
    assert np.all(out[~cov] == 0)
    assert np.max(np.abs(out[cov] - np.float32(0.37))) <= 16 * 2.0 ** -24


def test_resolve_matches_world_space_ray_hit():
    """Sec. 4.4 shades in world space: cast the pixel's ray, intersect the triangle's plane and
    interpolate there.  An attribute affine in world position must therefore resolve to that
    affine function at the ray hit."""
    rng = np.random.default_rng(9)
    eye = np.array([0.3, 1.2, 2.5])
    target = np.array([0.0, 0.0, 0.0])
    Wd, Hd = 80, 60
    view = W.View(W.camera(eye, target, aspect=Wd / Hd), 0.01, Wd, Hd)
    # random front-facing triangles near the origin
    pos = rng.uniform(-0.8, 0.8, (30, 3)).astype(np.float32)
    idx = np.arange(30, dtype=np.uint32).reshape(10, 3)
    G = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.3], [-0.6, 0.2, 0.2]])
    off = np.array([0.7, 0.2, 0.4])
    attrs = (pos.astype(np.float64) @ G.T + off).astype(np.float32)
    mesh = W.Mesh(pos, np.concatenate([idx, idx[:, [0, 2, 1]]]), attrs=attrs)
    vis = O.rasterize([mesh], view)
    out = O.resolve([mesh], view, vis, [attrs])
    vp = view.vp.astype(np.float64)
    inv = np.linalg.inv(np.stack([vp[0], vp[1], vp[3], [0, 0, 0, 1]]))
    cov = np.argwhere(vis != O.EMPTY)
    assert len(cov) > 300
    worst = 0.0
    for py, px in cov:
        t = int(O.key_id(vis[py, px]))
        tri = pos[mesh.idx[t]].astype(np.float64)
        # ray through the pixel centre: world points with clip (ndc_x * w, ndc_y * w, w)
        ndc = np.array([(px + 0.5) / Wd * 2 - 1, (py + 0.5) / Hd * 2 - 1])
        p1 = inv @ np.array([ndc[0], ndc[1], 1.0, 1.0])
        p2 = inv @ np.array([2 * ndc[0], 2 * ndc[1], 2.0, 1.0])
        d = p2[:3] - p1[:3]
        nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        s = np.dot(nrm, tri[0] - p1[:3]) / np.dot(nrm, d)
        hit = p1[:3] + s * d
        expect = G @ hit + off
        err = np.abs(out[py, px] - expect) / np.maximum(np.abs(expect), 0.1)
        worst = max(worst, float(err.max()))
    assert worst < 1e-5


def test_supersampled_resolve_pins():
    """Supersampling (Sec. 5, Table 5) = rasterize at k times the resolution with the same
    projection, resolve every sample, average k x k blocks.  Pins: k = 1 is the identity; a
    constant attribute 1 gives the covered-sample fraction (each sample resolves to 1 within a few
    ulp of the barycentric sum); on a fronto-parallel plane an
    attribute affine in screen space averages over the symmetric sample grid to its value at the
    pixel centre, i.e. the 1x resolve."""
    Wd, Hd = 24, 20
    vp = W.camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), aspect=Wd / Hd)
    # a triangle partly covering the view, one attribute row = 1
    tri = np.array([[-0.9, -0.6, -2.0], [1.1, -0.4, -2.0], [0.1, 0.9, -2.0]], np.float32)
    mesh = W.Mesh(tri, np.array([[0, 1, 2]], np.uint32))
    ones = np.ones((3, 1), np.float32)
    for k in (1, 2, 4):
        hi = W.View(vp, 0.05, Wd * k, Hd * k)
        vis = O.rasterize([mesh], hi)
        out = O.resolve_supersampled([mesh], hi, vis, [ones], k)
        cov = (vis != O.EMPTY).astype(np.float64).reshape(Hd, k, Wd, k).sum(axis=(1, 3)) / (k * k)
        assert np.max(np.abs(out[..., 0].astype(np.float64) - cov)) <= 16 * 2.0 ** -24, k
        assert cov.min() == 0 and cov.max() == 1 and (k == 1 or ((cov > 0) & (cov < 1)).sum() > 10)
        if k == 1:
            assert np.array_equal(out, O.resolve([mesh], hi, vis, [ones]))
    # full-screen fronto-parallel quad at depth 2, attribute = a x_ndc + b y_ndc + c at its corners
    f = 1.0 / np.tan(np.radians(W.FOVY_DEG) / 2.0)
    X, Y = 2.0 * (Wd / Hd) / f * 1.5, 2.0 / f * 1.5
    quad = np.array([[-X, -Y, -2.0], [X, -Y, -2.0], [X, Y, -2.0], [-X, Y, -2.0]], np.float32)
    qidx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    ndc = quad[:, :2].astype(np.float64) / np.array([X / 1.5, Y / 1.5])
    attr = (0.3 * ndc[:, :1] - 0.2 * ndc[:, 1:] + 0.5).astype(np.float32)
    plane = W.Mesh(quad, qidx)
    lo = W.View(vp, 0.05, Wd, Hd)
    ref = O.resolve([plane], lo, O.rasterize([plane], lo), [attr])
    for k in (2, 4):
        hi = W.View(vp, 0.05, Wd * k, Hd * k)
        out = O.resolve_supersampled([plane], hi, O.rasterize([plane], hi), [attr], k)
        assert np.max(np.abs(out - ref)) <= 1e-6, k


# ----------------------------------------------------------------------------------------------
# compressed geometry (Sec. 4.6)
# ----------------------------------------------------------------------------------------------
def test_index_width_matches_the_paper_example_and_boundaries():
    g = json.load(open(os.path.join(GOLDEN, "compression_example.json")))
    assert O.index_bits(g["index_max"] - g["index_min"]) == g["bits"]
    idx = np.array([[2500, 2750, 3000], [2999, 2501, 2600]], np.uint32)
    lo, bits, words = O.compress_indices(idx)
    assert (lo, bits) == (2500, 9) and words.size == (6 * 9 + 31) // 32 + 3
    # widths at powers of two: span 2^k - 1 needs k bits, span 2^k needs k + 1
    for k in range(1, 32):
        assert O.index_bits((1 << k) - 1) == k and O.index_bits(1 << k) == k + 1
    assert O.index_bits(0) == 1 and O.index_bits(0xFFFFFFFF) == 32


def test_index_packing_round_trip_and_layout():
    rng = np.random.default_rng(21)
    for b in (1, 2, 3, 7, 8, 9, 16, 17, 28, 31, 32):
        span = (1 << b) - 1
        base = 0 if b == 32 else int(rng.integers(0, (1 << 32) - 1 - span))
        idx = (rng.integers(0, span, (41, 3), dtype=np.uint64, endpoint=True) + base).astype(np.uint32)
        idx[0, 0], idx[5, 2] = base, base + span
        lo, bits, words = O.compress_indices(idx)
        assert (lo, bits) == (base, b)
        assert np.array_equal(O.decompress_indices(words, lo, bits, 41), idx)
        # little-endian bit stream: index i's lowest bit is bit (i b) % 32 of word (i b) / 32
        flat = idx.reshape(-1).astype(np.uint64) - base
        for i in (0, 1, 7, 122):
            w, r = divmod(i * b, 32)
            assert (int(words[w]) >> r) & 1 == int(flat[i]) & 1
        assert words.size == (123 * b + 31) // 32 + 3 and np.all(words[-3:] == 0)


def test_position_quantization_bounds():
    rng = np.random.default_rng(22)
    pos = rng.normal(0, 3, (500, 3)).astype(np.float32)
    pos[:, 2] = 1.25                                  # a flat axis
    lo, step = O.position_box(pos)
    assert step[2] == 0 and np.all(step[:2] > 0)
    q = O.quantize_positions(pos, lo, step)
    dec = O.decode_positions(q, lo, step)
    assert q[:, :2].min() == 0 and q[:, :2].max() == 65535
    assert np.all(dec[:, 2] == 1.25)
    # each decoded coordinate within half a step (plus binary32 rounding) of the original
    err = np.abs(dec.astype(np.float64) - pos)[:, :2]
    bound = 0.5 * step[:2].astype(np.float64) * (1 + 1e-6) + 4 * np.spacing(np.abs(pos[:, :2]).max())
    assert np.all(err <= bound), (err.max(axis=0), bound)
    # the box minimum decodes exactly, the maximum within one ulp
    i0 = np.argmin(pos[:, 0])
    assert q[i0, 0] == 0 and dec[i0, 0] == pos[i0, 0]
    # decoding is q step + lo with one rounding (a fused multiply-add): exact rational value,
    # rounded to the nearest binary32, ties to even
    from fractions import Fraction
    for c in range(2):
        for i in range(0, 500, 7):
            exact = Fraction(int(q[i, c])) * Fraction(float(step[c])) + Fraction(float(lo[c]))
            f = np.float32(float(exact))
            cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
            dist = [abs(Fraction(float(x)) - exact) for x in cands]
            best = min(dist)
            nearest = [x for x, d in zip(cands, dist) if d == best]
            want = nearest[0] if len(nearest) == 1 else [x for x in nearest if (x.view(np.uint32) & 1) == 0][0]
            assert dec[i, c] == want, (i, c)


# ----------------------------------------------------------------------------------------------
# backward
# ----------------------------------------------------------------------------------------------
def _small_diff_scene():
    s = W.scene_c5(n=64)
    view = W.View(s.views[0].vp, s.views[0].near, 96, 96)
    m = s.meshes[0]
    vis = O.rasterize([m], view)
    pss = O.project(m, view)
    return m, view, vis, pss


def test_backward_attribute_gradient_partition_of_unity_and_linearity():
    m, view, vis, pss = _small_diff_scene()
    rng = np.random.default_rng(1)
    g = rng.normal(size=(view.height, view.width, 3))
    ga, _ = O.resolve_screen_backward_f64(vis, m.idx, 0, pss, m.attrs, g)
    cov = vis != O.EMPTY
    # sum_k b_k = 1 at every pixel, so the total attribute gradient equals the total upstream gradient
    assert np.allclose(ga.sum(0), g[cov].sum(0), rtol=1e-10, atol=1e-9)
    # the output is linear in the attributes: directional derivative is exact
    da = rng.normal(size=m.attrs.shape)
    o1 = O.resolve_screen_f64(vis, m.idx, 0, pss, m.attrs.astype(np.float64) + da)
    o0 = O.resolve_screen_f64(vis, m.idx, 0, pss, m.attrs.astype(np.float64))
    assert np.isclose(np.sum(g * (o1 - o0)), np.sum(ga * da), rtol=1e-9)


def test_backward_position_gradient_matches_central_fd():
    m, view, vis, pss = _small_diff_scene()
    rng = np.random.default_rng(2)
    target = rng.normal(0.5, 0.1, (view.height, view.width, 3))
    out = O.resolve_screen_f64(vis, m.idx, 0, pss, m.attrs)
    cov = vis != O.EMPTY
    g = np.where(cov[..., None], 2.0 * (out - target), 0.0)
    _, gp = O.resolve_screen_backward_f64(vis, m.idx, 0, pss, m.attrs, g)
    used = np.unique(m.idx[O.key_id(vis[cov]).astype(np.int64)])
    verts = rng.choice(used, 64, replace=False).astype(np.uint32)
    # fourth-order central stencil: its truncation error (eps^4) is far below the tolerance even
    # for the sliver triangles a dense height field produces
    fd = O.fd_pos_grad_l2(vis, m.idx, 0, pss, m.attrs, target, verts, eps=1e-4, order4=True)
    ana = gp[verts]
    scale = np.maximum(np.abs(fd), 1e-3 * np.sqrt(np.mean(fd ** 2)))
    assert np.all(np.abs(ana - fd) <= 1e-5 * scale)
    # the plain two-point difference converges to the same values at second order
    fd2 = O.fd_pos_grad_l2(vis, m.idx, 0, pss, m.attrs, target, verts, eps=1e-5, order4=False)
    assert np.all(np.abs(ana - fd2) <= 1e-4 * scale)
    # a perturbation of the whole vector agrees with the directional derivative
    dp = rng.normal(size=pss.shape) * 1e-4
    lp = np.sum(np.where(cov[..., None], O.resolve_screen_f64(vis, m.idx, 0, pss + dp, m.attrs) - target, 0) ** 2)
    lm = np.sum(np.where(cov[..., None], O.resolve_screen_f64(vis, m.idx, 0, pss - dp, m.attrs) - target, 0) ** 2)
    assert np.isclose((lp - lm) / 2, np.sum(gp * dp), rtol=1e-5)


# ----------------------------------------------------------------------------------------------
# textured resolve (Sec. 4.4, "Shading and Mip Mapping")
# ----------------------------------------------------------------------------------------------
def _level_constant_chain(w, h, L, step=20):
    """A chain whose level l is the constant step * l in every channel."""
    chain = np.zeros(O.texture_texels(w, h, L), np.uint32)
    off = 0
    for l in range(L):
        hl, wl = O.level_shape(w, h, l)
        chain[off:off + hl * wl] = np.uint32(step * l * 0x01010101)
        off += hl * wl
    return chain


def test_mip_chain_pins():
    assert O.texture_texels(8, 16, 5) == 8 * 16 + 4 * 8 + 2 * 4 + 1 * 2 + 1 * 1
    assert O.texture_texels(8, 8, 4) == 85 and O.texture_texels(8, 8, 5) == 0 and O.texture_texels(6, 4, 1) == 0
    # a constant stays constant at every level
    ch = O.build_mips(np.full((16, 8), 0x80402010, np.uint32), 5)
    assert np.all(ch == 0x80402010)
    # one-texel checkerboard of 0 and 255: every coarser texel is (0 + 255 + 0 + 255 + 2) >> 2 = 128
    cb = np.where((np.add.outer(np.arange(8), np.arange(8)) & 1) == 1, 0xFFFFFFFF, 0).astype(np.uint32)
    ch = O.build_mips(cb, 4)
    assert np.all(ch[64:] == 0x80808080)
    # horizontal stripes (odd rows 255): both rows of each 2 x 2 block count, (0 + 0 + 255 + 255 + 2) >> 2
    stripes = np.where((np.arange(8)[:, None] & 1) == 1, 0xFFFFFFFF, 0).repeat(4, axis=1).astype(np.uint32)
    assert np.all(O.build_mips(stripes, 3)[32:] == 0x80808080)
    # by hand, a 4 x 1 row (rows clamped): [0, 1, 2, 5] -> [(0+1+0+1+2)>>2, (2+5+2+5+2)>>2] = [1, 4] -> [3]
    ch = O.build_mips(np.array([[0, 1, 2, 5]], np.uint32), 3)
    assert ch.tolist() == [0, 1, 2, 5, 1, 4, 3]
    assert O.texture_level(ch, 4, 1, 1).tolist() == [[1, 4]]


def test_trilinear_sampling_pins():
    # 256 x 4 ramp (R = column), one level: between texel centres 255 R = frac(u) 256 - 0.5
    w, h = 256, 4
    ch = O.build_mips(np.tile(np.arange(w, dtype=np.uint32), (h, 1)), 1)
    for u in (0.01, 0.25, 0.5, 0.777, 0.99, 3.25, -0.75):
        x = (u - math.floor(u)) * 256 - 0.5
        assert 0 <= x <= 255
        assert abs(O.sample_trilinear(ch, w, h, 1, u, 0.3, 0.0)[0] * 255 - x) < 1e-3, u
    # wrap-around: at u = 0 the sample lies halfway between the last texel (255) and the first (0)
    assert abs(O.sample_trilinear(ch, w, h, 1, 0.0, 0.3, 0.0)[0] * 255 - 127.5) < 1e-3
    # the same along v with a row ramp (G = row) on a 4 x 256 texture
    ch = O.build_mips(np.tile((np.arange(256, dtype=np.uint32) << 8)[:, None], (1, 4)), 1)
    for v in (0.1, 0.5, 0.9):
        assert abs(O.sample_trilinear(ch, 4, 256, 1, 0.2, v, 0.0)[1] * 255 - (v * 256 - 0.5)) < 1e-3
    # between levels: linear in lod, clamped to [0, levels - 1]
    w = h = 64
    chain = _level_constant_chain(w, h, 7)
    for lod, expect in ((-3.0, 0.0), (0.0, 0.0), (0.25, 5.0), (2.5, 50.0), (5.75, 115.0), (6.0, 120.0), (40.0, 120.0)):
        assert np.allclose(O.sample_trilinear(chain, w, h, 7, 0.37, 0.61, lod) * 255, expect, atol=2e-3), lod


def test_texture_lod_pins():
    w, h, L = 256, 128, 9
    for s, t, expect in ((1.0, 0.5, 0.0), (4.0, 1.0, 2.0), (3.0, 5.0, math.log2(5.0)), (0.25, 0.25, 0.0),
                         (1e6, 0.0, 8.0)):
        u = [0.25, 0.25 + s / w, 0.25, 0.25 + s / w]
        v = [0.5, 0.5, 0.5 + t / h, 0.5 + t / h]
        assert abs(O.texture_lod(w, h, L, u, v) - expect) < 1e-4, (s, t)
    assert O.texture_lod(w, h, L, [0.3] * 4, [0.3] * 4) == 0.0
    assert O.texture_lod(w, h, L, [0.3] * 4, [0.3] * 4, finite=False) == 8.0
    # the extent of all four hits, not the step from the first: a rotated footprint spans 4 texels
    u = [0.5, 0.5 + 2 / w, 0.5 - 2 / w, 0.5]
    v = [0.5, 0.5 + 2 / h, 0.5 + 2 / h, 0.5 + 4 / h]
    assert abs(O.texture_lod(w, h, L, u, v) - 2.0) < 1e-4


def test_textured_resolve_lod_closed_form():
    """A fronto-parallel quad filling a 64 x 48 view with u = k_u x + 1/2, v = k_v y + 1/2: at depth
    2 with fovy 90 the view is 4 world units high, so adjacent pixels are 1/12 apart in x and y and
    the footprint is s = 256 k_u / 12 texels (k_v = k_u / 2), the level of detail clamp(log2 s, 0, 8)."""
    Wd, Hd = 64, 48
    view = _view_cam(Wd, Hd, fovy=90.0)
    quad = np.array([[-4, -3, -2], [4, -3, -2], [4, 3, -2], [-4, 3, -2]], np.float32)
    qidx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    mesh = W.Mesh(quad, qidx)
    vis = O.rasterize([mesh], view)
    assert np.all(vis != O.EMPTY)
    chain = _level_constant_chain(256, 256, 9)
    for s in (0.5, 1.0, 2.0, 3.3, 16.0, 1000.0):
        ku = s * 12.0 / 256.0
        uv = np.stack([quad[:, 0] * ku + 0.5, quad[:, 1] * (ku / 2) + 0.5], axis=1).astype(np.float32)
        out = O.resolve_textured([mesh], view, vis, [uv], [(chain, 256, 256, 9)])
        expect = 20.0 * min(max(math.log2(s), 0.0), 8.0)
        assert np.max(np.abs(out[..., 0] * 255 - expect)) < 5e-3, s
        assert np.array_equal(out[..., 0], out[..., 1]) and np.all(out[..., 3] == out[..., 0])
    # the uv of each pixel's own hit: u = 0.15 x + 1/2 and v = 0.2 y + 1/2 at the pixel centre,
    # x = (2 (px + 1/2) / 64 - 1) 8/3 and y = (2 (py + 1/2) / 48 - 1) 2, read back through R / G ramps
    uv = np.stack([quad[:, 0] * 0.15 + 0.5, quad[:, 1] * 0.2 + 0.5], axis=1).astype(np.float32)
    ramp = (np.arange(256, dtype=np.uint32)[None, :] | (np.arange(256, dtype=np.uint32)[:, None] << 8))
    out = O.resolve_textured([mesh], view, vis, [uv], [(O.build_mips(ramp, 1), 256, 256, 1)])
    px = np.arange(Wd) + 0.5
    py = np.arange(Hd) + 0.5
    u = 0.15 * (2 * px / Wd - 1) * (8.0 / 3.0) + 0.5
    v = 0.2 * (2 * py / Hd - 1) * 2.0 + 0.5
    assert np.max(np.abs(out[..., 0] * 255 - (u[None, :] * 256 - 0.5))) < 2e-3
    assert np.max(np.abs(out[..., 1] * 255 - (v[:, None] * 256 - 0.5))) < 2e-3


def _ground_rays_f64(view, px, py, dx=0.5, dy=0.5):
    """fp64 world-space ray through window point (px + dx, py + dy) of the C1 camera (eye (0, 0, 3),
    looking down -z, fovy 60, aspect 1) hitting the ground plane y = -1: (x, z) of the hit."""
    f = 1.0 / math.tan(math.radians(W.FOVY_DEG) / 2.0)
    nx = 2.0 * (px + dx) / view.width - 1.0
    ny = 2.0 * (py + dy) / view.height - 1.0
    d = np.stack([nx / f, ny / f, -np.ones_like(nx)], axis=-1)
    t = -1.0 / d[..., 1]
    return t * d[..., 0], 3.0 + t * d[..., 2]


def test_textured_resolve_near_plane_ground_vs_world_space_rays():
    """The C1 ground quad reaches behind the camera (its triangles cross the near plane).  With
    u = (x + 10) / 20, v = (z + 10) / 20, the oracle's uv at each pixel (read back through R and G
    ramps) and its level of detail (through a level-constant chain) equal fp64 ray casting in
    world space: the pixel's ray and the rays through its right, top and top-right neighbours
    intersected with the plane y = -1."""
    s = W.scene_c1()
    ground = s.meshes[1]
    view = s.views[0]
    vis = O.rasterize([ground], view)
    cov = vis != O.EMPTY
    assert cov.sum() > 50000
    uv = np.stack([(ground.pos[:, 0] + 10) / 20, (ground.pos[:, 2] + 10) / 20], axis=1).astype(np.float32)
    py, px = np.nonzero(cov)
    # uv: R ramps with the column, G with the row (one level)
    ramp = (np.arange(256, dtype=np.uint32)[None, :] | (np.arange(256, dtype=np.uint32)[:, None] << 8))
    out = O.resolve_textured([ground], view, vis, [uv], [(O.build_mips(ramp, 1), 256, 256, 1)])
    x, z = _ground_rays_f64(view, px, py)
    u_ref, v_ref = (x + 10) / 20, (z + 10) / 20
    xr, xg = out[py, px, 0] * 255.0, out[py, px, 1] * 255.0
    inner = (u_ref * 256 - 0.5 > 0.01) & (u_ref * 256 - 0.5 < 254.99) & (v_ref * 256 - 0.5 > 0.01) & \
            (v_ref * 256 - 0.5 < 254.99)
    assert inner.sum() > 0.9 * len(px)
    assert np.max(np.abs((xr + 0.5) / 256 - u_ref)[inner]) < 2e-5
    assert np.max(np.abs((xg + 0.5) / 256 - v_ref)[inner]) < 2e-5
    # level of detail: extent of the four hits' uv (now 8 (x + 10) / 20, 8 (z + 10) / 20, so the
    # plane spans several levels) in texels of a 256 x 256 chain of 9 levels
    out = O.resolve_textured([ground], view, vis, [uv * np.float32(8)],
                             [(_level_constant_chain(256, 256, 9), 256, 256, 9)])
    us, vs = [], []
    for dx, dy in ((0.5, 0.5), (1.5, 0.5), (0.5, 1.5), (1.5, 1.5)):
        x, z = _ground_rays_f64(view, px, py, dx, dy)
        us.append(8 * (x + 10) / 20)
        vs.append(8 * (z + 10) / 20)
    us, vs = np.array(us), np.array(vs)
    rho = np.maximum((us.max(0) - us.min(0)) * 256, (vs.max(0) - vs.min(0)) * 256)
    lod_ref = np.clip(np.log2(rho), 0, 8)
    lod = out[py, px, 0] * 255.0 / 20.0
    assert lod_ref.max() > 4.0 and lod_ref.min() < 2.0
    assert np.max(np.abs(lod - lod_ref)) < 2e-3


# ----------------------------------------------------------------------------------------------
# instance transforms, the one-mesh screen resolve and triangle ranges
# ----------------------------------------------------------------------------------------------
def _random_rigid_instances(rng, n, spread=1.5):
    """Uniform random rotations times a scale in [0.5, 2] plus a translation (Sec. 4.5 instances:
    row-major 3x4 object-to-world matrices [s R | t])."""
    R = W.random_rotations(rng, n)
    return W.instance_matrices(R, rng.uniform(0.5, 2.0, n), rng.uniform(-spread, spread, (n, 3)))


def _fp64_window(pos, inst12, view):
    """Closed form of the projection of an instanced vertex in fp64: clip = VP [X; 0 0 0 1] (v, 1),
    sx = (x / w + 1) W / 2, sy likewise, plus the magnitude sums S_r = sum |VP_rj| |X_jc| |h_c| that
    bound the binary32 rounding of each clip row."""
    X = np.eye(4)
    X[:3, :] = np.asarray(inst12, np.float64).reshape(3, 4)
    vp = np.asarray(view.vp, np.float64).reshape(4, 4)
    h = np.concatenate([np.asarray(pos, np.float64), np.ones((len(pos), 1))], 1)
    clip = h @ (vp @ X).T
    S = np.abs(h) @ (np.abs(vp) @ np.abs(X)).T
    x, y, w = clip[:, 0], clip[:, 1], clip[:, 3]
    return (x / w + 1.0) * view.width / 2, (y / w + 1.0) * view.height / 2, w, x, y, S


def test_instanced_projection_matches_fp64_closed_form():
    """orc_project of random rigid instances (rotation x scale + translation) against the fp64
    product VP [X; 0 0 0 1] (v, 1).  The draw matrix rounds each entry after at most three
    products and two sums, the vertex transform adds three roundings, so clip row r is within
    7u S_r (u = 2^-24) of the fp64 value; the window position adds 1/w, x/w and the final fma.
    A transposed or column-major reading of the 3x4 layout, a dropped translation, or the wrong
    instance's matrix misses by orders of magnitude more."""
    u = 2.0 ** -24
    rng = np.random.default_rng(21)
    for Wd, Hd in [(640, 480), (333, 517)]:
        view = W.View(W.camera((0.4, 0.8, 6.0), (0.0, 0.0, 0.0), aspect=Wd / Hd), 0.01, Wd, Hd)
        pos = rng.uniform(-1, 1, (300, 3)).astype(np.float32)
        inst = _random_rigid_instances(rng, 24)
        mesh = W.Mesh(pos, np.zeros((0, 3), np.uint32), inst=inst)
        for i in range(inst.shape[0]):
            got = O.project(mesh, view, instance=i).astype(np.float64)
            ex, ey, ew, x, y, S = _fp64_window(pos, inst[i], view)
            assert np.all(ew > 1.0)
            dw = 7 * u * S[:, 3]
            dx = 7 * u * S[:, 0]
            dy = 7 * u * S[:, 1]
            tol_x = 2 * ((Wd / 2) * (dx / ew + np.abs(x) * dw / ew ** 2 + 3 * u * np.abs(x / ew)) + 2 * u * np.abs(ex))
            tol_y = 2 * ((Hd / 2) * (dy / ew + np.abs(y) * dw / ew ** 2 + 3 * u * np.abs(y / ew)) + 2 * u * np.abs(ey))
            assert np.all(np.abs(got[:, 0] - ex) <= tol_x), (Wd, i, np.max(np.abs(got[:, 0] - ex) / tol_x))
            assert np.all(np.abs(got[:, 1] - ey) <= tol_y), (Wd, i, np.max(np.abs(got[:, 1] - ey) / tol_y))
            assert np.all(np.abs(got[:, 2] - ew) <= 2 * dw), (Wd, i)
            # the bound is tight enough to matter: the errors are well above zero on some vertices
            assert np.max(tol_x) < 1e-3 * Wd


def test_instanced_rasterization_matches_pretransformed_meshes():
    """Rasterizing a mesh under instance matrices X_i against rasterizing copies of the mesh
    transformed on the host.  (1) Diagonal power-of-two scales with signs: X v is exact in
    binary32 and every product A_rc v_c equals VP_rc (X v)_c exactly, so both buffers must be
    identical bit for bit (IDs agree because instance i of one mesh and mesh i of the copies have
    the same base i T).  (2) General rigid instances (host transform in fp64, rounded to binary32):
    the buffers differ only where a pixel centre lies within rounding of an edge or where depths
    tie, so nearly every covered pixel holds the same triangle of the same instance."""
    rng = np.random.default_rng(22)
    s = W.random_tiny_scene(31, n_tris=40, width=96, height=72, spread=1.2)
    base = s.meshes[0]
    view = s.views[0]
    # shift the mesh so that its object-space origin is at its centre (instances then stay in view)
    centre = base.pos.astype(np.float64).mean(0)
    pos0 = (base.pos.astype(np.float64) - centre).astype(np.float32)
    signs = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, 1)]
    diag = []
    for k, sg in enumerate(signs):
        sc = [sg[0] * 2.0 ** rng.integers(-1, 2), sg[1] * 2.0 ** rng.integers(-1, 2), sg[2] * 1.0]
        m = np.zeros((3, 4), np.float32)
        m[0, 0], m[1, 1], m[2, 2] = sc
        diag.append(m.reshape(12))
    diag = np.array(diag, np.float32)
    # translation 0 keeps column 3 of the draw matrix equal to VP's; the camera looks at the origin
    view_o = W.View(W.camera((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), aspect=view.width / view.height), 0.01,
                    view.width, view.height)
    inst_mesh = W.Mesh(pos0, base.idx, inst=diag)
    copies = [W.Mesh((pos0 * np.array([d[0], d[5], d[10]], np.float32)).astype(np.float32), base.idx) for d in diag]
    a = O.rasterize([inst_mesh], view_o, threads=2)
    b = O.rasterize(copies, view_o, threads=2)
    assert (a != O.EMPTY).sum() > 500
    assert np.array_equal(a, b)
    # general rigid instances
    inst = _random_rigid_instances(rng, 6, spread=0.4)
    inst_mesh = W.Mesh(pos0, base.idx, inst=inst)
    h = np.concatenate([pos0.astype(np.float64), np.ones((len(pos0), 1))], 1)
    copies = [W.Mesh((h @ inst[i].astype(np.float64).reshape(3, 4).T).astype(np.float32), base.idx)
              for i in range(inst.shape[0])]
    a = O.rasterize([inst_mesh], view_o, threads=2)
    b = O.rasterize(copies, view_o, threads=2)
    cov = (a != O.EMPTY) | (b != O.EMPTY)
    assert cov.sum() > 1000
    same_id = (O.key_id(a) == O.key_id(b)) & (a != O.EMPTY) & (b != O.EMPTY)
    assert same_id.sum() >= 0.97 * cov.sum(), same_id.sum() / cov.sum()


def test_resolve_screen_equals_resolve_per_mesh_instance():
    """orc_resolve_screen of one (mesh, instance) from orc_project's positions equals orc_resolve
    of the whole scene bit for bit on that pair's pixels (same binary32 steps), and is 0 on every
    other pixel (other meshes, other instances, empty).  orc_resolve itself is pinned by the
    constant-attribute and world-space ray-hit tests above."""
    a = W.random_tiny_scene(41, n_tris=30, n_instances=3, spread=2.5, width=64, height=48)
    b = W.random_tiny_scene(42, n_tris=25, near_crossing=True, width=64, height=48)
    meshes = [a.meshes[0], b.meshes[0]]
    view = a.views[0]
    vis = O.rasterize(meshes, view)
    full = O.resolve(meshes, view, vis, [m.attrs for m in meshes])
    bases = O.id_bases(meshes)
    ids = O.key_id(vis).astype(np.int64)
    cov = vis != O.EMPTY
    pairs = [(0, i) for i in range(3)] + [(1, 0)]
    seen = np.zeros(vis.shape, bool)
    for p, (m, i) in enumerate(pairs):
        mesh = meshes[m]
        pss = O.project(mesh, view, instance=i)
        out = O.resolve_screen(vis, mesh.idx, int(bases[p]), pss, mesh.attrs)
        mine = cov & (ids >= bases[p]) & (ids < bases[p] + mesh.num_triangles)
        assert mine.sum() > 20, (m, i)
        assert np.array_equal(out[mine], full[mine]), (m, i)
        assert np.all(out[~mine] == 0), (m, i)
        seen |= mine
    assert np.array_equal(seen, cov)


def test_rasterize_range_splits_and_full_range():
    """orc_rasterize_range (the CPU-baseline sampler): the full range equals orc_rasterize, an
    empty range leaves every pixel empty, and the elementwise minimum over ranges that split the
    pairs and the triangles at every index equals the full buffer (an off-by-one at a range end
    drops or shifts a triangle)."""
    s = W.random_tiny_scene(51, n_tris=18, n_instances=3, spread=1.0)
    meshes, view = s.meshes, s.views[0]
    full = O.rasterize(meshes, view, threads=2)
    assert np.array_equal(O.rasterize_range(meshes, view, 0, 3, 0, 18, threads=2), full)
    assert np.array_equal(O.rasterize_range(meshes, view, 0, 1 << 40, 0, 1 << 40, threads=3), full)
    assert np.all(O.rasterize_range(meshes, view, 0, 3, 7, 7) == O.EMPTY)
    assert np.all(O.rasterize_range(meshes, view, 2, 2, 0, 18) == O.EMPTY)
    acc = np.full_like(full, O.EMPTY)
    visible_parts = 0
    for p in range(3):
        for t in range(18):
            part = O.rasterize_range(meshes, view, p, p + 1, t, t + 1)
            ids = O.key_id(part[part != O.EMPTY]).astype(np.int64)
            assert np.all(ids == p * 18 + t)
            visible_parts += int(ids.size > 0)
            acc = np.minimum(acc, part)
    assert visible_parts >= 20
    assert np.array_equal(acc, full)

"""Benchmark of the MI355X visibility-buffer rasterizer.

Headline: one frame (clear + stages 1-3 + resolve, the paper's timed scope plus the clear) of the
massive 4K workload C3 = 16384^2-vertex noise height field (536.8M triangles) + a 2.1M-triangle
noise sphere instanced 4096x (8.59G triangle instances) at 3840x2160, reported as Gtris/s of the
triangle instances that survive the host mesh/instance cull, and ms/frame.

The same JSON line carries every workload (`configs`):
  c1  UV sphere + ground quad at 512^2 (oracle size; clipping, stages 2 and 3),
  c2  33.5M-triangle height field at 1920x1080 (HBM-bound stage 1),
  c3  the headline frame,
  c4  64 views of uneven size over 513 meshes: one batched (hipGraph) launch vs 64 plain launches,
  c5  differentiable resolve of a 10M-triangle height field at 1024^2 (forward / backward ms),
each with its stage split, the roofline of its dominant kernel and the CPU oracle timed on this
host (all threads, and one thread for c1 and c2; core count and CPU model stated).

Per-stage and per-launch times come from HIP events the library records on the launch stream
(CURAST_FLAG_TIMING, events taken from a pool, so a timed frame creates none); the same frames are
also run without the flag and both wall times are reported.

Each workload first runs the library's autotuner (curast_autotune) once, before the untimed
warm-up; the chosen options are part of the JSON line (--no-autotune: library defaults).

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--config c3|c2|c1] [--no-secondary]
                  [--no-cpu-baseline] [--copy-probe] [--no-autotune] [--options JSON] [--only c4|c5]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gtris/s & ms/frame at 3840x2160 (plain vs batched); resolve bwd ms"
HBM_PEAK_GBS = 8000.0
# vector ALU of MI355X without packed fp32 (which the build turns off): 256 CUs x 4 SIMDs x 16 lanes
# at 2.4 GHz, i.e. 64 lane-operations per CU per clock, or one wave64 instruction per CU per clock
CUS, CLOCK_HZ = 256, 2.4e9
ALU_PEAK_TOPS = CUS * 64 * CLOCK_HZ / 1e12
VALU_ISSUE_PEAK = CUS * CLOCK_HZ            # wave64 VALU instructions per second

# Algorithmic lane-operations of the multi-draw stage-1 launch (the strip algorithm; every draw
# counted as an interior one, whose vertices need no range tests):
#   a vertex projection: three 4-term rows through the draw's prescaled matrix (9 FMA), one
#   reciprocal and two multiplies = 12;
#   the box test of n window positions: 4 (n - 1) min/max, then 2 margin subtracts, 2 margin adds,
#   2 floors and 6 compares = 4 (n - 1) + 12;
#   the sphere test of a strip (s1_mode 0 and 2): the centre's projection (12), the two vectors
#   a - x b (6 FMA), their squared norms (6) and square roots (2), the denominator (1 FMA, 1 multiply,
#   1 compare), its reciprocal and the radius scale (2), the two radii (2 FMA), the box +- radius (4)
#   and the extent test (12) = 49;
#   one (strip of S triangles, draw): the sphere test, then for a strip the sphere cannot reject
#   S + 2 projections and the union-box test of its S + 2 vertices (s1_mode 4: always the latter);
#   a strip whose union box may hold a pixel centre: S more box tests of 3 positions (20 each);
#   a triangle outside a strip (poles, row ends): 3 projections and its box test.
PROJ_OPS = 12
SPHERE_OPS = 49


def box_ops(n: int) -> int:
    return 4 * (n - 1) + 12


def strip_draw_ops(S: int) -> int:
    return (S + 2) * PROJ_OPS + box_ops(S + 2)


LONE_TRI_DRAW_OPS = 3 * PROJ_OPS + box_ops(3)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage1_algorithmic_bytes(meshes) -> int:
    """Indices and vertex positions of the given meshes, each read once per frame (instances share
    both)."""
    return int(sum(m.idx.nbytes + m.pos.nbytes for m in meshes))


def split_meshes(api, scene, gm):
    """Meshes of the first stage-1 launch (two or more surviving draws) and of the second, with the
    triangle x draw items of each launch after the host cull."""
    visible, _, _ = api.plan(gm, scene.views)
    multi, single = [], []
    multi_items = single_items = 0
    row = 0
    for m in scene.meshes:
        draws = int((visible[row:row + m.num_instances] > 0).sum())
        row += m.num_instances
        if draws >= 2:
            multi.append(m)
            multi_items += m.num_triangles * draws
        else:
            single.append(m)
            single_items += m.num_triangles * draws
    return multi, single, multi_items, single_items


def autotuned_options(args, ctx, gm, views, outs) -> dict:
    """Launch options from the library's autotuner (curast_autotune: coordinate descent over the
    stage-1 kernel shape, thresholds and grid sizes, results unchanged), run once before the
    untimed warm-up; {} with --no-autotune (library defaults)."""
    if args.options:
        fixed = json.loads(args.options)
        ctx.set_options(**fixed)
        log(f"[bench] options given: {json.dumps(fixed)}")
        return fixed
    if args.no_autotune:
        return {}
    t0 = time.time()
    best = ctx.autotune(gm, views, outs)
    tuned = {k: v for k, v in best.items() if v and k != "flags"}
    log(f"[bench] autotuned in {time.time() - t0:.1f}s: {json.dumps(tuned)}")
    return tuned


def frame_stats(api, ctx, gm, view, vis, tuned) -> dict:
    """Statistics of one frame at the options that are timed (CURAST_FLAG_STATS)."""
    ctx.set_options(**tuned, flags=api.FLAG_STATS)
    ctx.reset_stats()
    ctx.rasterize_meshes(gm, view, out=vis)
    st = ctx.stats()
    ctx.set_options(**tuned, flags=0)
    return st


def timed_frames(args, torch, step, after_warmup=None):
    """K frames of `step` after W warm-up frames: wall ms per frame (synchronized on both sides)
    and the per-frame HIP-event times on the launch stream (torch's current stream, which the
    binding passes to the library)."""
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if after_warmup:
        after_warmup()
        torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t1 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1000.0 / args.steps
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    return ms, {"mean_ms": round(sum(per) / len(per), 4), "median_ms": round(per[len(per) // 2], 4),
                "min_ms": round(per[0], 4), "max_ms": round(per[-1], 4)}


STAGES = ("clear", "stage1_multi", "stage1_single", "stage1_overflow", "stage2", "stage3", "resolve")


def run_frame_config(args, api, torch, W, name, secondary=False):
    """One plain frame (clear + stages 1-3 + RGB resolve) of a workload, timed twice over K frames:
    with the library's stage events (the stage split and the launch times of the rooflines) and
    without them."""
    t0 = time.time()
    scene = {"c1": W.scene_c1, "c2": W.scene_c2, "c3": W.scene_c3}[name]()
    view = scene.views[0]
    log(f"[bench] generated {scene.name} in {time.time() - t0:.1f}s: {scene.total_tri_instances} tri instances")
    gm = [api.GpuMesh.from_host(m) for m in scene.meshes]
    attrs = [m.attrs for m in gm]
    ctx = api.Context()
    vis = torch.empty((view.height, view.width), dtype=torch.int64, device="cuda")
    out = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    tuned = autotuned_options(args, ctx, gm, [view], [vis])
    st = frame_stats(api, ctx, gm, view, vis, tuned)
    visible = int(st["tri_draws"])

    def step():
        ctx.rasterize_meshes(gm, view, out=vis)
        ctx.resolve(gm, view, vis, attrs, out=out)

    ctx.set_options(**tuned, flags=api.FLAG_TIMING)
    ms, frame_ev = timed_frames(args, torch, step, ctx.reset_stage_times)
    times = ctx.stage_times()
    n = max(1, times["frames"])
    stage_ms = {k: times[k] / n for k in STAGES}
    stage_ms["frame_gpu"] = sum(stage_ms.values())
    ctx.set_options(**tuned, flags=0)
    ms_plain, frame_ev_plain = timed_frames(args, torch, step)
    log(f"[bench] {name}: {args.steps} frames {ms:.3f} ms/frame wall with stage events, {ms_plain:.3f} without; "
        f"events {json.dumps(frame_ev)}; stages {json.dumps({k: round(v, 4) for k, v in stage_ms.items()})}")
    multi, single, multi_items, single_items = split_meshes(api, scene, gm)
    h = {"name": name, "scene": scene, "gm": gm, "ctx": ctx, "vis": vis, "ms": ms, "ms_no_events": ms_plain,
         "stage_ms": stage_ms, "frame_events": frame_ev, "frame_events_no_events": frame_ev_plain,
         "visible": visible, "stats": st, "multi": multi, "single": single, "multi_items": multi_items,
         "single_items": single_items, "options": ctx.options(), "autotuned": bool(tuned)}
    h["supersampling"] = run_supersampling(args, api, torch, ctx, gm, attrs, view, ms_plain) if secondary else {}
    h["compressed"] = run_compressed(args, api, torch, ctx, gm, attrs, view, visible) if secondary else {}
    h["textured"] = run_textured(args, api, torch, W, ctx, gm, attrs, view, vis) if secondary else {}
    return h


def config_summary(h, rooflines) -> dict:
    scene = h["scene"]
    view = scene.views[0]
    return {"workload": scene.name, "width": view.width, "height": view.height,
            "unique_triangles": int(sum(m.num_triangles for m in scene.meshes)),
            "triangle_instances": int(scene.total_tri_instances),
            "triangle_instances_after_cull": int(h["visible"]),
            "ms_per_frame": round(h["ms_no_events"], 4), "ms_per_frame_with_stage_events": round(h["ms"], 4),
            "gtris_s": round(h["visible"] / (h["ms_no_events"] * 1e-3) / 1e9, 4),
            "frame_events_ms": h["frame_events_no_events"],
            "stage_ms": {k: round(v, 4) for k, v in h["stage_ms"].items()},
            "roofline": rooflines[0], "roofline_other_stage1_launch": rooflines[1],
            "options": ("autotuned: " if h["autotuned"] else "library defaults: ") +
                       json.dumps({k: v for k, v in h["options"].items() if k != "flags"}),
            "stage_counts": {k: int(h["stats"][k]) for k in (
                "culled_near", "culled_frustum", "culled_tiny", "culled_backface", "s1_rasterized", "q2_entries",
                "q2_overflow", "s2_rasterized", "q3_entries", "q3_overflow", "draws_culled", "strip_draws",
                "strip_sphere_pass", "strip_union_pass")}}


def run_supersampling(args, api, torch, ctx, gm, attrs, view, ms_plain):
    """The headline frame with 2x2 and 4x4 supersampling (Sec. 5, Table 5): rasterize at k times
    the resolution, resolve every sample and average k x k blocks into the 3840x2160 image."""
    from paper_2604_21749_amd.workloads import View
    res = {"no_ss_ms": round(ms_plain, 3)}
    out = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    for k in (2, 4):
        hi = View(view.vp, view.near, view.width * k, view.height * k)
        vis = torch.empty((hi.height, hi.width), dtype=torch.int64, device="cuda")

        def frame():
            ctx.rasterize_meshes(gm, hi, out=vis)
            ctx.resolve(gm, hi, vis, attrs, out=out, samples_per_axis=k)
        frame()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps = max(2, args.steps // 4)
        for _ in range(reps):
            frame()
        torch.cuda.synchronize()
        res[f"ss{k}x{k}_ms"] = round((time.perf_counter() - t1) * 1000.0 / reps, 3)
        del vis
        torch.cuda.empty_cache()
    log(f"[bench] supersampling {res}")
    return res


def run_compressed(args, api, torch, ctx, gm, attrs, view, visible):
    """The headline frame with every mesh compressed (Sec. 4.6: bit-packed indices, 16-bit
    positions): geometry bytes, ms/frame and the single-draw stage-1 launch."""
    t0 = time.perf_counter()
    cm = [ctx.compress(g) for g in gm]
    torch.cuda.synchronize()
    compress_s = time.perf_counter() - t0
    vis = torch.empty((view.height, view.width), dtype=torch.int64, device="cuda")
    out = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")

    def frame():
        ctx.rasterize_meshes(cm, view, out=vis)
        ctx.resolve(cm, view, vis, attrs, out=out)
    opts = ctx.options()
    ctx.set_options(**{k: v for k, v in opts.items() if k != "flags"}, flags=opts["flags"] | api.FLAG_TIMING)
    frame()
    torch.cuda.synchronize()
    ctx.reset_stage_times()
    reps = max(2, args.steps // 2)
    t1 = time.perf_counter()
    for _ in range(reps):
        frame()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1000.0 / reps
    st = ctx.stage_times()
    ctx.set_options(**{k: v for k, v in opts.items() if k != "flags"}, flags=opts["flags"])
    n = max(1, st["frames"])
    plain_bytes = int(sum(g.pos.numel() * 4 + g.idx.numel() * 4 for g in gm))
    comp_bytes = int(sum(c.compressed.packed.numel() * 4 + c.compressed.qpos.numel() * 2 for c in cm))
    single = [c for c, g in zip(cm, gm) if g.num_instances == 1]
    single_bytes = int(sum(c.compressed.packed.numel() * 4 + c.compressed.qpos.numel() * 2 for c in single))
    res = {"geometry_bytes_plain": plain_bytes, "geometry_bytes_compressed": comp_bytes,
           "index_bits": [c.compressed.index_bits for c in cm], "compress_s": round(compress_s, 3),
           "ms_per_frame": round(ms, 3), "gtris_s": round(visible / (ms * 1e-3) / 1e9, 2),
           "stage1_single_ms": round(st["stage1_single"] / n, 4), "stage1_multi_ms": round(st["stage1_multi"] / n, 4),
           "stage1_single_hbm_frac": round(single_bytes / max(st["stage1_single"] / n * 1e-3, 1e-12) / 1e9
                                           / HBM_PEAK_GBS, 4)}
    log(f"[bench] compressed {res}")
    del cm, vis, out
    torch.cuda.empty_cache()
    return res


def run_textured(args, api, torch, W, ctx, gm, attrs, view, vis):
    """Resolve of the headline frame's visibility buffer with textures (Sec. 4.4): per-pixel UVs
    interpolated at four ray-plane hits, mip level from their extent, trilinear RGBA8 sample.
    Height field: u, v = 64 x, 64 z over a 4096^2 texture; spheres: 4 x + 1/2, 4 y + 1/2 over
    1024^2.  Compared with the per-vertex RGB resolve of the same buffer."""
    t0 = time.perf_counter()
    uvs = [(g.pos[:, [0, 2]] * 64.0).contiguous() if g.num_instances == 1 else (g.pos[:, [0, 1]] * 4.0 + 0.5).contiguous()
           for g in gm]
    sizes = [4096 if g.num_instances == 1 else 1024 for g in gm]
    texs = [ctx.texture(torch.from_numpy(W.texture_rgba8(n, n, 80 + i).view(np.int32)).cuda())
            for i, n in enumerate(sizes)]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    out4 = torch.empty((view.height, view.width, 4), dtype=torch.float32, device="cuda")
    out3 = torch.empty((view.height, view.width, 3), dtype=torch.float32, device="cuda")
    res = {"textures": [f"{n}x{n} RGBA8, {t.levels} levels" for n, t in zip(sizes, texs)],
           "setup_s": round(setup_s, 2)}
    reps = max(4, args.steps)
    for name, fn in (("textured_ms", lambda: ctx.resolve_textured(gm, view, vis, uvs, texs, out=out4)),
                     ("rgb_ms", lambda: ctx.resolve(gm, view, vis, attrs, out=out3))):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name] = round((time.perf_counter() - t1) * 1000.0 / reps, 4)
    log(f"[bench] textured resolve {res}")
    del uvs, texs, out4, out3
    torch.cuda.empty_cache()
    return res


def read_profile(path: str, src_path: str, src_key: str = "", runtime_path: str = ""):
    """Fields of a committed profiler summary ('key: value' lines), if it was taken from the current
    kernel source (its recorded sha256 prefix matches) and, where it records one, from the current
    host runtime (which sets each launch's options), else None: the counters no longer describe
    the kernel."""
    import hashlib
    if not os.path.exists(path):
        return None
    sha = lambda p: hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.rsplit(":", 1)          # keys may hold a colon ("sha256[:16]"), values do not
            fields[k.strip()] = v.strip()
    src = src_key or os.path.basename(src_path)
    if fields.get(f"{src} sha256[:16]") != sha(src_path):
        return None
    rt = fields.get("runtime.hip sha256[:16]")
    if rt is not None and rt != sha(runtime_path or RUNTIME_SRC):
        return None
    return fields


RASTER_SRC = os.path.join(ROOT, "paper_2604_21749_amd", "csrc", "raster.hip")
RESOLVE_SRC = os.path.join(ROOT, "paper_2604_21749_amd", "csrc", "resolve.hip")
RUNTIME_SRC = os.path.join(ROOT, "paper_2604_21749_amd", "csrc", "runtime.hip")


def read_traffic(kernel: str, path: str = "", src_path: str = "", src_key: str = "raster.hip",
                 runtime_path: str = ""):
    """HBM bytes per launch of a kernel from the committed profiler summary, if it was taken from
    the current kernel source and runtime (else None)."""
    f = read_profile(path or os.path.join(ROOT, "profiles", "stage1_c3_traffic.txt"), src_path or RASTER_SRC,
                     src_key, runtime_path)
    v = (f or {}).get(f"{kernel} hbm bytes per launch")
    return int(v) if v else None


def read_valu(kernel: str, path: str = "", src_path: str = ""):
    """SQ_INSTS_VALU (wave64 VALU instructions) per launch of a kernel from the committed counter
    summary, if it was taken from the current kernel source (else None)."""
    f = read_profile(path or os.path.join(ROOT, "profiles", "stage1_c3_valu.txt"), src_path or RASTER_SRC,
                     "raster.hip")
    v = (f or {}).get(f"{kernel} SQ_INSTS_VALU per launch")
    return int(v) if v else None


def multi_launch_ops(h) -> int:
    """Algorithmic lane-operations of one multi-draw stage-1 launch (see the counts at the top):
    from the frame's statistics at the timed options, the (strip, draw) pairs, those whose union
    box may hold a pixel centre, and the triangle x draw items outside strips."""
    o, st = h["options"], h["stats"]
    strips = o["s1_multi_tris_per_thread"] in (2, 4, 8) and not (o["flags"] & 0x100) and o["s1_mode"] != 3
    if not strips:
        return h["multi_items"] * LONE_TRI_DRAW_OPS
    S = o["s1_multi_tris_per_thread"]
    pairs, passed = int(st["strip_draws"]), int(st["strip_union_pass"])
    lone = max(0, h["multi_items"] - pairs * S)
    if o["s1_mode"] in (0, 2):
        tested = pairs * SPHERE_OPS + int(st["strip_sphere_pass"]) * strip_draw_ops(S)
    else:
        tested = pairs * strip_draw_ops(S)
    return tested + passed * S * box_ops(3) + lone * LONE_TRI_DRAW_OPS


def stage1_rooflines(h):
    """Roofline objects of the two stage-1 launches of a frame, the longer one first.

    Single-draw launch (meshes drawn once, e.g. the height field): bound by HBM; algorithmic bytes
    = its indices and vertex positions, each read once.  Multi-draw launch (instanced meshes): its
    lanes keep each loaded strip over up to s1_draws_per_item draws, so it is bound by vector ALU
    throughput; algorithmic lane-operations from multi_launch_ops over the triangle x draw items
    that survive the host cull.  Both divide by the launch's own HIP-event time over the timed
    frames."""
    sm = h["stage_ms"]
    o = h["options"]
    strip = o["s1_multi_tris_per_thread"] in (2, 4, 8) and not (o["flags"] & 0x100)
    sph = "true" if strip and o["s1_mode"] in (0, 2) else "false"
    k_single = f"stage1_fast_kernel<{o['s1_block']}, {o['s1_tris_per_thread']}, false, false, 0, false>"
    k_multi = f"stage1_fast_kernel<{o['s1_block']}, {o['s1_multi_tris_per_thread']}, {'true' if strip else 'false'}, " \
              f"false, 0, {sph}>"
    single_bytes = stage1_algorithmic_bytes(h["single"])
    t_single = max(sm["stage1_single"] * 1e-3, 1e-12)
    t_multi = max(sm["stage1_multi"] * 1e-3, 1e-12)
    single_ach = single_bytes / t_single / 1e9
    items = h["multi_items"]
    ops = multi_launch_ops(h) if items else 0
    multi_ach = ops / t_multi / 1e12
    single = {
        "kernel": f"{k_single} (stage 1, single-draw launch: {h['single_items']} triangle x draw items)",
        "bound": "hbm", "achieved": round(single_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(single_ach / HBM_PEAK_GBS, 4),
        "traffic": read_traffic(k_single) if h["name"] == "c3" else None,
        "algorithmic_bytes": single_bytes, "launch_ms": round(sm["stage1_single"], 4),
    }
    valu = read_valu(k_multi) if h["name"] == "c3" else None
    multi = {
        "kernel": f"{k_multi} (stage 1, multi-draw launch: {items} triangle x draw items after the host cull)",
        "bound": "alu", "achieved": round(multi_ach, 2), "peak": round(ALU_PEAK_TOPS, 2), "unit": "T lane-ops/s",
        "frac": round(multi_ach / ALU_PEAK_TOPS, 4),
        "traffic": read_traffic(k_multi) if h["name"] == "c3" else None,
        "algorithmic_lane_ops": int(ops), "lane_ops_per_unit": round(ops / max(items, 1), 3),
        "unit_of_work": "triangle x draw item", "launch_ms": round(sm["stage1_multi"], 4),
        # VALU wave64 instructions the launch issued (rocprofv3 SQ_INSTS_VALU, committed summary) over
        # the same live launch time: issued lane-operations (x64, inactive lanes included) and the
        # fraction of the one-instruction-per-CU-per-clock issue peak
        "issued_lane_ops_per_s": None if valu is None else round(valu * 64 / t_multi / 1e12, 2),
        "issued_frac": None if valu is None else round(valu / t_multi / VALU_ISSUE_PEAK, 4),
        "issued_lane_ops_per_unit": None if valu is None else round(valu * 64 / max(items, 1), 3),
    }
    return (multi, single) if sm["stage1_multi"] >= sm["stage1_single"] else (single, multi)


def run_batched(args, api, torch, W):
    """C4: one batched frame (all views in one captured graph) against 64 per-view plain launches,
    same outputs.  Its stage split and the multi-draw roofline come from the same frame run through
    the eager launch sequence (CURAST_FLAG_NO_GRAPH) with the stage events, since a graph replay
    records only the whole frame."""
    t0 = time.time()
    scene = W.scene_c4()
    log(f"[bench] generated {scene.name} in {time.time() - t0:.1f}s: {scene.total_tri_instances} tris x "
        f"{len(scene.views)} views")
    gm = [api.GpuMesh.from_host(m) for m in scene.meshes]
    outs = [torch.empty((v.height, v.width), dtype=torch.int64, device="cuda") for v in scene.views]
    ctx = api.Context()
    tuned = autotuned_options(args, ctx, gm, scene.views, outs)
    ctx.set_options(**tuned, flags=api.FLAG_STATS)
    ctx.reset_stats()
    ctx.rasterize_batched(gm, scene.views, outs)
    st = ctx.stats()
    tri_views = int(st["tri_draws"])
    reps = max(2, args.steps // 4)

    def plain():
        for v, o in zip(scene.views, outs):
            ctx.rasterize_meshes(gm, v, out=o)

    def batched():
        ctx.rasterize_batched(gm, scene.views, outs)

    r = {}
    for name, fn, flags in (("plain", plain, 0), ("batched", batched, 0),
                            ("eager_staged", batched, api.FLAG_NO_GRAPH | api.FLAG_TIMING)):
        ctx.set_options(**tuned, flags=flags)
        fn()
        torch.cuda.synchronize()
        ctx.reset_stage_times()
        t1 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        r[name] = (time.perf_counter() - t1) * 1000.0 / reps
    times = ctx.stage_times()
    n = max(1, times["frames"])
    stage_ms = {k: times[k] / n for k in STAGES if k != "resolve"}
    multi, single, multi_items, single_items = split_meshes(api, scene, gm)
    h = {"name": "c4", "stage_ms": {**stage_ms, "resolve": 0.0}, "options": ctx.options(), "stats": st,
         "multi": multi, "single": single, "multi_items": multi_items, "single_items": single_items}
    rl = stage1_rooflines(h)
    ctx.close()
    del gm, outs
    torch.cuda.empty_cache()
    log(f"[bench] c4: plain {r['plain']:.2f} ms, batched {r['batched']:.2f} ms, eager {r['eager_staged']:.2f} ms")
    return {"workload": scene.name, "views": len(scene.views), "tri_views_after_cull": tri_views,
            "plain_ms": round(r["plain"], 3), "batched_ms": round(r["batched"], 3),
            "plain_gtris_s": round(tri_views / r["plain"] / 1e6, 3),
            "batched_gtris_s": round(tri_views / r["batched"] / 1e6, 3),
            "batched_speedup": round(r["plain"] / r["batched"], 3), "autotuned": bool(tuned),
            "eager_staged_ms": round(r["eager_staged"], 3),
            "stage_ms_eager": {k: round(v, 4) for k, v in stage_ms.items()},
            "roofline": rl[0], "roofline_other_stage1_launch": rl[1],
            "options": json.dumps({k: v for k, v in ctx_options_clean(h["options"]).items()})}


def ctx_options_clean(o):
    return {k: v for k, v in o.items() if k != "flags"}


# Algorithmic bytes of the resolve backward per pixel and per covered pixel: every key is read
# (8 B); a covered pixel reads its upstream gradient (4 C B), the three indices (12 B), three screen
# positions (36 B) and three attribute rows (12 C B), and adds 3 (C + 3) fp32 values atomically,
# each a 4-byte read and a 4-byte write of the gradient arrays.
def backward_bytes(pixels: int, covered: int, C: int = 3) -> int:
    return 8 * pixels + covered * (4 * C + 12 + 36 + 12 * C + 8 * 3 * (C + 3))


def run_resolve_bwd(args, api, torch, W):
    scene = W.scene_c5()
    m = scene.meshes[0]
    g = api.GpuMesh.from_host(m)
    view = scene.views[0]
    ctx = api.Context()
    vis = ctx.rasterize_meshes([g], view)
    pos_ss = ctx.project(g, view)
    target = torch.from_numpy(scene.meta["target"]).cuda()
    out = ctx.resolve_screen(vis, g.idx, pos_ss, g.attrs)
    grad_out = (2.0 * (out - target)).contiguous()
    covered = (vis != -1).unsqueeze(-1)
    grad_out = torch.where(covered, grad_out, torch.zeros_like(grad_out)).contiguous()
    ga = torch.zeros_like(g.attrs)
    gp = torch.zeros_like(pos_ss)
    reps = max(3, args.steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        ctx.resolve_screen(vis, g.idx, pos_ss, g.attrs, out=out)
        ctx.resolve_backward(vis, g.idx, pos_ss, g.attrs, grad_out, ga, gp)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        ctx.resolve_screen(vis, g.idx, pos_ss, g.attrs, out=out)
    ev[1].record()
    for _ in range(reps):
        ctx.resolve_backward(vis, g.idx, pos_ss, g.attrs, grad_out, ga, gp)
    ev[2].record()
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / reps
    bwd = ev[1].elapsed_time(ev[2]) / reps
    covered_px = int(covered.sum().item())
    ctx.close()
    # the fp32 atomic ceiling on this part for the same scatter: torch's index_add_ (one fp32 atomic
    # add per element) of as many rows of 3 values as the backward adds, at seeded random rows of
    # arrays of the backward's size
    n_rows = g.attrs.shape[0]
    rows = torch.randint(0, n_rows, (6 * covered_px,), device="cuda",
                         generator=torch.Generator(device="cuda").manual_seed(58))
    src = torch.ones((rows.numel(), 3), dtype=torch.float32, device="cuda")
    dst = torch.zeros((n_rows, 3), dtype=torch.float32, device="cuda")
    dst.index_add_(0, rows, src)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        dst.index_add_(0, rows, src)
    ev[1].record()
    torch.cuda.synchronize()
    probe_ms = ev[0].elapsed_time(ev[1]) / reps
    probe = {"atomics": 3 * rows.numel(), "ms": round(probe_ms, 4),
             "atomics_per_s": round(3 * rows.numel() / (probe_ms * 1e-3), 1),
             "what": "torch index_add_ of 3-float rows at seeded random rows of a [V][3] fp32 array"}
    del rows, src, dst
    px = view.width * view.height
    nbytes = backward_bytes(px, covered_px)
    ach = nbytes / (bwd * 1e-3) / 1e9
    atomics = 18 * covered_px
    return {"workload": scene.name, "covered_px": covered_px, "resolve_fwd_ms": round(fwd, 4),
            "resolve_bwd_ms": round(bwd, 4),
            "roofline": {"kernel": "resolve_backward_kernel", "bound": "hbm", "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": read_traffic("resolve_backward_kernel", os.path.join(ROOT, "profiles",
                                                 "resolve_backward_c5.txt"), RESOLVE_SRC, "resolve.hip"),
                         "algorithmic_bytes": nbytes, "launch_ms": round(bwd, 4),
                         "fp32_atomics": atomics, "atomics_per_s": round(atomics / (bwd * 1e-3), 1)},
            "atomic_probe": probe}


def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"nproc": os.cpu_count() or 1, "threads_available": avail, "cpu_model": model}


def oracle_threads() -> int:
    n = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    return max(1, min(n, os.cpu_count() or 1))


def cpu_baseline(scene, target_s: float = 15.0):
    """The CPU oracle on a bounded sample of the same workload, scaled to Gtris/s."""
    import oracle as O
    threads = oracle_threads()
    view = scene.views[0]
    # probe: the first 16M triangles of the first mesh
    probe = min(scene.meshes[0].num_triangles, 16_000_000)
    t0 = time.perf_counter()
    O.rasterize_range(scene.meshes[:1], view, 0, 1, 0, probe, threads=threads)
    rate = probe / max(time.perf_counter() - t0, 1e-6)
    # sample: triangles [0, n) of every (mesh, instance) pair, sized for about target_s seconds
    pairs = sum(m.num_instances for m in scene.meshes)
    total = scene.total_tri_instances
    budget = rate * target_s
    frac = min(1.0, budget / total)
    n_tris = max(1, int(max(m.num_triangles for m in scene.meshes) * frac))
    done = sum(min(m.num_triangles, n_tris) * m.num_instances for m in scene.meshes)
    t0 = time.perf_counter()
    O.rasterize_range(scene.meshes, view, 0, pairs, 0, n_tris, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(done / dt / 1e9, 5), "unit": "Gtris/s", "cores": threads, "kind": "oracle",
            "sample": f"triangles [0, {n_tris}) of each of the {pairs} (mesh, instance) pairs of {scene.name} "
                      f"({done} triangle instances, {dt:.1f} s), rasterization only, {threads} threads",
            "host": host_info()}


def cpu_frame_baseline(scene, visible: int, threads_list=(0, 1)):
    """The CPU oracle on a whole frame of a small workload (rasterization + RGB resolve), on all
    threads and on one thread: Gtris/s of the triangle instances the GPU frame counts."""
    import oracle as O
    view = scene.views[0]
    res = {"unit": "Gtris/s", "kind": "oracle", "host": host_info(),
           "sample": f"the whole {scene.name} frame (rasterization + RGB resolve)"}
    for t in threads_list:
        n = oracle_threads() if t == 0 else t
        t0 = time.perf_counter()
        vis = O.rasterize(scene.meshes, view, threads=n)
        O.resolve(scene.meshes, view, vis, [m.attrs for m in scene.meshes], threads=n)
        dt = time.perf_counter() - t0
        key = "value" if t == 0 else f"value_{n}_thread"
        res[key] = round(visible / dt / 1e9, 5)
        res["cores" if t == 0 else f"seconds_{n}_thread"] = n if t == 0 else round(dt, 3)
        if t == 0:
            res["seconds"] = round(dt, 3)
    return res


def cpu_batched_baseline(api, W, n_views: int = 4):
    """The CPU oracle on a seeded sample of the C4 views (all meshes into each), Gtris/s of the
    triangle x view items the GPU frame counts for those views."""
    import oracle as O
    scene = W.scene_c4()
    pick = sorted(np.random.default_rng(404).choice(len(scene.views), n_views, replace=False).tolist())
    views = [scene.views[i] for i in pick]
    gm = [api.GpuMesh.from_host(m) for m in scene.meshes]
    visible, _, _ = api.plan(gm, views)
    tris = np.repeat([m.num_triangles for m in scene.meshes], [m.num_instances for m in scene.meshes])
    items = int(sum(int(tris.astype(np.int64) @ (visible[:, j] > 0)) for j in range(len(views))))
    del gm
    n = oracle_threads()
    t0 = time.perf_counter()
    for v in views:
        O.rasterize(scene.meshes, v, threads=n)
    dt = time.perf_counter() - t0
    return {"value": round(items / dt / 1e9, 5), "unit": "Gtris/s", "cores": n, "kind": "oracle",
            "sample": f"views {pick} of {scene.name} ({items} triangle x view items after the host cull, "
                      f"{dt:.1f} s), rasterization only, {n} threads", "host": host_info()}


def cpu_backward_baseline(W):
    """The oracle's fp64 resolve backward (one thread) on the whole C5 frame, from its own
    visibility buffer and screen positions."""
    import oracle as O
    scene = W.scene_c5()
    m = scene.meshes[0]
    view = scene.views[0]
    vis = O.rasterize([m], view, threads=oracle_threads())
    pss = O.project(m, view)
    out = O.resolve_screen(vis, m.idx, 0, pss, m.attrs)
    cov = vis != O.EMPTY
    g = np.where(cov[..., None], 2.0 * (out.astype(np.float64) - scene.meta["target"]), 0.0)
    t0 = time.perf_counter()
    O.resolve_screen_backward_f64(vis, m.idx, 0, pss, m.attrs, g)
    dt = time.perf_counter() - t0
    return {"value": round(dt * 1e3, 2), "unit": "ms (resolve backward)", "cores": 1, "kind": "oracle",
            "sample": f"the whole {scene.name} backward ({int(cov.sum())} covered pixels), fp64, one thread",
            "host": host_info()}


def copy_probe(torch):
    """A plain device copy of known size, for scaling HBM byte counters of the profiler."""
    n = 1 << 28   # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy probe: 3 copies of {4 * n} bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="library default options instead of autotuned ones")
    ap.add_argument("--options", default="", help="JSON launch options to use instead of the autotuner's "
                                                  "(profiler runs repeat the timed configuration without tuning)")
    ap.add_argument("--only", default="", choices=["", "c4", "c5"],
                    help="run one secondary workload alone and print its entry (profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2604_21749_amd import api
    from paper_2604_21749_amd import workloads as W
    api.lib()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(torch)
    if args.only:
        entry = run_batched(args, api, torch, W) if args.only == "c4" else run_resolve_bwd(args, api, torch, W)
        print(json.dumps({"only": args.only, **entry}), flush=True)
        return

    h = run_frame_config(args, api, torch, W, args.config, secondary=not args.no_secondary)
    scene = h["scene"]
    view = scene.views[0]
    rl_main, rl_other = stage1_rooflines(h)
    head = config_summary(h, (rl_main, rl_other))
    result = {
        "metric": METRIC,
        "value": round(h["visible"] / (h["ms_no_events"] * 1e-3) / 1e9, 4),
        "unit": "Gtris/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_no_events"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": scene.name, "width": view.width, "height": view.height,
            "meshes": len(scene.meshes), "instances": [m.num_instances for m in scene.meshes],
            "unique_triangles": head["unique_triangles"], "triangle_instances": head["triangle_instances"],
            "triangle_instances_after_cull": head["triangle_instances_after_cull"],
            "frame": "clear + stages 1-3 + resolve (RGB)", "options": head["options"],
        },
        "ms_per_step_with_stage_events": head["ms_per_frame_with_stage_events"],
        "stage_ms": head["stage_ms"],
        "frame_events_ms": h["frame_events_no_events"],
        "roofline": rl_main,
        "roofline_other_stage1_launch": rl_other,
        "gtris_s_submitted": round(scene.total_tri_instances / (h["ms_no_events"] * 1e-3) / 1e9, 4),
        "supersampling": h["supersampling"],
        "compressed": h["compressed"],
        "textured_resolve": h["textured"],
        "stage_counts": head["stage_counts"],
    }
    h["ctx"].close()
    del h["gm"], h["vis"]
    torch.cuda.empty_cache()
    configs = {args.config: {k: v for k, v in head.items() if k not in ("options",)}}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scene)
        configs[args.config]["cpu_baseline"] = result["cpu_baseline"]
    del scene, h
    if not args.no_secondary:
        for name in ("c1", "c2"):
            if name == args.config:
                continue
            try:
                hc = run_frame_config(args, api, torch, W, name)
                summ = config_summary(hc, stage1_rooflines(hc))
                hc["ctx"].close()
                del hc["gm"], hc["vis"]
                torch.cuda.empty_cache()
                if not args.no_cpu_baseline:
                    summ["cpu_baseline"] = cpu_frame_baseline(hc["scene"], hc["visible"])
                configs[name] = summ
            except Exception as e:  # reported, not hidden
                configs[name] = {"error": repr(e)}
        try:
            configs["c4"] = run_batched(args, api, torch, W)
            if not args.no_cpu_baseline:
                configs["c4"]["cpu_baseline"] = cpu_batched_baseline(api, W)
        except Exception as e:
            configs["c4"] = {"error": repr(e)}
        try:
            configs["c5"] = run_resolve_bwd(args, api, torch, W)
            if not args.no_cpu_baseline:
                configs["c5"]["cpu_baseline"] = cpu_backward_baseline(W)
        except Exception as e:
            configs["c5"] = {"error": repr(e)}
        result["batched"] = {k: v for k, v in configs.get("c4", {}).items() if k not in ("roofline",
                                                                                           "roofline_other_stage1_launch")}
        result["resolve_backward"] = {k: v for k, v in configs.get("c5", {}).items() if k != "roofline"}
    result["configs"] = configs
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

/*
 * curast: brute-force visibility-buffer rasterization of dense, opaque, unstructured triangle
 * meshes on one AMD Instinct MI355X (gfx950), after CuRast (Schuetz, Lipp, Kristmann, Wimmer).
 *
 * The library builds no acceleration structure and no level of detail.  Every triangle of every
 * mesh instance is transformed, culled and rasterized into a 64-bit visibility buffer with a
 * 64-bit atomic minimum on (depth28 << 36 | global triangle ID) (Sec. 3.1, Sec. 4.1): small
 * triangles one per GPU lane (stage 1), medium ones one per wavefront (stage 2), large ones per
 * 64x64 screen tile (stage 3, Sec. 4.1-4.3).  A resolve pass turns the IDs into perspective-
 * correct interpolated vertex attributes (Sec. 4.4); its backward pass gives gradients with
 * respect to the attributes and the screen-space vertex positions.
 *
 * Result definition (what every entry point computes exactly, whatever the stage thresholds,
 * workgroup sizes, queue capacities or culling switches):
 *   - draw matrix A = VP * X (rows x, y and w of the view-projection VP, row 2 unused) per
 *     (mesh, instance), in binary32 with the operation order
 *       A[r][c] = (VP[r][0]*X[0][c] + VP[r][1]*X[1][c]) + VP[r][2]*X[2][c]              (c < 3)
 *       A[r][3] = ((VP[r][0]*X[0][3] + VP[r][1]*X[1][3]) + VP[r][2]*X[2][3]) + VP[r][3];
 *   - vertex x, y, w = fmaf(A[r][0], vx, fmaf(A[r][1], vy, fmaf(A[r][2], vz, A[r][3]))); w is the
 *     positive linear view depth (Sec. 4.1 Eqs. 1-2 are the special case of a look-at view and
 *     the projection vector [f/aspect, f, -1]);
 *   - triangles with every w < near produce nothing; triangles with any w < near or |x| > 16 w
 *     or |y| > 16 w are clipped (Sutherland-Hodgman, Sec. 4.2) against w >= near and the guard
 *     band |x|, |y| <= 16 w, intersections computed from the inside vertex, and fanned;
 *   - window position snapped to 1/256 pixel: zI = 1/w (correctly rounded), sx = fmaf(x*zI,
 *     W/2, W/2), X = rint(256*sx) (round half to even), and the same for y with H/2;
 *   - a pixel (px, py) (row 0 at the bottom) is covered when its centre lies inside the snapped
 *     triangle under int64 edge functions with the top-left rule; counter-clockwise triangles
 *     are front-facing, back-facing and degenerate ones cover nothing (Sec. 4.1 backface cull);
 *   - depth = area / (E0/w0 + E1/w1 + E2/w2) (interpolated 1/w, Sec. 4.1), key =
 *     (float bits of depth >> 3) << 36 | ID, visibility buffer = per-pixel minimum key, empty
 *     pixels all ones (0xFFFFFFFFFFFFFFFF);
 *   - global ID = exclusive prefix of triangle counts over all (mesh, instance) pairs in
 *     mesh-major order, plus the triangle index (Sec. 4, Sec. 4.4).
 *
 * Conventions for every entry point:
 *   - All functions return CURAST_OK (0) or a negative curast_status.  Argument errors are
 *     detected before any work is enqueued; nothing is enqueued on error.  No C++ exception
 *     crosses this boundary.  curast_last_error() describes the last failure of a context.
 *   - "device" pointers are HIP device allocations (e.g. torch CUDA tensor data pointers) owned
 *     by the caller; they must stay valid until the enqueued work has completed.  "host"
 *     pointers are read before the call returns.  The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued asynchronously;
 *     results are ready when the stream reaches that point.
 *   - A context owns its scratch (queues, counters, descriptor staging, graph cache) and binds
 *     to the HIP device that was current at curast_create.  Use one context per host thread;
 *     calls on one context must not overlap on different streams.
 *   - Vertex coordinates and matrices must be finite; width and height lie in [1, 16384];
 *     near > 0.  Indices >= the vertex count make their triangle produce nothing.
 */
#ifndef CURAST_H
#define CURAST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CURAST_OK = 0,
    CURAST_E_INVALID = -1,      /* null pointer, bad size, width/height/near out of range */
    CURAST_E_ID_RANGE = -2,     /* sum of triangle-instances exceeds the 36-bit ID space */
    CURAST_E_OOM = -3,          /* device or pinned host allocation failed */
    CURAST_E_HIP = -4,          /* a HIP runtime call failed (see curast_last_error) */
    CURAST_E_UNSUPPORTED = -5   /* feature not available on this device */
} curast_status;

/* Option flags. */
#define CURAST_FLAG_NO_TINY_CULL  0x1u  /* keep triangles whose bbox holds no pixel centre
                                           (result unchanged; Sec. 4.1, Table 4) */
#define CURAST_FLAG_NO_EARLY_OUT  0x2u  /* always issue the atomic, in every stage, even if the stored
                                           key is smaller (see CURAST_FLAG_EARLY_OUT_ALL) */
#define CURAST_FLAG_NO_MESH_CULL  0x4u  /* skip the host bounding-sphere frustum cull */
#define CURAST_FLAG_STATS         0x8u  /* count per-stage events (slower; read with curast_get_stats) */
#define CURAST_FLAG_NO_GRAPH      0x10u /* batched calls launch kernels directly instead of a hipGraph */
#define CURAST_FLAG_TIMING        0x20u /* record HIP events around every stage (curast_get_stage_times) */
#define CURAST_FLAG_S3_PER_PART   0x40u /* stage 3: one workgroup per tile part (Sec. 4.3) instead of
                                           the default one workgroup per binned screen tile */
#define CURAST_FLAG_NO_FAST_INTERIOR 0x80u /* stage 1: no prescaled window rows for draws whose
                                                bounding sphere lies well inside the view frustum */
#define CURAST_FLAG_NO_STRIPS     0x100u /* stage 1, meshes with several draws: do not detect
                                            triangle strips (each triangle then takes three window
                                            positions per draw) */
#define CURAST_FLAG_SINGLE_STRIPS 0x200u /* stage 1: detect triangle strips in the launch over
                                            single-draw meshes too */
#define CURAST_FLAG_S1_OVERLAP    0x400u /* stage 1: run the launch over single-draw meshes on a
                                            second stream of the context next to the launch over
                                            multi-draw meshes (forked from and joined back into the
                                            caller's stream, also under graph capture); stage times
                                            then report the multi-draw launch's span as stage1_multi
                                            and the rest of stage 1 as stage1_single */
#define CURAST_FLAG_EARLY_OUT_ALL 0x800u /* read the stored key before each atomic minimum and skip the
                                            atomic when the key is not smaller, in every stage; by
                                            default only the stage-1 launch over single-draw meshes,
                                            stage 3 and the overflow passes read first, while the
                                            stage-1 launch over multi-draw meshes and stage 2 issue
                                            the atomic directly as the paper does (Sec. 4.1), which
                                            measured faster there; CURAST_FLAG_NO_EARLY_OUT, when
                                            also set, wins (no stage reads first) */
#define CURAST_FLAG_ZERO_QUEUES   0x80000000u /* testing aid: run with stage queues of capacity 0, so
                                                 every forwarded triangle takes the overflow paths */

/* Host logging: with CURAST_LOG set in the environment to a value other than "0" (read once per
   process), the library prints one "[curast] ..." line to stderr for each context set-up, frame
   plan (meshes, views, draws kept and culled, work items), graph capture, autotuner result and
   error; unset, it prints nothing. */

/* Tuning knobs; 0 selects the default (or the autotuned value).  None of them changes results. */
typedef struct {
    uint32_t small_px;          /* stage-1 limit on pixel centres in the clamped bbox (default 32; the
                                   paper's 128, Sec. 4, measured slower here) */
    uint32_t medium_px;         /* stage-2 limit (default 4096, Sec. 4) */
    uint32_t s1_block;          /* stage-1 workgroup size: 64, 128, 256 or 512 (default 64, Sec. 4.1) */
    uint32_t s1_tris_per_thread;/* triangles per thread per stage-1 work item of a mesh drawn once:
                                   1, 2, 4 or 8 (default 4) */
    uint32_t s1_draws_per_item; /* (instance x view) draws per stage-1 work item (default 64, Sec. 4.5) */
    uint32_t s2_waves;          /* persistent stage-2 wavefronts (default 16 per CU) */
    uint32_t s3_blocks;         /* persistent stage-3 workgroups (default 2 per CU) */
    uint32_t q2_capacity;       /* stage-1 -> stage-2 queue entries (default 16M, 128 MB); overflow
                                   is rasterized in place, never dropped */
    uint32_t q3_capacity;       /* stage-2 -> stage-3 tile parts (default 1M); overflow as above */
    uint32_t large_capacity;    /* large (sub-)triangle records for stage 3 (default 256K) */
    uint32_t flags;             /* CURAST_FLAG_* */
    uint32_t s1_mode;           /* stage-1 kernel: 0 = auto (currently 2), 1 = one lane per
                                   triangle with exact arithmetic only, 2 = conservative fast reject
                                   with approximate reciprocals and wave-compacted exact work, where
                                   a strip of the multi-draw launch is first tested through the
                                   bounding sphere of its vertices, 3 = every mesh through the
                                   wave-level vertex-sharing kernel (each vertex transformed once
                                   per wave and draw), 4 = as 2 without the strip spheres */
    uint32_t s1_multi_tris_per_thread; /* as s1_tris_per_thread (1, 2, 4 or 8; 1, 2 or 4 with
                                   s1_mode 3), for meshes with two or more surviving draws, which
                                   stage 1 takes in a launch of its own; with 2 or more, a lane's
                                   consecutive triangles are tested as one strip when they form
                                   one (default 4) */
    uint32_t s1_blocks_per_cu;  /* stage-1 grid: at most this many workgroups per compute unit per
                                   launch, each looping over work items (default 2048, 1..65536) */
} curast_options;

/*
 * Compressed mesh geometry (Sec. 4.6, "Compression"): indices bit-packed relative to the mesh's
 * smallest index, positions as 16-bit fixed point relative to the mesh's bounding box.  A
 * compressed mesh renders exactly as the uncompressed mesh made of its decoded indices and
 * positions:
 *   index i (0 <= i < 3T)  = index_min + bits [i * index_bits, (i + 1) * index_bits) of the
 *                            little-endian bit stream `indices` (uint32 words, bit 0 first);
 *   position component c   = fmaf((float)positions[3 v + c], step[c], lo[c]).
 * curast_compress_prepare computes index_min, index_bits, lo and step; curast_compress fills the
 * two buffers.  The buffers are the caller's (device memory, 4-byte aligned).  Both carry
 * padding that the decoders read past the last value (a triangle's indices are read with one
 * load of up to four words, a vertex with one 8-byte load): three zero words after the index
 * stream and one zero element after the positions.
 */
typedef struct {
    const uint32_t* indices;    /* device, curast_compress_prepare's index_words uint32 words:
                                   ceil(3 T index_bits / 32) words of stream + 3 of padding */
    const uint16_t* positions;  /* device, 3 V + 1 elements: [V][3] quantized positions, then
                                   one padding element */
    uint32_t index_min;         /* smallest index of the mesh */
    uint32_t index_bits;        /* ceil(log2(max - min + 1)), at least 1 and at most 32 */
    float lo[3];                /* bounding-box minimum */
    float step[3];              /* (float)(((double)max - (double)min) / 65535) per axis */
} curast_compressed;

typedef struct {
    const float* vertices;      /* device [V][3] object-space positions */
    uint32_t num_vertices;      /* V */
    const uint32_t* indices;    /* device [T][3] vertex indices */
    uint64_t num_triangles;     /* T (at most 2^32 - 1) */
    const float* instances;     /* host [N][12] row-major 3x4 object-to-world matrices, or NULL
                                   for one identity instance */
    uint32_t num_instances;     /* N (ignored when instances is NULL) */
    float bsphere[4];           /* object-space bounding sphere (cx, cy, cz, r) containing every
                                   vertex, used for the host frustum cull; r <= 0: unknown */
    const curast_compressed* compressed; /* host, or NULL; when set, the mesh's geometry is read
                                   from it and `vertices` / `indices` are not used */
} curast_mesh;

typedef struct {
    float view_proj[16];        /* host, row-major; rows 0, 1, 3 give clip x, y and w */
    float near_plane;           /* > 0, in the units of w */
    int32_t width, height;      /* pixels, 1..16384 */
    uint64_t* visbuffer;        /* device [height][width], row 0 at the bottom */
} curast_view;

typedef struct {
    uint64_t tri_draws;         /* triangle x instance x view items submitted after the mesh cull */
    uint64_t draws_culled;      /* (mesh, instance, view) draws removed by the host cull */
    uint64_t culled_near;       /* all three vertices behind the near plane */
    uint64_t culled_frustum;    /* all vertices outside one side of the view */
    uint64_t culled_tiny;       /* bbox holds no pixel centre (Sec. 4.1, Table 4); also the fast
                                   stage-1 tests' rejections of triangles and strips wholly
                                   beyond a side or the near plane */
    uint64_t culled_backface;   /* snapped area <= 0 */
    uint64_t s1_rasterized;     /* triangles rasterized in stage 1 */
    uint64_t q2_entries;        /* triangles forwarded to stage 2 (high-water mark of the queue) */
    uint64_t q2_overflow;       /* forwarded triangles that did not fit and were rasterized in place */
    uint64_t s2_rasterized;     /* (sub-)triangles rasterized in stage 2 */
    uint64_t q3_entries;        /* tile parts forwarded to stage 3 */
    uint64_t q3_overflow;       /* (sub-)triangles stage 2 rasterized itself because stage 3 was full */
    uint64_t fragments;         /* covered pixel samples */
    uint64_t atomics;           /* 64-bit atomic minimums issued (the rest skipped by the early-out) */
    uint64_t strip_draws;       /* (strip, draw) pairs of the multi-draw stage-1 launch's strip path */
    uint64_t strip_union_pass;  /* of those, strips whose union box may hold a pixel centre (their
                                   triangles then take the per-triangle test) */
    uint64_t strip_sphere_pass; /* (strip, draw) pairs whose bounding-sphere test could not reject
                                   the strip (they then take the union-box test; s1_mode 0 and 2) */
} curast_stats;

typedef struct curast_ctx curast_ctx;

/* Create a context on the current HIP device.  opt may be NULL (all defaults).
   Errors: CURAST_E_INVALID (out NULL or an option out of range), CURAST_E_OOM, CURAST_E_HIP. */
int curast_create(const curast_options* opt, curast_ctx** out);

/* Destroy a context after its enqueued work has completed.  NULL is accepted. */
int curast_destroy(curast_ctx* ctx);

/* Replace / read the context options (same validation as curast_create). */
int curast_set_options(curast_ctx* ctx, const curast_options* opt);
int curast_get_options(const curast_ctx* ctx, curast_options* opt);

/*
 * Rasterize one mesh (optionally instanced, Sec. 4.5) into one view: the call shape of the paper's
 * frame (host cull + mesh list + stages 1-3, Sec. 4).  Clears `visbuffer` first.
 *   vertices  device [V][3]; indices device [T][3]; instances host [N][12] or NULL;
 *   view_proj host [16] row-major; visbuffer device [height][width].
 * Errors: CURAST_E_INVALID, CURAST_E_ID_RANGE (T * N >= 2^36), CURAST_E_HIP.
 */
int curast_rasterize(curast_ctx* ctx, const float* vertices, uint32_t num_vertices,
                     const uint32_t* indices, uint64_t num_triangles, const float* instances,
                     uint32_t num_instances, const float view_proj[16], float near_plane,
                     int32_t width, int32_t height, uint64_t* visbuffer, void* stream);

/*
 * Allocation-free form of curast_rasterize, for callers that cannot allocate memory: code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * the same visibility buffer as curast_rasterize; it calls no hipMalloc, hipFree, hipMemcpy or
 * hipMemset, and on the host it allocates nothing either (except the message it stores when it
 * returns an error).  The plan is built in fixed arrays, its
 * descriptors go to the device as the argument of one small kernel, and descriptors, queues,
 * counters and stage-3 bins live in a file-scope device array of about 17 MB per device (held
 * until the process ends; its address is taken once per device by curast_create), instead of the
 * context's buffers.  Its stage-2 queue holds 1M entries, its large-triangle store 64K records and
 * its stage-3 queue 512K tile parts (the context's capacities when those are smaller); overflow
 * falls back to in-place rasterization as in curast_rasterize, so results do not change.
 * Limits: at most 32 instances (CURAST_E_INVALID beyond), views up to 16384 x 16384;
 * CURAST_FLAG_STATS and CURAST_FLAG_TIMING are ignored.  All calls on one device share the one
 * array and it keeps the last call's contents (the clear kernel zeroes the counters and bins each
 * call needs): calls whose work overlaps on one device (other streams, other host threads) race.
 */
int curast_rasterize_noalloc(curast_ctx* ctx, const float* vertices, uint32_t num_vertices,
                             const uint32_t* indices, uint64_t num_triangles, const float* instances,
                             uint32_t num_instances, const float view_proj[16], float near_plane,
                             int32_t width, int32_t height, uint64_t* visbuffer, void* stream);

/*
 * Rasterize a list of meshes (Sec. 4: host-side mesh list with per-mesh/instance triangle-count
 * prefix sums) into one view.  meshes: host array of M descriptors.  Clears the view's buffer.
 */
int curast_rasterize_meshes(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M,
                            const curast_view* view, void* stream);

/*
 * Rasterize the same meshes into n_views views of independent sizes and cameras in one
 * persistent launch sequence (captured once into a hipGraph and replayed; Sec. 4.1 persistent
 * work loop and Sec. 4.5 instancing loop, extended over views).  Each stage-1 lane loads a
 * triangle once and draws it for every (instance, view) that survived the host cull.  Every
 * view's buffer equals what curast_rasterize_meshes would produce for it alone; IDs are shared.
 * views: host array; each visbuffer a distinct device allocation.
 */
int curast_rasterize_batched(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M,
                             const curast_view* views, uint32_t n_views, void* stream);

/*
 * Unsnapped window positions of one mesh instance for a view: pos_ss device [V][3] =
 * (sx, sy, w) with sx = fmaf(x*zI, W/2, W/2), sy likewise, zI = 1/w: the rasterizer's values
 * before the rounding to 1/256 pixel.
 * These are the differentiable inputs of curast_resolve_screen / curast_resolve_backward.
 */
int curast_project(curast_ctx* ctx, const curast_mesh* mesh, uint32_t instance,
                   const curast_view* view, float* pos_ss, void* stream);

/*
 * Compression (Sec. 4.6), step 1: from the uncompressed mesh (vertices and indices set), the
 * smallest and largest index and the positions' bounding box, giving info->index_min,
 * index_bits, lo and step, and the size of the packed index stream in uint32 words
 * (ceil(3 T index_bits / 32) + 3).  Synchronizes the stream.  info->indices / positions are not
 * touched.
 */
int curast_compress_prepare(curast_ctx* ctx, const curast_mesh* mesh, curast_compressed* info,
                            uint64_t* index_words, void* stream);

/*
 * Compression, step 2: writes the packed indices (index_words words, every bit defined, the
 * padding 0) and the 3 V + 1 position elements (the last one 0): quantized positions q = clamp(rint((p - lo) * scale), 0, 65535) with
 * scale = (float)(1.0 / (double)step) per axis (0 for a flat axis), the subtraction and product
 * in binary32, rint rounding half to even.
 */
int curast_compress(curast_ctx* ctx, const curast_mesh* mesh, const curast_compressed* info,
                    uint32_t* packed_indices, uint16_t* positions, void* stream);

/*
 * Resolve a view's visibility buffer into interpolated attributes (Sec. 4.4): per pixel decode
 * the 36-bit ID, binary-search the (mesh, instance) in the int64 prefix of triangle counts,
 * recompute the three vertices and interpolate perspective-correctly at the pixel centre.
 *   attrs: host array of M device pointers, mesh m's per-vertex attributes [V_m][C];
 *   out: device [height][width][C] float; empty pixels get 0.  1 <= C <= 16.
 */
int curast_resolve(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                   const float* const* attrs, uint32_t C, float* out, void* stream);

/*
 * Supersampled resolve (anti-aliasing, Sec. 5 "Anti-Aliasing (Super Sampling)", Table 5):
 * `view` is the view at samples_per_axis times the output size in each direction (same
 * view_proj), whose visibility buffer curast_rasterize_meshes filled, so every output pixel owns
 * a samples_per_axis x samples_per_axis block of samples at regular offsets.  Each sample is
 * resolved as in curast_resolve; the output pixel is their fp32 sum, taken row by row with empty
 * samples adding 0, times 1 / samples_per_axis^2.
 *   samples_per_axis: 1, 2 or 4 (1 is curast_resolve); the view's width and height must be
 *   multiples of it;
 *   out: device [height / s][width / s][C] float.  1 <= C <= 16.
 */
int curast_resolve_supersampled(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                                uint32_t samples_per_axis, const float* const* attrs, uint32_t C, float* out,
                                void* stream);

/*
 * A mip-mapped RGBA8 texture for curast_resolve_textured.  Texel (i, j) of level l holds R in
 * bits 0-7, G in 8-15, B in 16-23, A in 24-31, decoded as byte * (1.0f / 255.0f).  Level l is
 * max(1, width >> l) x max(1, height >> l) texels, row-major, row j at texture coordinate
 * v = (j + 0.5) / height_l; the levels follow each other without gaps, level 0 first, so
 * `texels` holds sum over l of width_l * height_l words (curast_texture_texels).
 */
typedef struct {
    const uint32_t* texels;     /* device */
    uint32_t width, height;     /* level 0: powers of two in [1, 16384] */
    uint32_t levels;            /* 1 .. 1 + log2(max(width, height)) */
} curast_texture;

/* Texels of a texture with all its levels (0 for an invalid size or level count). */
uint64_t curast_texture_texels(uint32_t width, uint32_t height, uint32_t levels);

/*
 * Fill levels 1 .. levels - 1 of a texture from level 0: texel (i, j) of level l + 1 is the
 * per-channel mean of texels (2i, 2j), (2i + 1, 2j), (2i, 2j + 1), (2i + 1, 2j + 1) of level l,
 * with coordinates clamped to level l and the sum rounded as (a + b + c + d + 2) >> 2.  Level 0 is
 * not touched.  texels: device, curast_texture_texels(width, height, levels) words.
 */
int curast_build_mips(curast_ctx* ctx, uint32_t* texels, uint32_t width, uint32_t height, uint32_t levels,
                      void* stream);

/*
 * Textured resolve with world-space mip-level selection (Sec. 4.4, "Shading and Mip Mapping").
 * For a covered pixel (px, py) of the view, the rays through the window points
 * (px + 0.5, py + 0.5), (px + 1.5, py + 0.5), (px + 0.5, py + 1.5) and (px + 1.5, py + 1.5)
 * (the pixel and its right, top and top-right neighbours; row 0 is at the bottom) are intersected
 * with the plane of the pixel's triangle, and the UVs of the intersections are interpolated or
 * extrapolated from its vertices.  Barycentrics of a ray-plane hit do not change under the
 * affine map from world to clip space, so they are solved there, which needs no division by w
 * and holds for vertices behind the camera: with n = ((sx - W/2) / (W/2), (sy - H/2) / (H/2)),
 *   a_k = fmaf(-n.x, w_k, x_k),  c_k = fmaf(-n.y, w_k, y_k)      (clip x, y, w of vertex k)
 *   e = a x c  (e0 = a1 c2 - a2 c1, ...),  s = (e0 + e1) + e2
 *   u = ((e0 u0 + e1 u1) + e2 u2) / s,  v likewise.
 * The level of detail is lod = log2(max((u_max - u_min) width, (v_max - v_min) height)) over the
 * four hits, clamped to [0, levels - 1]; levels - 1 when a hit is not finite.  The colour is the
 * trilinear sample at the first hit: bilinear within a level (texel centres at (i + 0.5) / w_l,
 * wrap-around addressing, weights from x = frac(u) w_l - 0.5), blended between levels
 * floor(lod) and floor(lod) + 1 by lod - floor(lod).  Every step is binary32 with the operation
 * order above.
 *   uvs: host array of M device pointers, mesh m's per-vertex texture coordinates [V_m][2];
 *   textures: host array of M textures (meshes may share one);
 *   out: device [height][width][4] float RGBA; empty pixels and pixels whose centre hit is not
 *   finite get 0.
 */
int curast_resolve_textured(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                            const float* const* uvs, const curast_texture* textures, float* out, void* stream);

/*
 * Resolve one mesh from explicit screen positions (the differentiable form):
 *   visbuffer device [H][W]; indices device [T][3]; pos_ss device [V][3] (sx, sy, w);
 *   attrs device [V][C]; out device [H][W][C].  Pixels whose ID is outside
 *   [id_base, id_base + T) (other meshes, empty) get 0.  Same arithmetic as curast_resolve.
 */
int curast_resolve_screen(curast_ctx* ctx, const uint64_t* visbuffer, int32_t width, int32_t height,
                          const uint32_t* indices, uint64_t num_triangles, uint64_t id_base,
                          const float* pos_ss, uint32_t num_vertices, const float* attrs, uint32_t C,
                          float* out, void* stream);

/*
 * Backward of curast_resolve_screen with visibility held fixed: for every covered pixel,
 * scatter-add grad_out through the barycentrics into grad_attr [V][C] and, through the
 * barycentrics' dependence on (sx, sy, w) of the three vertices, into grad_pos [V][3].
 * Gradients are ACCUMULATED with float atomics (the caller zeroes them); grad_pos may be NULL.
 * The accumulation order is not deterministic (float addition is not associative).
 */
int curast_resolve_backward(curast_ctx* ctx, const uint64_t* visbuffer, int32_t width, int32_t height,
                            const uint32_t* indices, uint64_t num_triangles, uint64_t id_base,
                            const float* pos_ss, uint32_t num_vertices, const float* attrs, uint32_t C,
                            const float* grad_out, float* grad_attr, float* grad_pos, void* stream);

/*
 * Backward of curast_resolve (the multi-mesh, multi-instance resolve of Sec. 4.4) with visibility
 * held fixed: for every covered pixel of view->visbuffer, the pixel's (mesh, instance) and
 * triangle are found as in the forward, its vertices projected with the same fp32 operations, and
 * grad_out [H][W][C] is scattered through the barycentrics (the chain rule of
 * curast_resolve_backward, fp64 per pixel, each contribution rounded once to fp32).
 *   attrs       host [M] array of device [V_m][C] attribute pointers (as curast_resolve);
 *   grad_out    device [H][W][C];
 *   grad_attrs  host [M] array of device [V_m][C] pointers, ACCUMULATED (the caller zeroes them);
 *               the instances of a mesh add into its one set of rows; a NULL entry skips mesh m;
 *   grad_pos    NULL, or host [M] array of device [V_m][3] pointers or NULL entries, ACCUMULATED:
 *               gradients to the unsnapped window positions (sx, sy, w) that curast_project gives
 *               for mesh m's only instance (a non-NULL entry for a mesh with several instances is
 *               CURAST_E_INVALID).
 * Float atomics: the accumulation order is not deterministic.  Errors: CURAST_E_INVALID (NULL
 * pointers, C outside [1, 16], a bad view or mesh), CURAST_E_ID_RANGE, CURAST_E_HIP.
 */
int curast_resolve_backward_meshes(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M,
                                   const curast_view* view, const float* const* attrs, uint32_t C,
                                   const float* grad_out, float* const* grad_attrs,
                                   float* const* grad_pos, void* stream);

/*
 * Pick stage thresholds, workgroup sizes, work-item sizes and queue capacities for this scene
 * by timing candidates with HIP events (coordinate descent over a fixed grid, Sec. 4's
 * "experimentally determined" thresholds made automatic).  Results never change outputs.
 * The chosen options are applied to ctx, returned in `chosen` (may be NULL) and, when
 * cache_path is not NULL, stored in a JSON file keyed by device and scene class; an existing
 * entry for the same key is loaded instead of measuring.  views' visbuffers are overwritten.
 * Candidates are timed with the context's stage timers (GPU time of the frame's kernels), which
 * are reset.  Queue capacities are raised to twice the measured fill when that exceeds the
 * library defaults and are never set below the defaults, so a cached choice does not push a
 * busier scene of the same class into the in-place overflow path (q2_overflow / q3_overflow in
 * curast_stats count triangles that took it).
 */
int curast_autotune(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* views,
                    uint32_t n_views, const char* cache_path, curast_options* chosen, void* stream);

/* Statistics accumulated since the last reset (needs CURAST_FLAG_STATS; synchronizes ctx's work). */
int curast_get_stats(curast_ctx* ctx, curast_stats* out);
int curast_reset_stats(curast_ctx* ctx);

/* Stage durations accumulated over frames run with CURAST_FLAG_TIMING, measured with HIP events
   on the launch stream (synchronizes those events): ms[0..8] = clear, stage-1 launch over the
   meshes with two or more draws (all meshes when s1_mode = 3), stage-1 launch over the other
   meshes, stage-1 overflow pass, stage 2, stage 3, resolve (either form), resolve backward, whole
   rasterized frame; *frames = number of rasterized frames timed.
   Batched (graph) frames contribute only the whole-frame time. */
int curast_get_stage_times(curast_ctx* ctx, double ms[9], uint64_t* frames);
int curast_reset_stage_times(curast_ctx* ctx);

/*
 * Host-side frame planning only (no GPU; Sec. 4 host mesh list): validates the arguments as the
 * rasterize calls do and reports which (mesh, instance, view) draws survive the conservative
 * bounding-sphere frustum cull.  visible: host [pairs][n_views] bytes (0 = culled, 1 = drawn,
 * 2 = drawn and proven to lie in front of the near plane inside |x|, |y| <= 1.99 w) or NULL;
 * bases: host [pairs + 1] exclusive prefix of triangle counts or NULL; counts: host [4] = draws
 * kept, draws culled, stage-1 work items, triangle x draw items, or NULL.  Views' visbuffer
 * pointers must be non-NULL but are not touched.
 */
int curast_plan(const curast_mesh* meshes, uint32_t M, const curast_view* views, uint32_t n_views,
                const curast_options* opt, uint8_t* visible, int64_t* bases, uint64_t counts[4]);

/* Exclusive prefix of triangle counts over all (mesh, instance) pairs (host only, no GPU):
   bases host [pairs + 1]; returns the number of pairs (>= 0) or a negative status. */
int64_t curast_id_bases(const curast_mesh* meshes, uint32_t M, int64_t* bases);

/* Static description of a status code; the last error message of a context (never NULL). */
const char* curast_status_string(int status);
const char* curast_last_error(const curast_ctx* ctx);

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int curast_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CURAST_H */

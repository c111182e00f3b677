// Descriptors shared by the host runtime and the gfx950 kernels of the rasterizer.
//
// Memory layout in HBM (all written by the host runtime each frame, read-only in kernels):
//   FrameHeader | ViewDesc[n_views] | MeshDesc[M] | Segment[n_segs] | DrawDesc[n_draws]
// plus context-owned scratch: the stage queues (Q2, large-triangle records, Q3) and counters.
// Per-vertex and per-index data stay in the caller's buffers ([V][3] float, [T][3] uint32) and are
// streamed once per frame by stage 1 (the paper's bandwidth-bound hot loop, Sec. 4.5).
#pragma once

#include <stdint.h>

namespace curast {

constexpr float kGuardBand = 16.0f;               // |x|, |y| <= 16 w needs no clipping
constexpr uint64_t kIdMask = (uint64_t(1) << 36) - 1;
constexpr uint64_t kEmptyKey = ~uint64_t(0);
constexpr int kTileSize = 64;                     // stage-3 screen tile (Sec. 4.2)
constexpr int kMaxDim = 16384;
constexpr uint32_t kNullRecord = 0xFFFFFFFFu;
// Stage 1 keeps triangles whose snapped bounding box spans less than this many 1/256-px units in
// x and y: every edge-function value at a pixel centre of the box (and one step past it) then
// fits in int32 (|E| <= 2 * ext * (ext + 384) < 2^31).
constexpr int32_t kSmallExtent = 32768 - 512;

struct FrameHeader {              // 48 B
    uint64_t total_batches;       // stage-1 work items over all segments
    uint32_t n_segs;
    uint32_t n_views;
    uint32_t batch_tris;          // triangles per work item of the plain stage-1 kernels
    uint32_t draws_per_item;      // draws per work item
    uint64_t shared_batches;      // work items [0, shared_batches) belong to meshes drawn more than once
    uint32_t n_tiles;             // 64x64 screen tiles over all views (stage-3 bins)
    uint32_t pad0;
    uint64_t pad1;
};

struct ViewDesc {                 // 48 B
    unsigned long long* vis;      // [H][W]
    int32_t W, H;
    float hW, hH;                 // W/2, H/2 (exact)
    float near_plane;
    uint32_t tile_base;           // first stage-3 tile of this view; its tiles are row-major
    float wmax, hmax;             // W - 1, H - 1 (exact)
    uint32_t pad[2];
};

struct MeshDesc {                 // 80 B
    const float* pos;             // [V][3], or NULL when compressed
    const uint32_t* idx;          // [T][3], or the packed index stream when compressed
    const uint16_t* qpos;         // [3 V + 1] quantized positions (+1 padding) when compressed, else NULL
    uint64_t T;
    uint32_t V;
    uint32_t idx_bits;            // 0: plain indices; else bits per packed index
    uint32_t idx_min;             // added to every packed index
    float lo[3], step[3];         // position = fmaf(q, step, lo) when compressed
    uint32_t pad;
};

// A run of stage-1 work items over one mesh: work item j of the segment covers the triangle batch
// j / n_groups and the draw group j % n_groups (consecutive items share triangles, so the
// index/vertex lines they read are still in L2 when the next draw group needs them).
struct Segment {                  // 32 B
    uint64_t batch_begin;         // first global work item of the segment
    uint32_t mesh;
    uint32_t draw_begin;          // first draw of the mesh
    uint32_t draw_count;          // draws of the mesh that survived the host cull
    uint32_t n_groups;            // ceil(draw_count / draws_per_item)
    uint32_t batch_tris;          // triangles per work item of this segment
    uint32_t pad;
};

// One (mesh, instance, view): rows x, y, w of VP * X, the global ID of triangle 0, the view.
// Bit 31 of `view` (kDrawInterior) marks draws whose bounding sphere the host proved to lie in
// front of the near plane and inside |x|, |y| <= 1.99 w: no vertex of such a draw needs the
// per-vertex near/guard tests of the fast stage-1 path.
struct DrawDesc {                 // 112 B
    float A[12];                  // rows x, y, w of VP * X (the exact transform)
    float R[8];                   // interior draws: hW (row x + row w), hH (row y + row w)
    uint64_t id_base;
    uint32_t view;                // view index | kDrawInterior
    uint32_t mesh;
    float wnorm;                  // interior draws: |(A[8], A[9], A[10])| rounded up (strip spheres)
    float slack;                  // interior draws: pixels added to a strip sphere's projected radius
    float wmax, hmax;             // W - 1, H - 1 of the view (copied, so the sphere test reads one record)
};
constexpr uint32_t kDrawInterior = 0x80000000u;
constexpr uint32_t kDrawViewMask = 0x7FFFFFFFu;

struct Q2Entry {                  // triangle forwarded by stage 1
    uint32_t draw;
    uint32_t tri;
};

struct LargeTri {                 // snapped (sub-)triangle forwarded by stage 2, 48 B
    int32_t X[3], Y[3];
    float zI[3];
    uint32_t view;
    uint64_t id;
};

struct Q3Entry {                  // one 64x64 tile part of a large triangle
    uint32_t rec;                 // LargeTri index or kNullRecord
    uint16_t tx, ty;
};

enum Counter : int {
    kCntQ2 = 0,                   // entries appended to Q2 (may exceed its capacity)
    kCntLarge = 1,                // large records reserved
    kCntQ3 = 2,                   // Q3 entries reserved
    kNumCounters = 4
};

enum Stat : int {
    kStTriDraws = 0, kStDrawsCulled, kStCulledNear, kStCulledFrustum, kStCulledTiny,
    kStCulledBack, kStS1Raster, kStQ2, kStQ2Overflow, kStS2Raster, kStQ3, kStQ3Overflow,
    kStFragments, kStAtomics, kStStripDraws, kStStripPass, kStSpherePass, kNumStats
};

// Option flags mirrored from the public header.
constexpr uint32_t kFlagNoTinyCull = 0x1u;
constexpr uint32_t kFlagNoEarlyOut = 0x2u;
constexpr uint32_t kFlagNoMeshCull = 0x4u;
constexpr uint32_t kFlagStats = 0x8u;
constexpr uint32_t kFlagNoGraph = 0x10u;
constexpr uint32_t kFlagS3PerPart = 0x40u;          // stage 3 per tile part instead of per binned tile
constexpr uint32_t kFlagNoFastInterior = 0x80u;     // no prescaled interior draws in stage 1
constexpr uint32_t kFlagNoStrips = 0x100u;          // no triangle strips in stage 1
constexpr uint32_t kFlagSingleStrips = 0x200u;      // strips in the single-draw stage-1 launch too
constexpr uint32_t kFlagS1Overlap = 0x400u;         // the two stage-1 launches on two streams at once
constexpr uint32_t kFlagEarlyOutAll = 0x800u;       // read the stored key before the atomic in every stage
constexpr uint32_t kFlagZeroQueues = 0x80000000u;   // testing aid: queue capacities of zero

struct RasterArgs {
    const FrameHeader* hdr;
    const ViewDesc* views;
    const MeshDesc* meshes;
    const Segment* segs;
    const DrawDesc* draws;
    Q2Entry* q2;
    LargeTri* large;
    Q3Entry* q3;
    unsigned long long* counters;
    unsigned long long* stats;
    uint32_t q2_cap, large_cap, q3_cap;
    uint32_t small_px, medium_px;
    uint32_t flags;
    uint32_t s1_mode;             // 0 auto (= 2), 1 exact only, 2 fast reject (strip spheres in the
                                  // multi-draw launch), 3 vertex sharing for every mesh, 4 as 2 without spheres
    uint32_t part;                // stage-1 work items: 0 all, 1 the shared prefix, 2 the rest
    uint32_t* tile_count;         // [n_tiles] parts per tile (zeroed by the clear kernel)
    uint32_t* tile_offset;        // [n_tiles + 1] exclusive prefix of tile_count
    uint32_t* q3_binned;          // [q3_cap] large-record index of every part, grouped by tile
    uint32_t compressed_parts;    // bit p: stage-1 part p has a compressed mesh; bit p + 8: every
                                  // mesh of part p is compressed (host-side kernel choice)
};

// A mip-mapped RGBA8 texture: level l is max(1, w >> l) x max(1, h >> l) texels from off[l].
struct TexDesc {
    const uint32_t* texels;
    uint32_t w, h, levels, pad;
    uint32_t off[16];
};

struct ResolveArgs {
    const unsigned long long* vis;
    int32_t W, H;
    float hW, hH;
    const uint64_t* bases;        // [n_meshes + 1] first global ID of each mesh (its instances follow
                                  // one another, T IDs apart); the last entry is the ID count
    const uint32_t* mesh_pair;    // [n_meshes] index of each mesh's first (mesh, instance) pair
    const DrawDesc* pairs;        // [n_pairs] draw matrix of every (mesh, instance) for this view
    const MeshDesc* meshes;
    const float* const* attrs;    // [M] per-mesh attribute pointers
    uint32_t n_pairs;
    uint32_t n_meshes;
    uint32_t C;
    float* out;                   // [H][W][C], or [H/ss][W/ss][C] when supersampled
    uint32_t ss;                  // samples per axis and output pixel (1: no supersampling)
    const TexDesc* tex;           // [M] textures of the textured resolve (attrs are then the UVs)
    const float* grad_out;        // backward input [H][W][C]
    float* const* grad_attrs;     // [M] per-mesh attribute gradients [V][C] (accumulated), entries may be null
    float* const* grad_pos;       // [M] per-mesh window-position gradients [V][3], or null (one-instance meshes)
};

struct ScreenArgs {
    const unsigned long long* vis;
    int32_t W, H;
    const uint32_t* idx;
    uint64_t T;
    uint64_t id_base;
    const float* pos_ss;          // [V][3]
    uint32_t V;
    const float* attrs;           // [V][C]
    uint32_t C;
    float* out;                   // forward output [H][W][C]
    const float* grad_out;        // backward input [H][W][C]
    float* grad_attr;             // [V][C]
    float* grad_pos;              // [V][3] or null
};

}  // namespace curast

// Host runtime of the rasterizer and its C ABI (include/curast.h).
//
// Per frame the host (Sec. 4: "before launching the rasterization stages") computes the draw
// matrix of every (mesh, instance, view), the int64 exclusive prefix of triangle counts that
// gives global triangle IDs, culls whole (mesh, instance, view) draws by their bounding sphere,
// splits the surviving work into stage-1 work items, and uploads these descriptors with one
// asynchronous copy from pinned memory.  Everything after that (clear, stages 1-3, resolve) is
// device-side and reads counts from device memory, so a batched frame is captured once into a
// hipGraph and replayed with new descriptor contents.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/curast.h"
#include "common.h"
#include "log.h"

namespace curast {
hipError_t launch_clear(const RasterArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_stage1(const RasterArgs& a, uint32_t block, uint32_t tpt, bool stats, uint32_t grid, hipStream_t s);
hipError_t launch_stage1_fast(const RasterArgs& a, uint32_t block, uint32_t tpt, bool strips, bool spheres, bool stats,
                              uint32_t grid, hipStream_t s);
hipError_t launch_stage1_share(const RasterArgs& a, uint32_t tpt, bool stats, uint32_t grid, hipStream_t s);
hipError_t launch_stage1_overflow(const RasterArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_stage2(const RasterArgs& a, uint32_t grid, bool stats, hipStream_t s);
hipError_t launch_stage3(const RasterArgs& a, uint32_t grid, bool stats, hipStream_t s);
hipError_t launch_stage3_binned(const RasterArgs& a, uint32_t grid, bool stats, hipStream_t s);
hipError_t launch_project(const MeshDesc& mesh, const float A[12], float hW, float hH, float* out, hipStream_t s);
hipError_t launch_compress_ranges(const uint32_t* idx, uint64_t n_idx, const float* pos, uint32_t V, uint32_t* out,
                                  uint32_t cus, hipStream_t s);
hipError_t launch_compress(const uint32_t* idx, uint64_t n_idx, uint32_t bits, uint32_t base, uint32_t* packed,
                           uint64_t words, const float* pos, uint32_t V, const float lo[3], const float scale[3],
                           uint16_t* qpos, hipStream_t s);
hipError_t launch_resolve(const ResolveArgs& a, hipStream_t s);
hipError_t launch_resolve_textured(const ResolveArgs& a, hipStream_t s);
hipError_t launch_build_mips(uint32_t* texels, uint32_t w, uint32_t h, uint32_t levels, hipStream_t s);
hipError_t launch_resolve_screen(const ScreenArgs& a, hipStream_t s);
hipError_t launch_resolve_backward(const ScreenArgs& a, hipStream_t s);
hipError_t launch_resolve_backward_meshes(const ResolveArgs& a, hipStream_t s);
}  // namespace curast

using namespace curast;

namespace {

constexpr uint64_t kMaxIds = uint64_t(1) << 36;

// Stage timing slots (CURAST_FLAG_TIMING).
enum Slot : int {
    kTClear = 0, kTS1Share, kTS1Plain, kTS1Overflow, kTS2, kTS3, kTResolve, kTResolveBwd, kTFrame, kNumSlots
};

struct TimedFrame {
    hipEvent_t ev[kNumSlots + 1];
    int used[kNumSlots];
};

// Pinned staging buffer + device buffer + event guarding reuse of the host side.
struct Staging {
    void* host = nullptr;
    void* dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

struct GraphEntry {
    uint64_t key[11];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct curast_ctx {
    int device = 0;
    int cus = 256;
    curast_options user{};
    curast_options opt{};   // user options with defaults filled in
    std::string err;
    Staging raster_stage, resolve_stage;
    Q2Entry* q2 = nullptr;
    LargeTri* large = nullptr;
    Q3Entry* q3 = nullptr;
    uint32_t q2_alloc = 0, large_alloc = 0, q3_alloc = 0;
    unsigned long long* counters = nullptr;
    unsigned long long* stats = nullptr;
    uint32_t* tile_count = nullptr;
    uint32_t* tile_offset = nullptr;
    uint32_t* q3_binned = nullptr;
    uint32_t tiles_alloc = 0;
    hipStream_t capture_stream = nullptr;
    // the second stream of the overlapped stage-1 launches, and the events that fork it from the
    // caller's stream and join it back
    hipStream_t side_stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    std::vector<GraphEntry> graphs;
    std::vector<TimedFrame> timed;
    std::vector<hipEvent_t> event_pool;   // timing events of collected frames, reused by later frames
    double stage_ms[kNumSlots] = {0};
    uint64_t timed_frames = 0;
    uint64_t draws_culled = 0;
    uint32_t* ranges = nullptr;   // [8] index range and bounding box of curast_compress_prepare
    char* na_scratch = nullptr;   // this device's copy of the allocation-free form's scratch array
};

namespace {

int fail(curast_ctx* ctx, int code, const std::string& msg)
{
    log_line("error %d: %s", code, msg.c_str());
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(curast_ctx* ctx, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    log_line("error %d: %s", CURAST_E_HIP, m.c_str());
    if (ctx) ctx->err = m;
    return CURAST_E_HIP;
}

// One log line describing a frame's plan (CURAST_LOG).
template <class PlanType>
void log_plan(const char* what, const PlanType& P, uint32_t M, uint32_t n_views)
{
    if (!log_on()) return;
    size_t interior = 0;
    for (const auto& D : P.draws) interior += (D.view & kDrawInterior) ? 1 : 0;
    log_line("%s: %u meshes, %u views, %zu draws (%zu interior, %llu culled), %llu work items (%llu multi-draw), "
             "%llu triangle x draw items, %llu pixels",
             what, M, n_views, (size_t)P.draws.size(), interior, (unsigned long long)P.draws_culled,
             (unsigned long long)P.hdr.total_batches, (unsigned long long)P.hdr.shared_batches,
             (unsigned long long)P.tri_draws, (unsigned long long)P.total_pixels);
}

#define HIP_TRY(ctx, expr)                                  \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

int validate_options(const curast_options& o, std::string& msg)
{
    auto bad = [&](const char* m) { msg = m; return CURAST_E_INVALID; };
    if (o.s1_block && o.s1_block != 64 && o.s1_block != 128 && o.s1_block != 256 && o.s1_block != 512)
        return bad("s1_block must be 64, 128, 256 or 512");
    if (o.s1_tris_per_thread && o.s1_tris_per_thread != 1 && o.s1_tris_per_thread != 2 && o.s1_tris_per_thread != 4 &&
        o.s1_tris_per_thread != 8)
        return bad("s1_tris_per_thread must be 1, 2, 4 or 8");
    if (o.s1_multi_tris_per_thread && o.s1_multi_tris_per_thread != 1 && o.s1_multi_tris_per_thread != 2 &&
        o.s1_multi_tris_per_thread != 4 && o.s1_multi_tris_per_thread != 8)
        return bad("s1_multi_tris_per_thread must be 1, 2, 4 or 8");
    if (o.s1_mode == 3 && o.s1_multi_tris_per_thread == 8)
        return bad("s1_mode 3 takes s1_multi_tris_per_thread 1, 2 or 4");
    if (o.small_px > 65536) return bad("small_px must be <= 65536");
    if (o.s1_mode > 4) return bad("s1_mode must be 0, 1, 2, 3 or 4");
    if (o.s1_draws_per_item > 65536) return bad("s1_draws_per_item must be <= 65536");
    if (o.s1_blocks_per_cu > 65536) return bad("s1_blocks_per_cu must be <= 65536");
    if (o.q2_capacity > (1u << 30) || o.q3_capacity > (1u << 30) || o.large_capacity > (1u << 28))
        return bad("queue capacity too large");
    return CURAST_OK;
}

curast_options resolve_defaults(const curast_options& u, int cus)
{
    curast_options o = u;
    if (!o.small_px) o.small_px = 32;
    if (!o.medium_px) o.medium_px = 4096;
    if (!o.s1_block) o.s1_block = 64;
    if (!o.s1_tris_per_thread) o.s1_tris_per_thread = 4;
    if (!o.s1_multi_tris_per_thread) o.s1_multi_tris_per_thread = 4;
    if (!o.s1_draws_per_item) o.s1_draws_per_item = 64;
    if (!o.s1_blocks_per_cu) o.s1_blocks_per_cu = 2048;
    if (!o.s2_waves) o.s2_waves = (uint32_t)cus * 16;
    if (!o.s3_blocks) o.s3_blocks = (uint32_t)cus * 2;
    if (!o.q2_capacity) o.q2_capacity = 1u << 24;
    if (!o.q3_capacity) o.q3_capacity = 1u << 20;
    if (!o.large_capacity) o.large_capacity = 1u << 18;
    return o;
}

void drop_graphs(curast_ctx* ctx)
{
    for (auto& g : ctx->graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        if (g.graph) hipGraphDestroy(g.graph);
    }
    ctx->graphs.clear();
}

int ensure_tiles(curast_ctx* ctx, uint32_t n_tiles)
{
    if (n_tiles + 1 <= ctx->tiles_alloc) return CURAST_OK;
    const uint32_t n = std::max<uint32_t>(n_tiles + 1, 4096);
    if (ctx->tile_count) hipFree(ctx->tile_count);
    if (ctx->tile_offset) hipFree(ctx->tile_offset);
    ctx->tile_count = ctx->tile_offset = nullptr;
    ctx->tiles_alloc = 0;
    if (hipMalloc(&ctx->tile_count, sizeof(uint32_t) * n) != hipSuccess ||
        hipMalloc(&ctx->tile_offset, sizeof(uint32_t) * n) != hipSuccess)
        return fail(ctx, CURAST_E_OOM, "tile bin allocation failed");
    ctx->tiles_alloc = n;
    drop_graphs(ctx);
    return CURAST_OK;
}

int ensure_staging(curast_ctx* ctx, Staging& st, size_t bytes)
{
    if (st.pending) {
        HIP_TRY(ctx, hipEventSynchronize(st.ev));
        st.pending = false;
    }
    if (bytes <= st.cap) return CURAST_OK;
    size_t cap = std::max<size_t>(bytes, std::max<size_t>(st.cap * 2, 64 * 1024));
    if (st.host) hipHostFree(st.host);
    if (st.dev) hipFree(st.dev);
    st.host = nullptr;
    st.dev = nullptr;
    st.cap = 0;
    if (hipHostMalloc(&st.host, cap, hipHostMallocDefault) != hipSuccess) return fail(ctx, CURAST_E_OOM, "pinned staging allocation failed");
    if (hipMalloc(&st.dev, cap) != hipSuccess) return fail(ctx, CURAST_E_OOM, "descriptor allocation failed");
    st.cap = cap;
    drop_graphs(ctx);   // descriptor buffers moved: captured graphs refer to the old ones
    return CURAST_OK;
}

int ensure_queues(curast_ctx* ctx)
{
    const bool zero = ctx->opt.flags & kFlagZeroQueues;
    const uint32_t q2 = zero ? 1 : ctx->opt.q2_capacity;
    const uint32_t q3 = zero ? 1 : ctx->opt.q3_capacity;
    const uint32_t lg = zero ? 1 : ctx->opt.large_capacity;
    if (q2 > ctx->q2_alloc) {
        if (ctx->q2) hipFree(ctx->q2);
        ctx->q2 = nullptr;
        ctx->q2_alloc = 0;
        if (hipMalloc(&ctx->q2, sizeof(Q2Entry) * (size_t)q2) != hipSuccess) return fail(ctx, CURAST_E_OOM, "Q2 allocation failed");
        ctx->q2_alloc = q2;
        drop_graphs(ctx);
    }
    if (q3 > ctx->q3_alloc) {
        if (ctx->q3) hipFree(ctx->q3);
        ctx->q3 = nullptr;
        ctx->q3_alloc = 0;
        if (ctx->q3_binned) hipFree(ctx->q3_binned);
        ctx->q3_binned = nullptr;
        if (hipMalloc(&ctx->q3, sizeof(Q3Entry) * (size_t)q3) != hipSuccess) return fail(ctx, CURAST_E_OOM, "Q3 allocation failed");
        if (hipMalloc(&ctx->q3_binned, sizeof(uint32_t) * (size_t)q3) != hipSuccess)
            return fail(ctx, CURAST_E_OOM, "Q3 bin allocation failed");
        ctx->q3_alloc = q3;
        drop_graphs(ctx);
    }
    if (lg > ctx->large_alloc) {
        if (ctx->large) hipFree(ctx->large);
        ctx->large = nullptr;
        ctx->large_alloc = 0;
        if (hipMalloc(&ctx->large, sizeof(LargeTri) * (size_t)lg) != hipSuccess) return fail(ctx, CURAST_E_OOM, "large-triangle allocation failed");
        ctx->large_alloc = lg;
        drop_graphs(ctx);
    }
    return CURAST_OK;
}

// Draw matrix: rows x, y, w of VP times the object-to-world matrix X (identity when null), in the
// fixed binary32 operation order of the result definition.
void draw_matrix(const float vp[16], const float* X, float A[12])
{
    static const float I[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    const float* x = X ? X : I;
    static const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r) {
        const float* v = vp + 4 * rows[r];
        for (int c = 0; c < 4; ++c) {
            float t = v[0] * x[c];
            t = t + v[1] * x[4 + c];
            t = t + v[2] * x[8 + c];
            if (c == 3) t = t + v[3];
            A[4 * r + c] = t;
        }
    }
}

// Conservative bounding-sphere test against the view frustum (x = +-w, y = +-w, w = near) in
// double precision with a relative safety margin: true only when every point of the sphere lies
// strictly outside one plane, so no pixel centre can be covered by any triangle inside it.
bool sphere_outside(const float A[12], const float bs[4], float near_plane)
{
    if (!(bs[3] > 0.0f)) return false;
    double rx[4], ry[4], rw[4];
    for (int c = 0; c < 4; ++c) {
        rx[c] = A[c];
        ry[c] = A[4 + c];
        rw[c] = A[8 + c];
    }
    const double cx = bs[0], cy = bs[1], cz = bs[2], r = bs[3];
    auto test = [&](const double* pl) {
        const double v = pl[0] * cx + pl[1] * cy + pl[2] * cz + pl[3];
        const double g = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        const double mag = std::fabs(pl[0] * cx) + std::fabs(pl[1] * cy) + std::fabs(pl[2] * cz) + std::fabs(pl[3]) + r * g;
        return v + r * g + 1e-4 * mag < 0.0;
    };
    double pl[4];
    for (int c = 0; c < 4; ++c) pl[c] = rw[c] + rx[c];
    if (test(pl)) return true;
    for (int c = 0; c < 4; ++c) pl[c] = rw[c] - rx[c];
    if (test(pl)) return true;
    for (int c = 0; c < 4; ++c) pl[c] = rw[c] + ry[c];
    if (test(pl)) return true;
    for (int c = 0; c < 4; ++c) pl[c] = rw[c] - ry[c];
    if (test(pl)) return true;
    for (int c = 0; c < 4; ++c) pl[c] = rw[c] - (c == 3 ? (double)near_plane : 0.0);
    return test(pl);
}

// True when every point of the bounding sphere satisfies w >= near (with slack), w < 1e29 and
// |x|, |y| <= 1.99 w: the fast stage-1 path may then skip its per-vertex range tests.  The slack
// (relative 1e-3 and the 1.99 factor) dwarfs the binary32 error of the kernel's transform.
bool sphere_interior(const float A[12], const float bs[4], float near_plane)
{
    if (!(bs[3] > 0.0f)) return false;
    const double c[4] = {bs[0], bs[1], bs[2], 1.0};
    const double r = bs[3];
    auto range = [&](const double* pl, double& lo, double& hi) {
        double v = 0.0, mag = 0.0;
        for (int k = 0; k < 4; ++k) {
            v += pl[k] * c[k];
            mag += std::fabs(pl[k] * c[k]);
        }
        const double g = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        const double slack = 1e-4 * (mag + r * g);
        lo = v - r * g - slack;
        hi = v + r * g + slack;
    };
    double x[4], y[4], w[4], pl[4], lo, hi;
    for (int k = 0; k < 4; ++k) {
        x[k] = A[k];
        y[k] = A[4 + k];
        w[k] = A[8 + k];
    }
    range(w, lo, hi);
    if (!(lo >= 1.001 * (double)near_plane) || !(hi < 1e29)) return false;
    for (int k = 0; k < 4; ++k) pl[k] = 1.99 * w[k] - x[k];
    range(pl, lo, hi);
    if (!(lo > 0.0)) return false;
    for (int k = 0; k < 4; ++k) pl[k] = 1.99 * w[k] + x[k];
    range(pl, lo, hi);
    if (!(lo > 0.0)) return false;
    for (int k = 0; k < 4; ++k) pl[k] = 1.99 * w[k] - y[k];
    range(pl, lo, hi);
    if (!(lo > 0.0)) return false;
    for (int k = 0; k < 4; ++k) pl[k] = 1.99 * w[k] + y[k];
    range(pl, lo, hi);
    return lo > 0.0;
}

// Prescaled window rows of an interior draw, R = (hW (row x + row w), hH (row y + row w)), rounded
// once from binary64.  Returns false when the error bound of the fast positions they give (see the
// stage-1 kernels: hW u ((7 S_x + 19 S_w) / w + 16) against the exact path, plus 2^-9 px of
// snapping and (3 hW + 1) u of box arithmetic, 1% slack) may exceed the fast margin of 1/32 px
// anywhere in the bounding sphere; S_r bounds sum_j |row_rj| |v_j| + |row_r3| over the sphere and
// w is bounded below by its smallest depth.
bool prescaled_rows(const float A[12], const float bs[4], float hW, float hH, float R[8], float* wnorm, float* slack)
{
    const double u = std::ldexp(1.0, -24);
    const double c[3] = {bs[0], bs[1], bs[2]}, r = bs[3];
    auto S = [&](int row) {
        double s = std::fabs((double)A[4 * row + 3]);
        for (int j = 0; j < 3; ++j) s += std::fabs((double)A[4 * row + j]) * (std::fabs(c[j]) + r);
        return s;
    };
    double w_lo = A[11], g = 0.0, mag = std::fabs((double)A[11]);
    for (int j = 0; j < 3; ++j) {
        w_lo += (double)A[8 + j] * c[j];
        mag += std::fabs((double)A[8 + j] * c[j]);
        g += (double)A[8 + j] * A[8 + j];
    }
    g = std::sqrt(g);
    w_lo -= r * g + 1e-4 * (mag + r * g);
    if (!(w_lo > 0.0)) return false;
    const double sx = S(0), sy = S(1), sw = S(2);
    auto bound = [&](double h, double s_row) {
        return 1.01 * (h * u * ((7.0 * s_row + 19.0 * sw) / w_lo + 16.0) + (3.0 * h + 1.0) * u) + std::ldexp(1.0, -9);
    };
    if (!(bound(hW, sx) <= 1.0 / 32.0) || !(bound(hH, sy) <= 1.0 / 32.0)) return false;
    for (int k = 0; k < 4; ++k) {
        R[k] = (float)((double)hW * ((double)A[k] + (double)A[8 + k]));
        R[4 + k] = (float)((double)hH * ((double)A[4 + k] + (double)A[8 + k]));
    }
    // strip spheres (stage 1, multi-draw launch): |(w row)| rounded up, and the pixels a sphere's
    // projected radius gets on top, which cover the binary32 error of the projected centre
    // (3.01u S_R / w + |x| (3.01u S_w / w + 3u) with S_R <= hW (S_x + S_w) and |x| <= 3 hW), the same
    // error carried into the radius, and two roundings of box arithmetic at |x| <= 3 hW
    *wnorm = std::nextafter((float)std::sqrt((double)A[8] * A[8] + (double)A[9] * A[9] + (double)A[10] * A[10]),
                            INFINITY);
    auto slack_of = [&](double h, double s_row) {
        return 2.0 * h * u * (3.01 * s_row / w_lo + 12.04 * sw / w_lo + 9.0) + 6.0 * h * u;
    };
    *slack = std::nextafter((float)(1.01 * std::max(slack_of(hW, sx), slack_of(hH, sy))), INFINITY);
    return true;
}

int check_view(curast_ctx* ctx, const curast_view& v, bool need_vis = true)
{
    if (v.width < 1 || v.height < 1 || v.width > kMaxDim || v.height > kMaxDim)
        return fail(ctx, CURAST_E_INVALID, "view width/height must lie in [1, 16384]");
    if (!(v.near_plane > 0.0f) || !std::isfinite(v.near_plane) || v.near_plane < 1e-30f)
        return fail(ctx, CURAST_E_INVALID, "near plane must be finite and > 0");
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(v.view_proj[i])) return fail(ctx, CURAST_E_INVALID, "view_proj must be finite");
    if (need_vis && !v.visbuffer) return fail(ctx, CURAST_E_INVALID, "visbuffer is NULL");
    return CURAST_OK;
}

int check_mesh(curast_ctx* ctx, const curast_mesh& m)
{
    if (m.num_triangles > 0xFFFFFFFFull) return fail(ctx, CURAST_E_INVALID, "a mesh may hold at most 2^32-1 triangles");
    if (m.compressed) {
        const curast_compressed& c = *m.compressed;
        if (m.num_triangles && (!c.indices || !c.positions || m.num_vertices == 0))
            return fail(ctx, CURAST_E_INVALID, "compressed mesh with triangles needs packed indices and positions");
        if (c.index_bits < 1 || c.index_bits > 32) return fail(ctx, CURAST_E_INVALID, "index_bits must lie in [1, 32]");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(c.lo[k]) || !std::isfinite(c.step[k]) || c.step[k] < 0.0f)
                return fail(ctx, CURAST_E_INVALID, "compressed lo / step must be finite, step >= 0");
    } else if (m.num_triangles && (!m.vertices || !m.indices || m.num_vertices == 0)) {
        return fail(ctx, CURAST_E_INVALID, "mesh with triangles needs vertices and indices");
    }
    if (m.instances && m.num_instances == 0) return fail(ctx, CURAST_E_INVALID, "instances given with num_instances == 0");
    if (m.instances)
        for (uint64_t i = 0; i < 12ull * m.num_instances; ++i)
            if (!std::isfinite(m.instances[i])) return fail(ctx, CURAST_E_INVALID, "instance matrices must be finite");
    return CURAST_OK;
}

uint32_t n_inst(const curast_mesh& m) { return m.instances ? m.num_instances : 1u; }

// Device descriptor of a mesh's geometry, plain or compressed.
MeshDesc mesh_desc(const curast_mesh& m)
{
    MeshDesc d{};
    d.T = m.num_triangles;
    d.V = m.num_vertices;
    if (m.compressed) {
        const curast_compressed& c = *m.compressed;
        d.idx = c.indices;
        d.qpos = c.positions;
        d.idx_bits = c.index_bits;
        d.idx_min = c.index_min;
        for (int k = 0; k < 3; ++k) {
            d.lo[k] = c.lo[k];
            d.step[k] = c.step[k];
        }
    } else {
        d.pos = m.vertices;
        d.idx = m.indices;
    }
    return d;
}

// Plan storage: heap vectors for the ordinary entry points, fixed arrays for the allocation-free
// one (which takes one mesh, one view and at most kFixedDraws instances).
template <class T>
using HeapVec = std::vector<T>;

constexpr size_t kFixedDraws = 32;

template <class T, size_t N>
struct FixedVec {
    T buf[N];
    size_t n = 0;
    bool overflow = false;
    void push_back(const T& v)
    {
        if (n < N) buf[n++] = v;
        else overflow = true;
    }
    void resize(size_t k)
    {
        overflow |= k > N;
        n = std::min(k, N);
        for (size_t i = 0; i < n; ++i) buf[i] = T{};
    }
    size_t size() const { return n; }
    bool empty() const { return n == 0; }
    T* data() { return buf; }
    const T* data() const { return buf; }
    T& operator[](size_t i) { return buf[i]; }
    const T& operator[](size_t i) const { return buf[i]; }
    T& back() { return buf[n - 1]; }
};

template <class T>
using FixVec = FixedVec<T, kFixedDraws>;

template <template <class> class Vec>
struct PlanT {
    FrameHeader hdr{};
    Vec<ViewDesc> views;
    Vec<MeshDesc> meshes;
    Vec<Segment> segs;
    Vec<DrawDesc> draws;
    Vec<uint32_t> mesh_draw_begin, mesh_draw_count;
    uint64_t tri_draws = 0;
    uint64_t draws_culled = 0;
    uint64_t total_pixels = 0;
    uint64_t max_batches = 0;        // without any culling (graph grid bound)
    uint64_t pair_count = 0;
    bool compressed = false;         // some mesh is compressed
    uint32_t compressed_parts = 0;   // RasterArgs::compressed_parts of this frame's stage-1 parts
    size_t max_draws = 0;            // without any culling
    size_t off_views = 0, off_meshes = 0, off_segs = 0, off_draws = 0, bytes = 0, max_bytes = 0;
    bool full() const;
};
template <>
bool PlanT<HeapVec>::full() const { return false; }
template <>
bool PlanT<FixVec>::full() const
{
    return views.overflow || meshes.overflow || segs.overflow || draws.overflow || mesh_draw_begin.overflow ||
           mesh_draw_count.overflow;
}
using Plan = PlanT<HeapVec>;

template <template <class> class Vec>
int build_plan(curast_ctx* ctx, const curast_options& o, const curast_mesh* meshes, uint32_t M,
               const curast_view* views, uint32_t n_views, PlanT<Vec>& P, uint8_t* visible = nullptr)
{
    if (M && !meshes) return fail(ctx, CURAST_E_INVALID, "meshes is NULL");
    if (!views || n_views == 0) return fail(ctx, CURAST_E_INVALID, "no view");
    for (uint32_t v = 0; v < n_views; ++v) {
        int rc = check_view(ctx, views[v]);
        if (rc) return rc;
        for (uint32_t u = 0; u < v; ++u)
            if (views[u].visbuffer == views[v].visbuffer)
                return fail(ctx, CURAST_E_INVALID, "views must have distinct visibility buffers");
    }
    uint64_t total_ids = 0;
    for (uint32_t m = 0; m < M; ++m) {
        int rc = check_mesh(ctx, meshes[m]);
        if (rc) return rc;
        total_ids += meshes[m].num_triangles * (uint64_t)n_inst(meshes[m]);
        if (total_ids > kMaxIds) return fail(ctx, CURAST_E_ID_RANGE, "more than 2^36 triangle instances");
    }
    const bool cull = !(o.flags & kFlagNoMeshCull);
    const uint32_t bt = o.s1_block * o.s1_tris_per_thread;   // triangles per stage-1 work item
    const uint32_t dpi = o.s1_draws_per_item;
    P.views.resize(n_views);
    for (uint32_t v = 0; v < n_views; ++v) {
        ViewDesc& d = P.views[v];
        d.vis = reinterpret_cast<unsigned long long*>(views[v].visbuffer);
        d.W = views[v].width;
        d.H = views[v].height;
        d.hW = 0.5f * (float)views[v].width;
        d.hH = 0.5f * (float)views[v].height;
        d.near_plane = views[v].near_plane;
        d.wmax = (float)(views[v].width - 1);
        d.hmax = (float)(views[v].height - 1);
        d.pad[0] = d.pad[1] = 0;
        d.tile_base = P.hdr.n_tiles;
        P.hdr.n_tiles += (uint32_t)(((d.W + kTileSize - 1) / kTileSize) * ((d.H + kTileSize - 1) / kTileSize));
        P.total_pixels += (uint64_t)d.W * (uint64_t)d.H;
    }
    P.meshes.resize(M);
    uint64_t base = 0;
    // triangles per work item of the first stage-1 launch (the vertex-sharing kernel runs 64-lane
    // workgroups)
    const uint32_t bt_multi = (o.s1_mode == 3 ? 64u : o.s1_block) * o.s1_multi_tris_per_thread;
    P.mesh_draw_begin.resize(M);
    P.mesh_draw_count.resize(M);
    if (P.full()) return fail(ctx, CURAST_E_INVALID, "too many meshes or views for the allocation-free form");
    auto& mesh_draw_begin = P.mesh_draw_begin;
    auto& mesh_draw_count = P.mesh_draw_count;
    for (uint32_t m = 0; m < M; ++m) {
        const curast_mesh& me = meshes[m];
        P.meshes[m] = mesh_desc(me);
        P.compressed |= me.compressed != nullptr;
        const uint32_t ni = n_inst(me);
        const uint32_t draw_begin = (uint32_t)P.draws.size();
        for (uint32_t i = 0; i < ni; ++i, base += me.num_triangles) {
            if (me.num_triangles == 0) {
                if (visible)
                    for (uint32_t v = 0; v < n_views; ++v) visible[(P.pair_count + i) * (uint64_t)n_views + v] = 0;
                continue;
            }
            for (uint32_t v = 0; v < n_views; ++v) {
                DrawDesc D;
                draw_matrix(views[v].view_proj, me.instances ? me.instances + 12ull * i : nullptr, D.A);
                const bool out = cull && sphere_outside(D.A, me.bsphere, views[v].near_plane);
                for (int k = 0; k < 8; ++k) D.R[k] = 0.0f;
                D.wnorm = D.slack = 0.0f;
                D.wmax = (float)(views[v].width - 1);
                D.hmax = (float)(views[v].height - 1);
                const bool inner = !out && !(o.flags & kFlagNoFastInterior) &&
                                   sphere_interior(D.A, me.bsphere, views[v].near_plane) &&
                                   prescaled_rows(D.A, me.bsphere, 0.5f * (float)views[v].width,
                                                  0.5f * (float)views[v].height, D.R, &D.wnorm, &D.slack);
                if (visible) visible[(P.pair_count + i) * (uint64_t)n_views + v] = out ? 0 : inner ? 2 : 1;
                if (out) {
                    P.draws_culled++;
                    continue;
                }
                D.id_base = base;
                D.view = v | (inner ? kDrawInterior : 0u);
                D.mesh = m;
                P.draws.push_back(D);
            }
        }
        P.pair_count += ni;
        mesh_draw_begin[m] = draw_begin;
        mesh_draw_count[m] = (uint32_t)P.draws.size() - draw_begin;
        if (me.num_triangles) {
            const uint64_t all = (uint64_t)ni * n_views;
            const uint64_t groups = (all + dpi - 1) / dpi;
            P.max_draws += all;
            P.max_batches += ((me.num_triangles + std::min(bt, bt_multi) - 1) / std::min(bt, bt_multi)) * groups;
        }
    }
    if (P.full()) return fail(ctx, CURAST_E_INVALID, "the allocation-free form takes at most 32 instances");
    // stage-1 segments: meshes drawn more than once first (their own launch, whose lanes reuse each
    // loaded triangle over many draws), then the rest; mode 3 sends every mesh to the first
    auto shared_mesh = [&](uint32_t m) { return o.s1_mode == 3 || mesh_draw_count[m] >= 2; };
    for (int pass = 0; pass < 2; ++pass) {
        bool any_cmp = false, all_cmp = true;
        for (uint32_t m = 0; m < M; ++m) {
            const uint32_t dc = mesh_draw_count[m];
            if (!dc || !meshes[m].num_triangles || shared_mesh(m) != (pass == 0)) continue;
            any_cmp |= meshes[m].compressed != nullptr;
            // the all-compressed kernels use 32-bit offsets into the quantized positions
            all_cmp &= meshes[m].compressed != nullptr && meshes[m].num_vertices <= (1u << 29);
            Segment sg{};
            sg.batch_begin = P.hdr.total_batches;
            sg.mesh = m;
            sg.draw_begin = mesh_draw_begin[m];
            sg.draw_count = dc;
            sg.n_groups = (dc + dpi - 1) / dpi;
            sg.batch_tris = pass == 0 ? bt_multi : bt;
            P.segs.push_back(sg);
            P.hdr.total_batches += ((meshes[m].num_triangles + sg.batch_tris - 1) / sg.batch_tris) * sg.n_groups;
            P.tri_draws += meshes[m].num_triangles * (uint64_t)dc;
        }
        if (pass == 0) P.hdr.shared_batches = P.hdr.total_batches;
        const uint32_t part = pass + 1;
        if (any_cmp) P.compressed_parts |= (1u << part) | (all_cmp ? 1u << (part + 8) : 0u);
    }
    if (P.full()) return fail(ctx, CURAST_E_INVALID, "the allocation-free form takes one mesh and one view");
    P.hdr.n_segs = (uint32_t)P.segs.size();
    P.hdr.n_views = n_views;
    P.hdr.batch_tris = bt;
    P.hdr.draws_per_item = dpi;
    P.off_views = align_up(sizeof(FrameHeader), 256);
    P.off_meshes = align_up(P.off_views + sizeof(ViewDesc) * n_views, 256);
    P.off_segs = align_up(P.off_meshes + sizeof(MeshDesc) * std::max<uint32_t>(M, 1), 256);
    P.off_draws = align_up(P.off_segs + sizeof(Segment) * std::max<uint32_t>(M, 1), 256);
    P.bytes = align_up(P.off_draws + sizeof(DrawDesc) * std::max<size_t>(P.draws.size(), 1), 256);
    P.max_bytes = align_up(P.off_draws + sizeof(DrawDesc) * std::max<size_t>(P.max_draws, 1), 256);
    return CURAST_OK;
}

void write_plan(const Plan& P, void* host)
{
    char* h = static_cast<char*>(host);
    std::memcpy(h, &P.hdr, sizeof(FrameHeader));
    std::memcpy(h + P.off_views, P.views.data(), sizeof(ViewDesc) * P.views.size());
    if (!P.meshes.empty()) std::memcpy(h + P.off_meshes, P.meshes.data(), sizeof(MeshDesc) * P.meshes.size());
    if (!P.segs.empty()) std::memcpy(h + P.off_segs, P.segs.data(), sizeof(Segment) * P.segs.size());
    if (!P.draws.empty()) std::memcpy(h + P.off_draws, P.draws.data(), sizeof(DrawDesc) * P.draws.size());
}

RasterArgs make_args(curast_ctx* ctx, const Plan& P)
{
    char* d = static_cast<char*>(ctx->raster_stage.dev);
    RasterArgs a;
    a.hdr = reinterpret_cast<const FrameHeader*>(d);
    a.views = reinterpret_cast<const ViewDesc*>(d + P.off_views);
    a.meshes = reinterpret_cast<const MeshDesc*>(d + P.off_meshes);
    a.segs = reinterpret_cast<const Segment*>(d + P.off_segs);
    a.draws = reinterpret_cast<const DrawDesc*>(d + P.off_draws);
    a.q2 = ctx->q2;
    a.large = ctx->large;
    a.q3 = ctx->q3;
    a.counters = ctx->counters;
    a.stats = ctx->stats;
    const bool zero = ctx->opt.flags & kFlagZeroQueues;
    a.q2_cap = zero ? 0 : ctx->opt.q2_capacity;
    a.large_cap = zero ? 0 : ctx->opt.large_capacity;
    a.q3_cap = zero ? 0 : ctx->opt.q3_capacity;
    a.small_px = ctx->opt.small_px;
    a.medium_px = ctx->opt.medium_px;
    a.flags = ctx->opt.flags;
    a.s1_mode = ctx->opt.s1_mode;
    a.part = 0;
    a.tile_count = ctx->tile_count;
    a.tile_offset = ctx->tile_offset;
    a.q3_binned = ctx->q3_binned;
    a.compressed_parts = P.compressed_parts;
    return a;
}

TimedFrame* begin_timing(curast_ctx* ctx)
{
    if (!(ctx->opt.flags & CURAST_FLAG_TIMING)) return nullptr;
    // events come from the context's pool, which grows 32 frames' worth at a time and gets every
    // event back when the frames are collected (curast_get_stage_times / curast_reset_stage_times),
    // so a timed frame in steady state costs event records on the stream, not event creation
    if (ctx->event_pool.size() < kNumSlots + 1)
        for (int i = 0; i < 32 * (kNumSlots + 1); ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) break;
            ctx->event_pool.push_back(e);
        }
    if (ctx->event_pool.size() < kNumSlots + 1) return nullptr;
    TimedFrame f;
    for (int i = 0; i <= kNumSlots; ++i) {
        f.ev[i] = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    }
    for (int i = 0; i < kNumSlots; ++i) f.used[i] = 0;
    ctx->timed.push_back(f);
    return &ctx->timed.back();
}

// Launch the device part of a frame over the buffers in `a` (descriptors, queues, counters):
// clear, stage 1, overflow pass, stage 2, stage 3.  Options other than a.flags come from ctx.
int launch_frame(curast_ctx* ctx, const RasterArgs& a, uint64_t total_pixels, uint32_t grid1, uint32_t grid_share,
                 hipStream_t s, TimedFrame* tf)
{
    const bool stats = a.flags & kFlagStats;
    const uint32_t cus = (uint32_t)ctx->cus;
    const uint64_t pairs = (total_pixels + 1) / 2;
    const uint32_t clear_grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((pairs + 255) / 256, cus * 16ull));
    hipError_t e;
    if (tf) hipEventRecord(tf->ev[0], s);
    e = launch_clear(a, clear_grid, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "clear kernel launch");
    if (tf) hipEventRecord(tf->ev[1], s);
    {
        // work items [0, shared_batches) are the multi-draw meshes' (part 1), the rest part 2; each
        // launch's kernel processes s1_block x (its tris-per-thread) triangles per work item,
        // matching the batch size the plan gave those segments
        // each launch has at most s1_blocks_per_cu workgroups per CU, which loop over the work
        // items: a workgroup's set-up is then shared by several items, and the dispatcher
        // launches fewer workgroups (one per item measured slower on the HBM-bound launch)
        const uint32_t mode = ctx->opt.s1_mode, blk = ctx->opt.s1_block;
        const uint32_t grid_cap = (uint32_t)std::min<uint64_t>((uint64_t)cus * ctx->opt.s1_blocks_per_cu, 1ull << 24);
        auto launch_part = [&](uint32_t part, uint32_t tpt, uint32_t grid, hipStream_t st) {
            grid = std::min(grid, grid_cap);
            RasterArgs a1 = a;
            a1.part = part;
            // the multi-draw launch writes with the atomic alone: its fragments come from small
            // instanced triangles, and a read before each atomic cost a memory round trip per
            // fragment there; the single-draw launch, bound by memory, gains from skipping atomics
            if (part == 1 && !(a.flags & kFlagEarlyOutAll)) a1.flags |= kFlagNoEarlyOut;
            if (part == 1 && mode == 3) return launch_stage1_share(a1, tpt, stats, grid, st);
            if (mode == 1) return launch_stage1(a1, blk, tpt, stats, grid, st);
            const bool strips = !(a.flags & kFlagNoStrips) && tpt >= 2 &&
                                (part == 1 || (a.flags & kFlagSingleStrips));
            // strip spheres in the multi-draw launch, s1_mode 0 and 2 (s1_mode 4: union boxes only)
            const bool spheres = strips && part == 1 && mode != 4;
            return launch_stage1_fast(a1, blk, tpt, strips, spheres, stats, grid, st);
        };
        if (grid_share && (a.flags & kFlagS1Overlap)) {
            // the single-draw launch (bound by memory) on the side stream next to the multi-draw one
            // (bound by the vector ALUs), so that the two share the compute units; both only append
            // to the queues and take atomic minima, so the result does not depend on their order
            e = hipEventRecord(ctx->fork_ev, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side_stream, ctx->fork_ev, 0);
            if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 stream fork");
            e = launch_part(2, ctx->opt.s1_tris_per_thread, std::max<uint32_t>(grid1, 1), ctx->side_stream);
            if (e == hipSuccess) e = hipEventRecord(ctx->join_ev, ctx->side_stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 kernel launch");
            e = launch_part(1, ctx->opt.s1_multi_tris_per_thread, grid_share, s);
            if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 kernel launch (multi-draw meshes)");
            if (tf) hipEventRecord(tf->ev[2], s);
            e = hipStreamWaitEvent(s, ctx->join_ev, 0);
            if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 stream join");
        } else {
            if (grid_share) {
                e = launch_part(1, ctx->opt.s1_multi_tris_per_thread, grid_share, s);
                if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 kernel launch (multi-draw meshes)");
            }
            if (tf) hipEventRecord(tf->ev[2], s);
            e = launch_part(2, ctx->opt.s1_tris_per_thread, std::max<uint32_t>(grid1, 1), s);
            if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 kernel launch");
        }
    }
    if (tf) hipEventRecord(tf->ev[3], s);
    e = launch_stage1_overflow(a, cus * 4, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "stage-1 overflow kernel launch");
    if (tf) hipEventRecord(tf->ev[4], s);
    {
        // stage 2 writes with the atomic alone as well (see the stage-1 launches)
        RasterArgs a2 = a;
        if (!(a.flags & kFlagEarlyOutAll)) a2.flags |= kFlagNoEarlyOut;
        e = launch_stage2(a2, std::max<uint32_t>(1, ctx->opt.s2_waves / 4), stats, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "stage-2 kernel launch");
    if (tf) hipEventRecord(tf->ev[5], s);
    e = (a.flags & kFlagS3PerPart) ? launch_stage3(a, std::max<uint32_t>(1, ctx->opt.s3_blocks), stats, s)
                                          : launch_stage3_binned(a, std::max<uint32_t>(1, ctx->opt.s3_blocks), stats, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "stage-3 kernel launch");
    if (tf) {
        hipEventRecord(tf->ev[6], s);
        for (int i = kTClear; i <= kTS3; ++i) tf->used[i] = 1;
    }
    return CURAST_OK;
}

uint32_t grid_for(uint64_t batches) { return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(batches, 1), 1ull << 24); }

int rasterize_impl(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* views, uint32_t n_views,
                   hipStream_t s, bool use_graph)
{
    if (!ctx) return CURAST_E_INVALID;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Plan P;
    int rc = build_plan(ctx, ctx->opt, meshes, M, views, n_views, P);
    if (rc) return rc;
    rc = ensure_queues(ctx);
    if (rc) return rc;
    rc = ensure_tiles(ctx, P.hdr.n_tiles);
    if (rc) return rc;
    const size_t bytes = use_graph ? P.max_bytes : P.bytes;
    rc = ensure_staging(ctx, ctx->raster_stage, bytes);
    if (rc) return rc;
    write_plan(P, ctx->raster_stage.host);
    ctx->draws_culled += P.draws_culled;
    log_plan(use_graph ? "batched frame" : "frame", P, M, n_views);
    TimedFrame* tf = begin_timing(ctx);
    if (!use_graph) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->raster_stage.dev, ctx->raster_stage.host, P.bytes, hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipEventRecord(ctx->raster_stage.ev, s));
        ctx->raster_stage.pending = true;
        const uint64_t shared = P.hdr.shared_batches;
        rc = launch_frame(ctx, make_args(ctx, P), P.total_pixels, grid_for(P.hdr.total_batches - shared),
                          shared ? grid_for(shared) : 0, s, tf);
        return rc;
    }
    // graph path: one captured sequence per structure (sizes of the descriptor block, grid bound,
    // options); replays copy the new descriptor contents from the same pinned buffer
    const uint32_t grid1 = grid_for(P.max_batches);
    // the queue capacities are kernel arguments of the captured launches, so they are part of the key
    uint64_t key[11] = {(uint64_t)M, (uint64_t)n_views, (uint64_t)P.max_bytes, (uint64_t)grid1,
                       ((uint64_t)ctx->opt.s1_block << 32) | (ctx->opt.s1_tris_per_thread << 8) |
                           (ctx->opt.s1_multi_tris_per_thread << 4) | ctx->opt.s1_mode,
                       ((uint64_t)ctx->opt.s2_waves << 32) | ctx->opt.s3_blocks,
                       ((uint64_t)ctx->opt.flags << 32) | ctx->opt.small_px,
                       ((uint64_t)ctx->opt.medium_px << 32) | ctx->opt.s1_draws_per_item,
                       ((uint64_t)P.compressed << 32) | P.compressed_parts,
                       ((uint64_t)ctx->opt.large_capacity << 32) | ctx->opt.s1_blocks_per_cu,
                       ((uint64_t)ctx->opt.q2_capacity << 32) | ctx->opt.q3_capacity};
    GraphEntry* ge = nullptr;
    for (auto& g : ctx->graphs)
        if (std::memcmp(g.key, key, sizeof key) == 0) ge = &g;
    if (!ge) {
        GraphEntry g;
        std::memcpy(g.key, key, sizeof key);
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipMemcpyAsync(ctx->raster_stage.dev, ctx->raster_stage.host, P.max_bytes, hipMemcpyHostToDevice,
                                      ctx->capture_stream);
        int lrc = e == hipSuccess ? launch_frame(ctx, make_args(ctx, P), P.total_pixels, grid1, grid1,
                                                 ctx->capture_stream, nullptr)
                                  : hip_fail(ctx, e, "capture memcpy");
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &graph);
        if (lrc) {
            if (graph) hipGraphDestroy(graph);
            return lrc;
        }
        if (e2 != hipSuccess) return hip_fail(ctx, e2, "hipStreamEndCapture");
        g.graph = graph;
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(graph);
            return hip_fail(ctx, e, "hipGraphInstantiate");
        }
        ctx->graphs.push_back(g);
        log_line("captured a frame graph (%zu held by the context)", ctx->graphs.size());
        ge = &ctx->graphs.back();
    }
    if (tf) HIP_TRY(ctx, hipEventRecord(tf->ev[0], s));
    HIP_TRY(ctx, hipGraphLaunch(ge->exec, s));
    HIP_TRY(ctx, hipEventRecord(ctx->raster_stage.ev, s));
    ctx->raster_stage.pending = true;
    if (tf) {
        HIP_TRY(ctx, hipEventRecord(tf->ev[kNumSlots], s));
        tf->used[kTFrame] = 1;
    }
    return CURAST_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// Allocation-free rasterization (curast_rasterize_noalloc)
// ------------------------------------------------------------------------------------------------
// One mesh (at most kFixedDraws instances) into one view with no allocation of any kind: the plan
// is built in fixed arrays on the stack, its descriptors reach the device as the argument of one
// small kernel, and descriptors, queues, counters and stage-3 bins live in the file-scope device
// array `scratch` below instead of context buffers.  Host code must not use the array's name as an
// address (it is a host-side handle): curast_create takes the device address with
// hipGetSymbolAddress once per device and every use goes through that pointer.  Queues smaller
// than the context's are safe: overflow falls back to in-place rasterization.
namespace {

constexpr uint32_t kNaQ2 = 1u << 20;       // stage-2 queue entries (8 MB)
constexpr uint32_t kNaLarge = 1u << 16;    // large-triangle records (3 MB)
constexpr uint32_t kNaQ3 = 1u << 19;       // stage-3 tile parts (4 MB + 2 MB of bins)
constexpr uint32_t kNaTiles = (uint32_t)(kMaxDim / kTileSize) * (uint32_t)(kMaxDim / kTileSize) + 1;

struct NaDesc {
    FrameHeader hdr;
    ViewDesc view;
    MeshDesc mesh;
    Segment segs[2];
    DrawDesc draws[kFixedDraws];
};
static_assert(sizeof(NaDesc) % 4 == 0 && sizeof(NaDesc) <= 4096, "descriptor block fits one kernel argument");

constexpr size_t kNaOffCounters = align_up(sizeof(NaDesc), 256);
constexpr size_t kNaOffStats = kNaOffCounters + 256;
constexpr size_t kNaOffTileCount = kNaOffStats + 256;
constexpr size_t kNaOffTileOffset = align_up(kNaOffTileCount + sizeof(uint32_t) * kNaTiles, 256);
constexpr size_t kNaOffQ2 = align_up(kNaOffTileOffset + sizeof(uint32_t) * kNaTiles, 256);
constexpr size_t kNaOffLarge = align_up(kNaOffQ2 + sizeof(Q2Entry) * kNaQ2, 256);
constexpr size_t kNaOffQ3 = align_up(kNaOffLarge + sizeof(LargeTri) * kNaLarge, 256);
constexpr size_t kNaOffBinned = align_up(kNaOffQ3 + sizeof(Q3Entry) * kNaQ3, 256);
constexpr size_t kNaBytes = align_up(kNaOffBinned + sizeof(uint32_t) * kNaQ3, 256);
static_assert(kNumCounters * sizeof(unsigned long long) <= 256 && kNumStats * sizeof(unsigned long long) <= 256,
              "counter areas");

}  // namespace

// The allocation-free form's scratch (about 17 MB per device, held until the process ends).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Copies the frame's descriptor block from the kernel argument into the scratch array.
__global__ void __launch_bounds__(256) noalloc_descriptor_kernel(NaDesc d, NaDesc* out)
{
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&d);
    uint32_t* dst = reinterpret_cast<uint32_t*>(out);
    for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(NaDesc) / 4); i += blockDim.x) dst[i] = src[i];
}

namespace {

// Device address of `scratch` on the current device, looked up once per device and kept.
std::mutex g_scratch_mutex;
constexpr int kMaxDevices = 64;
char* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int device, char** out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

int rasterize_noalloc(curast_ctx* ctx, const curast_mesh& mesh, const curast_view& view, hipStream_t s)
{
    if (!ctx->na_scratch) return fail(ctx, CURAST_E_HIP, "scratch address of the allocation-free form is unknown");
    if (mesh.instances && mesh.num_instances > kFixedDraws)
        return fail(ctx, CURAST_E_INVALID, "the allocation-free form takes at most 32 instances");
    PlanT<FixVec> P;
    int rc = build_plan(ctx, ctx->opt, &mesh, 1, &view, 1, P);
    if (rc) return rc;
    NaDesc d;
    std::memset(&d, 0, sizeof d);
    d.hdr = P.hdr;
    d.view = P.views[0];
    d.mesh = P.meshes[0];
    for (size_t i = 0; i < P.segs.size() && i < 2; ++i) d.segs[i] = P.segs[i];
    for (size_t i = 0; i < P.draws.size(); ++i) d.draws[i] = P.draws[i];
    char* base = ctx->na_scratch;
    NaDesc* dd = reinterpret_cast<NaDesc*>(base);
    RasterArgs a;
    std::memset(&a, 0, sizeof a);
    a.hdr = &dd->hdr;
    a.views = &dd->view;
    a.meshes = &dd->mesh;
    a.segs = dd->segs;
    a.draws = dd->draws;
    a.counters = reinterpret_cast<unsigned long long*>(base + kNaOffCounters);
    a.stats = reinterpret_cast<unsigned long long*>(base + kNaOffStats);
    a.tile_count = reinterpret_cast<uint32_t*>(base + kNaOffTileCount);
    a.tile_offset = reinterpret_cast<uint32_t*>(base + kNaOffTileOffset);
    a.q2 = reinterpret_cast<Q2Entry*>(base + kNaOffQ2);
    a.large = reinterpret_cast<LargeTri*>(base + kNaOffLarge);
    a.q3 = reinterpret_cast<Q3Entry*>(base + kNaOffQ3);
    a.q3_binned = reinterpret_cast<uint32_t*>(base + kNaOffBinned);
    const bool zero = ctx->opt.flags & kFlagZeroQueues;
    a.q2_cap = zero ? 0 : std::min(ctx->opt.q2_capacity, kNaQ2);
    a.large_cap = zero ? 0 : std::min(ctx->opt.large_capacity, kNaLarge);
    a.q3_cap = zero ? 0 : std::min(ctx->opt.q3_capacity, kNaQ3);
    a.small_px = ctx->opt.small_px;
    a.medium_px = ctx->opt.medium_px;
    a.flags = ctx->opt.flags & ~(uint32_t)(kFlagStats | CURAST_FLAG_TIMING);   // no statistics, no events
    a.s1_mode = ctx->opt.s1_mode;
    a.part = 0;
    a.compressed_parts = P.compressed_parts;
    noalloc_descriptor_kernel<<<1, 256, 0, s>>>(d, dd);
    HIP_TRY(ctx, hipGetLastError());
    const uint64_t shared = P.hdr.shared_batches;
    return launch_frame(ctx, a, P.total_pixels, grid_for(P.hdr.total_batches - shared), shared ? grid_for(shared) : 0,
                        s, nullptr);
}

void collect_timings(curast_ctx* ctx)
{
    // raster frames: ev[0..6] bracket clear, stage-1 sharing, stage-1 plain, overflow pass, stage 2,
    // stage 3; resolve calls: ev[7] .. ev[8]; graph frames: ev[0] .. ev[kNumSlots]
    for (auto& f : ctx->timed) {
        float ms = 0.0f;
        if (f.used[kTClear]) {
            hipEventSynchronize(f.ev[6]);
            for (int i = kTClear; i <= kTS3; ++i)
                if (hipEventElapsedTime(&ms, f.ev[i], f.ev[i + 1]) == hipSuccess) ctx->stage_ms[i] += ms;
            if (hipEventElapsedTime(&ms, f.ev[0], f.ev[6]) == hipSuccess) ctx->stage_ms[kTFrame] += ms;
        } else if (f.used[kTFrame]) {
            hipEventSynchronize(f.ev[kNumSlots]);
            if (hipEventElapsedTime(&ms, f.ev[0], f.ev[kNumSlots]) == hipSuccess) ctx->stage_ms[kTFrame] += ms;
        }
        if (f.used[kTResolve] || f.used[kTResolveBwd]) {
            hipEventSynchronize(f.ev[8]);
            const int slot = f.used[kTResolve] ? kTResolve : kTResolveBwd;
            if (hipEventElapsedTime(&ms, f.ev[7], f.ev[8]) == hipSuccess) ctx->stage_ms[slot] += ms;
        }
        if (f.used[kTClear] || f.used[kTFrame]) ctx->timed_frames++;
        for (int i = 0; i <= kNumSlots; ++i) ctx->event_pool.push_back(f.ev[i]);
    }
    ctx->timed.clear();
}

int build_resolve_desc(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view& view,
                       const float* const* attrs, const curast_texture* textures, ResolveArgs& a, size_t& bytes_out,
                       float* const* grad_attrs = nullptr, float* const* grad_pos = nullptr)
{
    uint64_t np = 0;
    for (uint32_t m = 0; m < M; ++m) np += n_inst(meshes[m]);
    if (np > 0xFFFFFFF0ull) return fail(ctx, CURAST_E_INVALID, "too many (mesh, instance) pairs");
    const size_t off_bases = 0;
    const size_t off_mpair = align_up(sizeof(uint64_t) * ((size_t)M + 1), 256);
    const size_t off_pairs = align_up(off_mpair + sizeof(uint32_t) * std::max<uint32_t>(M, 1), 256);
    const size_t off_meshes = align_up(off_pairs + sizeof(DrawDesc) * std::max<uint64_t>(np, 1), 256);
    const size_t off_attrs = align_up(off_meshes + sizeof(MeshDesc) * std::max<uint32_t>(M, 1), 256);
    const size_t off_tex = align_up(off_attrs + sizeof(float*) * std::max<uint32_t>(M, 1), 256);
    const size_t off_grad = textures ? align_up(off_tex + sizeof(TexDesc) * std::max<uint32_t>(M, 1), 256) : off_tex;
    const size_t bytes = grad_attrs ? align_up(off_grad + 2 * sizeof(float*) * std::max<uint32_t>(M, 1), 256) : off_grad;
    int rc = ensure_staging(ctx, ctx->resolve_stage, bytes);
    if (rc) return rc;
    char* h = static_cast<char*>(ctx->resolve_stage.host);
    uint64_t* bases = reinterpret_cast<uint64_t*>(h + off_bases);
    uint32_t* mpair = reinterpret_cast<uint32_t*>(h + off_mpair);
    DrawDesc* pairs = reinterpret_cast<DrawDesc*>(h + off_pairs);
    MeshDesc* md = reinterpret_cast<MeshDesc*>(h + off_meshes);
    const float** ap = reinterpret_cast<const float**>(h + off_attrs);
    TexDesc* td = reinterpret_cast<TexDesc*>(h + off_tex);
    float** gap = reinterpret_cast<float**>(h + off_grad);
    float** gpp = gap + std::max<uint32_t>(M, 1);
    uint64_t base = 0, p = 0;
    for (uint32_t m = 0; m < M; ++m) {
        md[m] = mesh_desc(meshes[m]);
        ap[m] = attrs[m];
        if (grad_attrs) {
            gap[m] = grad_attrs[m];
            gpp[m] = grad_pos ? grad_pos[m] : nullptr;
        }
        bases[m] = base;
        mpair[m] = (uint32_t)p;
        if (textures) {
            TexDesc t{};
            t.texels = textures[m].texels;
            t.w = textures[m].width;
            t.h = textures[m].height;
            t.levels = textures[m].levels;
            uint32_t off = 0;
            for (uint32_t l = 0; l < t.levels; ++l) {
                t.off[l] = off;
                off += std::max(1u, t.w >> l) * std::max(1u, t.h >> l);
            }
            td[m] = t;
        }
        for (uint32_t i = 0; i < n_inst(meshes[m]); ++i, ++p) {
            draw_matrix(view.view_proj, meshes[m].instances ? meshes[m].instances + 12ull * i : nullptr, pairs[p].A);
            pairs[p].id_base = base;
            pairs[p].view = 0;
            pairs[p].mesh = m;
            base += meshes[m].num_triangles;
        }
    }
    bases[M] = base;
    char* d = static_cast<char*>(ctx->resolve_stage.dev);
    a.vis = reinterpret_cast<const unsigned long long*>(view.visbuffer);
    a.W = view.width;
    a.H = view.height;
    a.hW = 0.5f * (float)view.width;
    a.hH = 0.5f * (float)view.height;
    a.bases = reinterpret_cast<const uint64_t*>(d + off_bases);
    a.mesh_pair = reinterpret_cast<const uint32_t*>(d + off_mpair);
    a.pairs = reinterpret_cast<const DrawDesc*>(d + off_pairs);
    a.meshes = reinterpret_cast<const MeshDesc*>(d + off_meshes);
    a.attrs = reinterpret_cast<const float* const*>(d + off_attrs);
    a.tex = textures ? reinterpret_cast<const TexDesc*>(d + off_tex) : nullptr;
    a.grad_attrs = grad_attrs ? reinterpret_cast<float* const*>(d + off_grad) : nullptr;
    a.grad_pos = grad_attrs && grad_pos ? reinterpret_cast<float* const*>(d + off_grad) + std::max<uint32_t>(M, 1) : nullptr;
    a.n_pairs = (uint32_t)np;
    a.n_meshes = M;
    bytes_out = bytes;
    return CURAST_OK;
}

int check_screen(curast_ctx* ctx, const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                 const float* pos_ss, uint32_t V, const float* attrs, uint32_t C)
{
    if (!vis || !pos_ss || !attrs || (T && !idx)) return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    if (W < 1 || H < 1 || W > kMaxDim || H > kMaxDim) return fail(ctx, CURAST_E_INVALID, "width/height must lie in [1, 16384]");
    if (C < 1 || C > 16) return fail(ctx, CURAST_E_INVALID, "C must lie in [1, 16]");
    if (V == 0) return fail(ctx, CURAST_E_INVALID, "num_vertices must be > 0");
    return CURAST_OK;
}

}  // namespace

// ================================================================================================
// C ABI
// ================================================================================================
extern "C" {

int curast_version(void) { return 10000; }

const char* curast_status_string(int status)
{
    switch (status) {
    case CURAST_OK: return "ok";
    case CURAST_E_INVALID: return "invalid argument";
    case CURAST_E_ID_RANGE: return "triangle IDs exceed 36 bits";
    case CURAST_E_OOM: return "out of memory";
    case CURAST_E_HIP: return "HIP runtime error";
    case CURAST_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* curast_last_error(const curast_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int curast_create(const curast_options* opt, curast_ctx** out)
{
    if (!out) return CURAST_E_INVALID;
    *out = nullptr;
    curast_options u{};
    if (opt) u = *opt;
    std::string msg;
    if (validate_options(u, msg)) return CURAST_E_INVALID;
    curast_ctx* ctx = new (std::nothrow) curast_ctx();
    if (!ctx) return CURAST_E_OOM;
    auto cleanup = [&](int rc) {
        curast_destroy(ctx);
        return rc;
    };
    if (hipGetDevice(&ctx->device) != hipSuccess) return cleanup(CURAST_E_HIP);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return cleanup(CURAST_E_HIP);
    ctx->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    ctx->user = u;
    ctx->opt = resolve_defaults(u, ctx->cus);
    if (hipMalloc(&ctx->counters, sizeof(unsigned long long) * kNumCounters) != hipSuccess) return cleanup(CURAST_E_OOM);
    if (hipMalloc(&ctx->stats, sizeof(unsigned long long) * kNumStats) != hipSuccess) return cleanup(CURAST_E_OOM);
    if (hipMemset(ctx->counters, 0, sizeof(unsigned long long) * kNumCounters) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipMemset(ctx->stats, 0, sizeof(unsigned long long) * kNumStats) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipEventCreateWithFlags(&ctx->raster_stage.ev, hipEventDisableTiming) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (hipEventCreateWithFlags(&ctx->resolve_stage.ev, hipEventDisableTiming) != hipSuccess) return cleanup(CURAST_E_HIP);
    if (ensure_queues(ctx)) return cleanup(CURAST_E_OOM);
    // device address of the allocation-free form's scratch array (looked up once per device)
    const hipError_t se = scratch_address(ctx->device, &ctx->na_scratch);
    if (se != hipSuccess) {
        fprintf(stderr, "curast_create: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(se));
        return cleanup(CURAST_E_HIP);
    }
    log_line("context on device %d (%d CUs): s1_mode %u, s1_block %u, tris/lane %u/%u (single/multi), draws/item %u, "
             "small_px %u, medium_px %u, queues %u/%u/%u, flags 0x%x",
             ctx->device, ctx->cus, ctx->opt.s1_mode, ctx->opt.s1_block, ctx->opt.s1_tris_per_thread,
             ctx->opt.s1_multi_tris_per_thread, ctx->opt.s1_draws_per_item, ctx->opt.small_px, ctx->opt.medium_px,
             ctx->opt.q2_capacity, ctx->opt.large_capacity, ctx->opt.q3_capacity, ctx->opt.flags);
    *out = ctx;
    return CURAST_OK;
}

int curast_destroy(curast_ctx* ctx)
{
    if (!ctx) return CURAST_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    collect_timings(ctx);
    drop_graphs(ctx);
    for (Staging* st : {&ctx->raster_stage, &ctx->resolve_stage}) {
        if (st->host) hipHostFree(st->host);
        if (st->dev) hipFree(st->dev);
        if (st->ev) hipEventDestroy(st->ev);
    }
    for (hipEvent_t ev : ctx->event_pool) hipEventDestroy(ev);
    if (ctx->q2) hipFree(ctx->q2);
    if (ctx->q3) hipFree(ctx->q3);
    if (ctx->q3_binned) hipFree(ctx->q3_binned);
    if (ctx->tile_count) hipFree(ctx->tile_count);
    if (ctx->tile_offset) hipFree(ctx->tile_offset);
    if (ctx->large) hipFree(ctx->large);
    if (ctx->counters) hipFree(ctx->counters);
    if (ctx->stats) hipFree(ctx->stats);
    if (ctx->ranges) hipFree(ctx->ranges);
    if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
    if (ctx->side_stream) hipStreamDestroy(ctx->side_stream);
    if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) hipEventDestroy(ctx->join_ev);
    delete ctx;
    return CURAST_OK;
}

int curast_set_options(curast_ctx* ctx, const curast_options* opt)
{
    if (!ctx || !opt) return CURAST_E_INVALID;
    std::string msg;
    if (validate_options(*opt, msg)) return fail(ctx, CURAST_E_INVALID, msg);
    ctx->user = *opt;
    ctx->opt = resolve_defaults(*opt, ctx->cus);
    return ensure_queues(ctx);
}

int curast_get_options(const curast_ctx* ctx, curast_options* opt)
{
    if (!ctx || !opt) return CURAST_E_INVALID;
    *opt = ctx->opt;
    return CURAST_OK;
}

int curast_rasterize_meshes(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view, void* stream)
{
    if (!ctx || !view) return ctx ? fail(ctx, CURAST_E_INVALID, "view is NULL") : CURAST_E_INVALID;
    return rasterize_impl(ctx, meshes, M, view, 1, static_cast<hipStream_t>(stream), false);
}

int curast_rasterize(curast_ctx* ctx, const float* vertices, uint32_t num_vertices, const uint32_t* indices,
                     uint64_t num_triangles, const float* instances, uint32_t num_instances, const float view_proj[16],
                     float near_plane, int32_t width, int32_t height, uint64_t* visbuffer, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!view_proj) return fail(ctx, CURAST_E_INVALID, "view_proj is NULL");
    curast_mesh m{};
    m.vertices = vertices;
    m.num_vertices = num_vertices;
    m.indices = indices;
    m.num_triangles = num_triangles;
    m.instances = instances;
    m.num_instances = num_instances;
    curast_view v{};
    std::memcpy(v.view_proj, view_proj, sizeof(float) * 16);
    v.near_plane = near_plane;
    v.width = width;
    v.height = height;
    v.visbuffer = visbuffer;
    return rasterize_impl(ctx, &m, 1, &v, 1, static_cast<hipStream_t>(stream), false);
}

int curast_rasterize_noalloc(curast_ctx* ctx, const float* vertices, uint32_t num_vertices, const uint32_t* indices,
                             uint64_t num_triangles, const float* instances, uint32_t num_instances,
                             const float view_proj[16], float near_plane, int32_t width, int32_t height,
                             uint64_t* visbuffer, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!view_proj) return fail(ctx, CURAST_E_INVALID, "view_proj is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    curast_mesh m{};
    m.vertices = vertices;
    m.num_vertices = num_vertices;
    m.indices = indices;
    m.num_triangles = num_triangles;
    m.instances = instances;
    m.num_instances = num_instances;
    curast_view v{};
    std::memcpy(v.view_proj, view_proj, sizeof(float) * 16);
    v.near_plane = near_plane;
    v.width = width;
    v.height = height;
    v.visbuffer = visbuffer;
    return rasterize_noalloc(ctx, m, v, static_cast<hipStream_t>(stream));
}

int curast_rasterize_batched(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* views,
                             uint32_t n_views, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    const bool graph = !(ctx->opt.flags & kFlagNoGraph);
    return rasterize_impl(ctx, meshes, M, views, n_views, static_cast<hipStream_t>(stream), graph);
}

int curast_project(curast_ctx* ctx, const curast_mesh* mesh, uint32_t instance, const curast_view* view, float* pos_ss,
                   void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!mesh || !view || !pos_ss) return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    int rc = check_view(ctx, *view, false);
    if (rc) return rc;
    rc = check_mesh(ctx, *mesh);
    if (rc) return rc;
    if (instance >= n_inst(*mesh)) return fail(ctx, CURAST_E_INVALID, "instance out of range");
    if (mesh->num_vertices && !mesh->vertices && !mesh->compressed)
        return fail(ctx, CURAST_E_INVALID, "vertices is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    float A[12];
    draw_matrix(view->view_proj, mesh->instances ? mesh->instances + 12ull * instance : nullptr, A);
    HIP_TRY(ctx, launch_project(mesh_desc(*mesh), A, 0.5f * (float)view->width,
                                0.5f * (float)view->height, pos_ss, static_cast<hipStream_t>(stream)));
    return CURAST_OK;
}

namespace {
int resolve_impl(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                 const float* const* attrs, uint32_t C, float* out, uint32_t ss, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!view || !out || (M && (!meshes || !attrs))) return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    if (C < 1 || C > 16) return fail(ctx, CURAST_E_INVALID, "C must lie in [1, 16]");
    if (ss != 1 && ss != 2 && ss != 4) return fail(ctx, CURAST_E_INVALID, "samples per axis must be 1, 2 or 4");
    int rc = check_view(ctx, *view);
    if (rc) return rc;
    if (view->width % (int32_t)ss || view->height % (int32_t)ss)
        return fail(ctx, CURAST_E_INVALID, "view size must be a multiple of the samples per axis");
    uint64_t total = 0;
    for (uint32_t m = 0; m < M; ++m) {
        rc = check_mesh(ctx, meshes[m]);
        if (rc) return rc;
        if (meshes[m].num_triangles && !attrs[m]) return fail(ctx, CURAST_E_INVALID, "attrs[m] is NULL");
        total += meshes[m].num_triangles * (uint64_t)n_inst(meshes[m]);
        if (total > kMaxIds) return fail(ctx, CURAST_E_ID_RANGE, "more than 2^36 triangle instances");
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ResolveArgs a{};
    size_t bytes = 0;
    rc = build_resolve_desc(ctx, meshes, M, *view, attrs, nullptr, a, bytes);
    if (rc) return rc;
    a.C = C;
    a.out = out;
    a.ss = ss;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->resolve_stage.dev, ctx->resolve_stage.host, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipEventRecord(ctx->resolve_stage.ev, s));
    ctx->resolve_stage.pending = true;
    TimedFrame* tf = begin_timing(ctx);
    if (tf) hipEventRecord(tf->ev[7], s);
    HIP_TRY(ctx, launch_resolve(a, s));
    if (tf) {
        hipEventRecord(tf->ev[8], s);
        tf->used[kTResolve] = 1;
    }
    return CURAST_OK;
}
}  // namespace

int curast_resolve(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                   const float* const* attrs, uint32_t C, float* out, void* stream)
{
    return resolve_impl(ctx, meshes, M, view, attrs, C, out, 1, stream);
}

int curast_resolve_supersampled(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                                uint32_t samples_per_axis, const float* const* attrs, uint32_t C, float* out,
                                void* stream)
{
    return resolve_impl(ctx, meshes, M, view, attrs, C, out, samples_per_axis, stream);
}

uint64_t curast_texture_texels(uint32_t width, uint32_t height, uint32_t levels)
{
    auto pow2 = [](uint32_t d) { return d && !(d & (d - 1)) && d <= (uint32_t)kMaxDim; };
    if (!pow2(width) || !pow2(height) || levels < 1) return 0;
    const uint32_t max_levels = 1 + (31 - (uint32_t)__builtin_clz(std::max(width, height)));
    if (levels > max_levels) return 0;
    uint64_t n = 0;
    for (uint32_t l = 0; l < levels; ++l) n += (uint64_t)std::max(1u, width >> l) * std::max(1u, height >> l);
    return n;
}

int curast_build_mips(curast_ctx* ctx, uint32_t* texels, uint32_t width, uint32_t height, uint32_t levels,
                      void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!texels) return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    if (!curast_texture_texels(width, height, levels))
        return fail(ctx, CURAST_E_INVALID, "texture sizes must be powers of two in [1, 16384] with 1 .. 1 + log2(max) levels");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_build_mips(texels, width, height, levels, static_cast<hipStream_t>(stream)));
    return CURAST_OK;
}

int curast_resolve_textured(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                            const float* const* uvs, const curast_texture* textures, float* out, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!view || !out || (M && (!meshes || !uvs || !textures))) return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    int rc = check_view(ctx, *view);
    if (rc) return rc;
    uint64_t total = 0;
    for (uint32_t m = 0; m < M; ++m) {
        rc = check_mesh(ctx, meshes[m]);
        if (rc) return rc;
        const curast_texture& t = textures[m];
        if (!curast_texture_texels(t.width, t.height, t.levels))
            return fail(ctx, CURAST_E_INVALID, "texture sizes must be powers of two in [1, 16384] with 1 .. 1 + log2(max) levels");
        if (meshes[m].num_triangles && (!uvs[m] || !t.texels))
            return fail(ctx, CURAST_E_INVALID, "uvs[m] and textures[m].texels must be set for a mesh with triangles");
        total += meshes[m].num_triangles * (uint64_t)n_inst(meshes[m]);
        if (total > kMaxIds) return fail(ctx, CURAST_E_ID_RANGE, "more than 2^36 triangle instances");
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ResolveArgs a{};
    size_t bytes = 0;
    rc = build_resolve_desc(ctx, meshes, M, *view, uvs, textures, a, bytes);
    if (rc) return rc;
    a.C = 2;
    a.out = out;
    a.ss = 1;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->resolve_stage.dev, ctx->resolve_stage.host, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipEventRecord(ctx->resolve_stage.ev, s));
    ctx->resolve_stage.pending = true;
    TimedFrame* tf = begin_timing(ctx);
    if (tf) hipEventRecord(tf->ev[7], s);
    HIP_TRY(ctx, launch_resolve_textured(a, s));
    if (tf) {
        hipEventRecord(tf->ev[8], s);
        tf->used[kTResolve] = 1;
    }
    return CURAST_OK;
}

namespace {
int check_plain_mesh(curast_ctx* ctx, const curast_mesh* mesh)
{
    if (!mesh) return fail(ctx, CURAST_E_INVALID, "mesh is NULL");
    if (mesh->compressed) return fail(ctx, CURAST_E_INVALID, "the mesh to compress must be uncompressed");
    int rc = check_mesh(ctx, *mesh);
    if (rc) return rc;
    if (mesh->num_vertices && !mesh->vertices) return fail(ctx, CURAST_E_INVALID, "vertices is NULL");
    return CURAST_OK;
}

// Inverse of the device's order-preserving map of binary32 to uint32.
float binary32_of_ordered(uint32_t o)
{
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

// Quantization scale of an axis from its step: the rounded reciprocal, 0 for a flat axis.
float quant_scale(float step) { return step > 0.0f ? (float)(1.0 / (double)step) : 0.0f; }
}  // namespace

int curast_compress_prepare(curast_ctx* ctx, const curast_mesh* mesh, curast_compressed* info, uint64_t* index_words,
                            void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!info || !index_words) return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    int rc = check_plain_mesh(ctx, mesh);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ctx->ranges) HIP_TRY(ctx, hipMalloc(&ctx->ranges, 8 * sizeof(uint32_t)));
    const uint64_t n_idx = 3ull * mesh->num_triangles;
    HIP_TRY(ctx, launch_compress_ranges(mesh->indices, n_idx, mesh->vertices, mesh->num_vertices, ctx->ranges,
                                        (uint32_t)ctx->cus, s));
    uint32_t r[8];
    HIP_TRY(ctx, hipMemcpyAsync(r, ctx->ranges, sizeof r, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const uint32_t imin = n_idx ? r[0] : 0u, imax = n_idx ? r[1] : 0u;
    const uint32_t span = imax - imin;
    info->index_min = imin;
    info->index_bits = span ? 32u - (uint32_t)__builtin_clz(span) : 1u;
    for (int c = 0; c < 3; ++c) {
        const float lo = mesh->num_vertices ? binary32_of_ordered(r[2 + c]) : 0.0f;
        const float hi = mesh->num_vertices ? binary32_of_ordered(r[5 + c]) : 0.0f;
        if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(ctx, CURAST_E_INVALID, "positions must be finite");
        info->lo[c] = lo;
        info->step[c] = (float)(((double)hi - (double)lo) / 65535.0);
    }
    *index_words = (n_idx * info->index_bits + 31) / 32 + 3;
    return CURAST_OK;
}

int curast_compress(curast_ctx* ctx, const curast_mesh* mesh, const curast_compressed* info, uint32_t* packed_indices,
                    uint16_t* positions, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!info || !packed_indices || !positions)
        return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    int rc = check_plain_mesh(ctx, mesh);
    if (rc) return rc;
    if (info->index_bits < 1 || info->index_bits > 32) return fail(ctx, CURAST_E_INVALID, "index_bits must lie in [1, 32]");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const uint64_t n_idx = 3ull * mesh->num_triangles;
    const uint64_t words = (n_idx * info->index_bits + 31) / 32 + 3;
    const float scale[3] = {quant_scale(info->step[0]), quant_scale(info->step[1]), quant_scale(info->step[2])};
    HIP_TRY(ctx, launch_compress(mesh->indices, n_idx, info->index_bits, info->index_min, packed_indices, words,
                                 mesh->vertices, mesh->num_vertices, info->lo, scale, positions,
                                 static_cast<hipStream_t>(stream)));
    return CURAST_OK;
}

int curast_resolve_screen(curast_ctx* ctx, const uint64_t* visbuffer, int32_t width, int32_t height,
                          const uint32_t* indices, uint64_t num_triangles, uint64_t id_base, const float* pos_ss,
                          uint32_t num_vertices, const float* attrs, uint32_t C, float* out, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    int rc = check_screen(ctx, visbuffer, width, height, indices, num_triangles, pos_ss, num_vertices, attrs, C);
    if (rc) return rc;
    if (!out) return fail(ctx, CURAST_E_INVALID, "out is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ScreenArgs a{};
    a.vis = reinterpret_cast<const unsigned long long*>(visbuffer);
    a.W = width;
    a.H = height;
    a.idx = indices;
    a.T = num_triangles;
    a.id_base = id_base;
    a.pos_ss = pos_ss;
    a.V = num_vertices;
    a.attrs = attrs;
    a.C = C;
    a.out = out;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TimedFrame* tf = begin_timing(ctx);
    if (tf) hipEventRecord(tf->ev[7], s);
    HIP_TRY(ctx, launch_resolve_screen(a, s));
    if (tf) {
        hipEventRecord(tf->ev[8], s);
        tf->used[kTResolve] = 1;
    }
    return CURAST_OK;
}

int curast_resolve_backward(curast_ctx* ctx, const uint64_t* visbuffer, int32_t width, int32_t height,
                            const uint32_t* indices, uint64_t num_triangles, uint64_t id_base, const float* pos_ss,
                            uint32_t num_vertices, const float* attrs, uint32_t C, const float* grad_out,
                            float* grad_attr, float* grad_pos, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    int rc = check_screen(ctx, visbuffer, width, height, indices, num_triangles, pos_ss, num_vertices, attrs, C);
    if (rc) return rc;
    if (!grad_out || !grad_attr) return fail(ctx, CURAST_E_INVALID, "grad_out and grad_attr are required");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ScreenArgs a{};
    a.vis = reinterpret_cast<const unsigned long long*>(visbuffer);
    a.W = width;
    a.H = height;
    a.idx = indices;
    a.T = num_triangles;
    a.id_base = id_base;
    a.pos_ss = pos_ss;
    a.V = num_vertices;
    a.attrs = attrs;
    a.C = C;
    a.grad_out = grad_out;
    a.grad_attr = grad_attr;
    a.grad_pos = grad_pos;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TimedFrame* tf = begin_timing(ctx);
    if (tf) hipEventRecord(tf->ev[7], s);
    HIP_TRY(ctx, launch_resolve_backward(a, s));
    if (tf) {
        hipEventRecord(tf->ev[8], s);
        tf->used[kTResolveBwd] = 1;
    }
    return CURAST_OK;
}

int curast_resolve_backward_meshes(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* view,
                                   const float* const* attrs, uint32_t C, const float* grad_out,
                                   float* const* grad_attrs, float* const* grad_pos, void* stream)
{
    if (!ctx) return CURAST_E_INVALID;
    if (!view || !grad_out || (M && (!meshes || !attrs || !grad_attrs)))
        return fail(ctx, CURAST_E_INVALID, "NULL pointer argument");
    if (C < 1 || C > 16) return fail(ctx, CURAST_E_INVALID, "C must lie in [1, 16]");
    int rc = check_view(ctx, *view);
    if (rc) return rc;
    uint64_t total = 0;
    for (uint32_t m = 0; m < M; ++m) {
        rc = check_mesh(ctx, meshes[m]);
        if (rc) return rc;
        if (meshes[m].num_triangles && !attrs[m]) return fail(ctx, CURAST_E_INVALID, "attrs[m] is NULL");
        if (grad_pos && grad_pos[m] && n_inst(meshes[m]) != 1)
            return fail(ctx, CURAST_E_INVALID, "position gradients only for meshes with one instance");
        total += meshes[m].num_triangles * (uint64_t)n_inst(meshes[m]);
        if (total > kMaxIds) return fail(ctx, CURAST_E_ID_RANGE, "more than 2^36 triangle instances");
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ResolveArgs a{};
    size_t bytes = 0;
    rc = build_resolve_desc(ctx, meshes, M, *view, attrs, nullptr, a, bytes, grad_attrs, grad_pos);
    if (rc) return rc;
    a.C = C;
    a.grad_out = grad_out;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->resolve_stage.dev, ctx->resolve_stage.host, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipEventRecord(ctx->resolve_stage.ev, s));
    ctx->resolve_stage.pending = true;
    TimedFrame* tf = begin_timing(ctx);
    if (tf) hipEventRecord(tf->ev[7], s);
    HIP_TRY(ctx, launch_resolve_backward_meshes(a, s));
    if (tf) {
        hipEventRecord(tf->ev[8], s);
        tf->used[kTResolveBwd] = 1;
    }
    return CURAST_OK;
}

int curast_get_stats(curast_ctx* ctx, curast_stats* out)
{
    if (!ctx || !out) return CURAST_E_INVALID;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    unsigned long long s[kNumStats];
    HIP_TRY(ctx, hipMemcpy(s, ctx->stats, sizeof s, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof *out);
    out->tri_draws = s[kStTriDraws];
    out->draws_culled = ctx->draws_culled;
    out->culled_near = s[kStCulledNear];
    out->culled_frustum = s[kStCulledFrustum];
    out->culled_tiny = s[kStCulledTiny];
    out->culled_backface = s[kStCulledBack];
    out->s1_rasterized = s[kStS1Raster];
    out->q2_entries = s[kStQ2];
    out->q2_overflow = s[kStQ2Overflow];
    out->s2_rasterized = s[kStS2Raster];
    out->q3_entries = s[kStQ3];
    out->q3_overflow = s[kStQ3Overflow];
    out->fragments = s[kStFragments];
    out->atomics = s[kStAtomics];
    out->strip_draws = s[kStStripDraws];
    out->strip_union_pass = s[kStStripPass];
    out->strip_sphere_pass = s[kStSpherePass];
    return CURAST_OK;
}

int curast_reset_stats(curast_ctx* ctx)
{
    if (!ctx) return CURAST_E_INVALID;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemset(ctx->stats, 0, sizeof(unsigned long long) * kNumStats));
    ctx->draws_culled = 0;
    return CURAST_OK;
}

int curast_get_stage_times(curast_ctx* ctx, double* ms, uint64_t* frames)
{
    if (!ctx || !ms) return CURAST_E_INVALID;
    collect_timings(ctx);
    for (int i = 0; i < kNumSlots; ++i) ms[i] = ctx->stage_ms[i];
    if (frames) *frames = ctx->timed_frames;
    return CURAST_OK;
}

int curast_reset_stage_times(curast_ctx* ctx)
{
    if (!ctx) return CURAST_E_INVALID;
    collect_timings(ctx);
    for (int i = 0; i < kNumSlots; ++i) ctx->stage_ms[i] = 0.0;
    ctx->timed_frames = 0;
    return CURAST_OK;
}

int curast_plan(const curast_mesh* meshes, uint32_t M, const curast_view* views, uint32_t n_views,
                const curast_options* opt, uint8_t* visible, int64_t* bases, uint64_t counts[4])
{
    curast_options u{};
    if (opt) u = *opt;
    std::string msg;
    if (validate_options(u, msg)) return CURAST_E_INVALID;
    const curast_options o = resolve_defaults(u, 256);
    Plan P;
    int rc = build_plan(nullptr, o, meshes, M, views, n_views, P, visible);
    if (rc) return rc;
    log_plan("plan", P, M, n_views);
    if (bases) {
        int64_t n = curast_id_bases(meshes, M, bases);
        if (n < 0) return (int)n;
    }
    if (counts) {
        counts[0] = P.draws.size();
        counts[1] = P.draws_culled;
        counts[2] = P.hdr.total_batches;
        counts[3] = P.tri_draws;
    }
    return CURAST_OK;
}

// Queue fill of the last frame (internal, used by the autotuner): Q2, large records, Q3.
int curast_internal_queue_counts(curast_ctx* ctx, uint64_t out[3])
{
    if (!ctx || !out) return CURAST_E_INVALID;
    HIP_TRY(ctx, hipDeviceSynchronize());
    unsigned long long c[kNumCounters];
    HIP_TRY(ctx, hipMemcpy(c, ctx->counters, sizeof c, hipMemcpyDeviceToHost));
    out[0] = c[kCntQ2];
    out[1] = c[kCntLarge];
    out[2] = c[kCntQ3];
    return CURAST_OK;
}

int curast_internal_num_cus(const curast_ctx* ctx) { return ctx ? ctx->cus : 0; }

// The library defaults on this context's device (internal, used by the autotuner).
int curast_internal_default_options(const curast_ctx* ctx, curast_options* out)
{
    if (!ctx || !out) return CURAST_E_INVALID;
    *out = resolve_defaults(curast_options{}, ctx->cus);
    return CURAST_OK;
}

int64_t curast_id_bases(const curast_mesh* meshes, uint32_t M, int64_t* bases)
{
    if (M && !meshes) return CURAST_E_INVALID;
    int64_t p = 0;
    uint64_t acc = 0;
    for (uint32_t m = 0; m < M; ++m) {
        if (meshes[m].instances && meshes[m].num_instances == 0) return CURAST_E_INVALID;
        for (uint32_t i = 0; i < n_inst(meshes[m]); ++i) {
            if (bases) bases[p] = (int64_t)acc;
            ++p;
            acc += meshes[m].num_triangles;
        }
    }
    if (acc > kMaxIds) return CURAST_E_ID_RANGE;
    if (bases) bases[p] = (int64_t)acc;
    return p;
}

}  // extern "C"

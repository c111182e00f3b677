// Rasterization kernels for gfx950: clear, stage 1 (one lane per small triangle), the stage-1
// overflow pass, stage 2 (a wavefront sets up 64 medium triangles in parallel, clipping them, then
// rasterizes them one by one) and stage 3 (one workgroup per 64x64 tile part of a large
// triangle).  Sec. 4.1-4.3 describe the three stages; the wave64
// mapping, ballot-compacted queues and in-place overflow handling are this implementation's.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"

namespace curast {

// ----------------------------------------------------------------------------------------------
// Statistics (compiled in only for the STATS variants)
// ----------------------------------------------------------------------------------------------
template <bool ON>
struct StatAcc {
    uint32_t v[kNumStats];
    __device__ StatAcc()
    {
        for (int i = 0; i < kNumStats; ++i) v[i] = 0;
    }
    __device__ void add(int i, uint32_t n = 1) { v[i] += n; }
    __device__ void flush(unsigned long long* out)
    {
        for (int i = 0; i < kNumStats; ++i) {
            uint32_t s = v[i];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if ((threadIdx.x & 63) == 0 && s) atomicAdd(out + i, (unsigned long long)s);
        }
    }
};

template <>
struct StatAcc<false> {
    __device__ void add(int, uint32_t = 1) {}
    __device__ void flush(unsigned long long*) {}
};

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_in(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-aggregated append: one 64-bit atomic per wavefront reserves slots for every lane with
// `want`, each lane writes its entry at base + its rank among the wanting lanes.  Must be called
// by all lanes of the wavefront.  Returns the slot (or ~0 when the lane did not append).
__device__ __forceinline__ unsigned long long wave_reserve(bool want, unsigned long long* counter)
{
    const unsigned long long mask = __ballot(want);
    if (mask == 0) return ~0ull;
    const uint32_t leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    return want ? base + rank_in(mask) : ~0ull;
}

// ----------------------------------------------------------------------------------------------
// Stage-1 classification of one triangle under one draw (shared by stage 1 and its overflow pass)
// ----------------------------------------------------------------------------------------------
enum Route : int { kRouteNone = 0, kRouteSmall = 1, kRouteForward = 2 };

struct SmallTri {
    int32_t X[3], Y[3];
    float zI[3];
    int32_t px0, px1, py0, py1;
    int32_t area;
};

template <bool STATS>
__device__ __forceinline__ int classify(const Clip c[3], const ViewDesc& V, uint32_t small_px, bool tiny_cull,
                                        SmallTri& s, StatAcc<STATS>& st)
{
    const float n = V.near_plane;
    if (c[0].w < n && c[1].w < n && c[2].w < n) {
        st.add(kStCulledNear);
        return kRouteNone;
    }
    if (outside_guard(c[0], n) || outside_guard(c[1], n) || outside_guard(c[2], n)) return kRouteForward;
    // all vertices beyond one side of the view: no pixel centre can be covered (the half-pixel
    // between the view border and the first centre absorbs every rounding of the projection)
    if ((c[0].x > c[0].w && c[1].x > c[1].w && c[2].x > c[2].w) ||
        (c[0].x < -c[0].w && c[1].x < -c[1].w && c[2].x < -c[2].w) ||
        (c[0].y > c[0].w && c[1].y > c[1].w && c[2].y > c[2].w) ||
        (c[0].y < -c[0].w && c[1].y < -c[1].w && c[2].y < -c[2].w)) {
        st.add(kStCulledFrustum);
        return kRouteNone;
    }
    for (int k = 0; k < 3; ++k) snap_vertex(c[k], V.hW, V.hH, s.X[k], s.Y[k], s.zI[k]);
    const int32_t minX = min(s.X[0], min(s.X[1], s.X[2])), maxX = max(s.X[0], max(s.X[1], s.X[2]));
    const int32_t minY = min(s.Y[0], min(s.Y[1], s.Y[2])), maxY = max(s.Y[0], max(s.Y[1], s.Y[2]));
    s.px0 = max(first_centre(minX), 0);
    s.px1 = min(last_centre(maxX), V.W - 1);
    s.py0 = max(first_centre(minY), 0);
    s.py1 = min(last_centre(maxY), V.H - 1);
    const bool empty = s.px0 > s.px1 || s.py0 > s.py1;
    if (empty && tiny_cull) {
        st.add(kStCulledTiny);
        return kRouteNone;
    }
    if (maxX - minX >= kSmallExtent || maxY - minY >= kSmallExtent) return kRouteForward;
    const int32_t cnt = empty ? 0 : (s.px1 - s.px0 + 1) * (s.py1 - s.py0 + 1);
    if (cnt > (int32_t)small_px) return kRouteForward;
    // extents < 2^15: the products fit 24-bit multiplies and the area fits int32
    s.area = __mul24(s.X[1] - s.X[0], s.Y[2] - s.Y[0]) - __mul24(s.Y[1] - s.Y[0], s.X[2] - s.X[0]);
    if (s.area <= 0) {
        st.add(kStCulledBack);
        return kRouteNone;
    }
    return kRouteSmall;
}

// One lane rasterizes a small triangle over its bounding box (Sec. 4.1): y outer, x inner,
// incremental int32 edge values (see kSmallExtent for the range argument).
template <bool STATS>
__device__ __forceinline__ void raster_small(const SmallTri& s, uint64_t id, const ViewDesc& V, bool early_out,
                                             StatAcc<STATS>& st)
{
    int32_t sdx[3], sdy[3], row[3], bias[3];
    const int32_t Px0 = 256 * s.px0 + 128, Py0 = 256 * s.py0 + 128;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = k == 2 ? 0 : k + 1;
        const int b = k == 0 ? 2 : k - 1;
        const int32_t dx = s.X[b] - s.X[a];
        const int32_t dy = s.Y[b] - s.Y[a];
        bias[k] = top_left(dx, dy) ? 0 : -1;
        row[k] = __mul24(dx, Py0 - s.Y[a]) - __mul24(dy, Px0 - s.X[a]) + bias[k];
        sdx[k] = dx * 256;
        sdy[k] = dy * 256;
    }
    const float area_f = (float)s.area;
    for (int32_t py = s.py0; py <= s.py1; ++py) {
        int32_t g0 = row[0], g1 = row[1], g2 = row[2];
        for (int32_t px = s.px0; px <= s.px1; ++px) {
            if ((g0 | g1 | g2) >= 0) {
                const float depth = frag_depth((float)(g0 - bias[0]), (float)(g1 - bias[1]), (float)(g2 - bias[2]),
                                               s.zI, area_f);
                unsigned long long* p = V.vis + (size_t)py * (size_t)V.W + (size_t)px;
                const unsigned long long key = make_key(depth, id);
                st.add(kStFragments);
                if (STATS) {
                    if (!early_out || key < *p) st.add(kStAtomics);
                }
                write_fragment(p, key, early_out);
            }
            g0 -= sdy[0];
            g1 -= sdy[1];
            g2 -= sdy[2];
        }
        row[0] += sdx[0];
        row[1] += sdx[1];
        row[2] += sdx[2];
    }
}

// One thread rasterizes any triangle (clipping, fan, int64 edges): the overflow fallback.
__device__ inline void raster_any_thread(const Clip c[3], uint64_t id, const ViewDesc& V, bool early_out)
{
    Clip poly[8];
    int n = 3;
    if (outside_guard(c[0], V.near_plane) || outside_guard(c[1], V.near_plane) || outside_guard(c[2], V.near_plane)) {
        n = clip_triangle(c, V.near_plane, poly);
    } else {
        poly[0] = c[0];
        poly[1] = c[1];
        poly[2] = c[2];
    }
    if (n < 3) return;
    int32_t X[8], Y[8];
    float zI[8];
    for (int k = 0; k < n; ++k) snap_vertex(poly[k], V.hW, V.hH, X[k], Y[k], zI[k]);
    for (int j = 1; j + 1 < n; ++j) {
        const int32_t tx[3] = {X[0], X[j], X[j + 1]}, ty[3] = {Y[0], Y[j], Y[j + 1]};
        const float tz[3] = {zI[0], zI[j], zI[j + 1]};
        Tri64 t;
        if (!setup_tri64(tx, ty, tz, V.W, V.H, t)) continue;
        for (int32_t py = t.py0; py <= t.py1; ++py)
            for (int32_t px = t.px0; px <= t.px1; ++px) raster_pixel64(t, px, py, id, V.vis, V.W, early_out);
    }
}

// ----------------------------------------------------------------------------------------------
// Clear (also resets the queue counters of the frame)
// ----------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) clear_kernel(RasterArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x < kNumCounters) a.counters[threadIdx.x] = 0;
    const uint32_t nv = a.hdr->n_views;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t nt = a.hdr->n_tiles;
    for (uint64_t i = tid; i < nt; i += stride) a.tile_count[i] = 0;
    for (uint32_t v = 0; v < nv; ++v) {
        const ViewDesc V = a.views[v];
        const uint64_t n = (uint64_t)V.W * (uint64_t)V.H;
        if (((uintptr_t)V.vis & 15) == 0) {
            ulonglong2* p = reinterpret_cast<ulonglong2*>(V.vis);
            const uint64_t n2 = n >> 1;
            for (uint64_t i = tid; i < n2; i += stride) p[i] = make_ulonglong2(~0ull, ~0ull);
            if ((n & 1) && tid == 0) V.vis[n - 1] = ~0ull;
        } else {
            for (uint64_t i = tid; i < n; i += stride) V.vis[i] = ~0ull;
        }
    }
}

// ----------------------------------------------------------------------------------------------
// Stage 1: one lane per triangle, looping over the draws (instances x views) of its work item
// ----------------------------------------------------------------------------------------------
// Work-item values are the same on every lane; readfirstlane puts them in scalar registers so the
// draw and view descriptors they index are fetched with scalar loads.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

struct WorkItem {
    uint32_t mesh;
    uint64_t tri_batch;
    uint32_t d0, d1;
    uint32_t batch_tris;
};

__device__ __forceinline__ WorkItem locate_work(const Segment* __restrict__ segs, uint32_t n_segs, uint32_t dpi, uint64_t b);

__device__ __forceinline__ uint32_t find_segment(const Segment* __restrict__ segs, uint32_t n_segs, uint64_t b)
{
    uint32_t lo = 0, hi = n_segs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (segs[mid].batch_begin <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Range of stage-1 work items a launch covers (see RasterArgs::part).
__device__ __forceinline__ void work_range(const FrameHeader& h, uint32_t part, uint64_t& begin, uint64_t& end)
{
    begin = part == 2 ? uni64(h.shared_batches) : 0;
    end = part == 1 ? uni64(h.shared_batches) : uni64(h.total_batches);
}

// Work item b -> (mesh, triangle batch, draw range), all uniform.
__device__ __forceinline__ WorkItem locate_work(const Segment* __restrict__ segs, uint32_t n_segs, uint32_t dpi, uint64_t b)
{
    const uint32_t si = uni(find_segment(segs, n_segs, b));
    const Segment sg = segs[si];
    const uint64_t begin = uni64(sg.batch_begin);
    const uint32_t ng = uni(sg.n_groups);
    const uint32_t db = uni(sg.draw_begin);
    const uint32_t dc = uni(sg.draw_count);
    const uint64_t j = b - begin;
    WorkItem w;
    w.mesh = uni(sg.mesh);
    w.batch_tris = uni(sg.batch_tris);
    uint32_t g = 0;
    if (ng == 1) {
        w.tri_batch = j;
    } else {
        w.tri_batch = uni64(j / ng);
        g = uni((uint32_t)(j - w.tri_batch * ng));
    }
    w.d0 = db + g * dpi;
    w.d1 = min(db + dc, w.d0 + dpi);
    return w;
}

#define CURAST_DESC_PARAMS                                                                       \
    const FrameHeader* __restrict__ d_hdr, const ViewDesc* __restrict__ d_views,                  \
        const MeshDesc* __restrict__ d_meshes, const Segment* __restrict__ d_segs,                \
        const DrawDesc* __restrict__ d_draws
#define CURAST_DESC_ARGS(a) (a).hdr, (a).views, (a).meshes, (a).segs, (a).draws

template <int BLOCK, int TPT, bool STATS>
__global__ void __launch_bounds__(BLOCK) stage1_kernel(RasterArgs a, CURAST_DESC_PARAMS)
{
    const FrameHeader hdr = *d_hdr;
    uint64_t first, total;
    work_range(hdr, a.part, first, total);
    const uint32_t n_segs = uni(hdr.n_segs);
    const uint32_t dpi = uni(hdr.draws_per_item);
    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    const bool tiny_cull = !(a.flags & kFlagNoTinyCull);
    StatAcc<STATS> st;
    for (uint64_t b = first + blockIdx.x; b < total; b += gridDim.x) {
        const WorkItem wi = locate_work(d_segs, n_segs, dpi, b);
        const uint64_t tb = wi.tri_batch;
        const uint32_t d0 = wi.d0, d1 = wi.d1;
        const MeshDesc mesh = d_meshes[wi.mesh];
#pragma unroll 1
        for (int k = 0; k < TPT; ++k) {
            const uint64_t t = tb * (uint64_t)(BLOCK * TPT) + (uint64_t)(k * BLOCK) + threadIdx.x;
            bool valid = t < mesh.T;
            float p[9];
            if (valid) {
                uint32_t iv[3];
                mesh_triangle(mesh, t, iv);
                valid = iv[0] < mesh.V && iv[1] < mesh.V && iv[2] < mesh.V;
                if (valid) {
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        float q[3];
                        mesh_vertex(mesh, iv[v], q);
                        p[3 * v] = q[0];
                        p[3 * v + 1] = q[1];
                        p[3 * v + 2] = q[2];
                    }
                }
            }
#pragma unroll 1
            for (uint32_t d = d0; d < d1; ++d) {
                const DrawDesc D = d_draws[d];
                const ViewDesc V = d_views[D.view & kDrawViewMask];
                int route = kRouteNone;
                SmallTri s;
                if (valid) {
                    st.add(kStTriDraws);
                    const Clip c[3] = {transform(D.A, p[0], p[1], p[2]), transform(D.A, p[3], p[4], p[5]),
                                       transform(D.A, p[6], p[7], p[8])};
                    route = classify<STATS>(c, V, a.small_px, tiny_cull, s, st);
                }
                const unsigned long long slot = wave_reserve(route == kRouteForward, a.counters + kCntQ2);
                if (route == kRouteForward) {
                    st.add(kStQ2);
                    if (slot < a.q2_cap) {
                        Q2Entry e;
                        e.draw = d;
                        e.tri = (uint32_t)t;
                        a.q2[slot] = e;
                    } else {
                        st.add(kStQ2Overflow);
                    }
                }
                if (route == kRouteSmall) {
                    st.add(kStS1Raster);
                    raster_small<STATS>(s, D.id_base + t, V, early_out, st);
                }
            }
        }
    }
    st.flush(a.stats);
}

// ----------------------------------------------------------------------------------------------
// Stage 1, fast variant.  Changes to the lane-per-triangle loop, none of which changes a single
// fragment:
//  (1) a conservative reject with approximate window positions (v_rcp_f32 instead of the correctly
//      rounded 1/w) and a bounding box widened by kFastMargin pixels: when the widened box holds no
//      pixel centre inside the view, the exact box cannot hold one either, so the triangle is
//      culled without the exact arithmetic (almost every triangle of a dense mesh ends here);
//  (2) the few undecided (triangle, draw) pairs are appended to a list in LDS and run through the
//      exact classification and rasterization together, so no lane idles while one lane of its
//      wavefront takes the long path;
//  (3) interior draws (bounding sphere inside |x|, |y| <= 1.99 w, w >= 1.001 near, checked on the
//      host) skip the per-vertex range tests and take their window position from two prescaled
//      rows, x'' = hW (row x + row w) . (v, 1) and likewise y'', so that x''/w is the window x;
//  (4) with STRIPS a lane owns TPT consecutive triangles; when every lane's triangles form a
//      strip (each shares an edge with the next, as along the rows of a grid or the bands of a
//      sphere) they need TPT + 2 window positions per draw instead of 3 TPT, and one test of the
//      box around all of them rejects the whole strip (it contains each triangle's box).
//
// Error bounds (u = 2^-24; S_r = sum_j |row_rj| |v_j| + |row_r3| over the vertex, w its depth):
//  exact path: x and w carry at most 3u S_x and 3u S_w of fma-chain error, and 1/w, x*zI and the
//      window fma add 7u hW; snapping adds 2^-9 px;
//  fast path from the exact x, w (general draws, |x|, |y| <= 2w): rcp (1 ulp) and the two roundings
//      after it differ from the exact path by at most 1.625 hW 2^-20 px;
//  prescaled path: rounding the rows to binary32 and the fma chain give |x'' - hW (x + w)| <=
//      4u hW (S_x + S_w), the reciprocal of the same w adds 9u S_w hW / w, and rcp with the
//      multiply 9u hW, so the fast position is within hW u ((7 S_x + 19 S_w) / w + 16) of the
//      exact one; the host enables the path for a draw only when this bound over its bounding
//      sphere, plus 2^-9 px of snapping and 3.1u hW of box arithmetic, is below kFastMargin.
// ----------------------------------------------------------------------------------------------
constexpr float kFastMargin = 1.0f / 32.0f;
constexpr float kFastGuard = 2.0f;

// Clip-plane bits of a vertex: 1 x > w, 2 x < -w, 4 y > w, 8 y < -w, 16 w < near.  A bit that all
// vertices of a strip share puts every triangle of it (the convex hull of its clip-space vertices)
// outside the view or in front of the near plane: the exact near and side tests of the stage-1
// classification.
__device__ __forceinline__ uint32_t clip_bits(const Clip& c, float near_plane)
{
    return (uint32_t)(c.x > c.w) | (uint32_t)(c.x < -c.w) << 1 | (uint32_t)(c.y > c.w) << 2 |
           (uint32_t)(c.y < -c.w) << 3 | (uint32_t)(c.w < near_plane) << 4;
}

// With BITS, the y of a vertex outside the fast range carries its clip_bits (bit pattern).
template <bool BITS = false>
__device__ __forceinline__ float2 fast_window(const Clip& c, const ViewDesc& V)
{
    const float g = kFastGuard * c.w;
    if (!(c.w >= V.near_plane) || !(c.w < 1e30f) || __builtin_fabsf(c.x) > g || __builtin_fabsf(c.y) > g)
        return make_float2(__builtin_nanf(""), BITS ? __builtin_bit_cast(float, clip_bits(c, V.near_plane)) : 0.0f);
    const float r = __builtin_amdgcn_rcpf(c.w);
    return make_float2(__builtin_fmaf(c.x * r, V.hW, V.hW), __builtin_fmaf(c.y * r, V.hH, V.hH));
}

// Same for a vertex of an interior draw (range tests proven on the host).
__device__ __forceinline__ float2 fast_window_interior(const Clip& c, const ViewDesc& V)
{
    const float r = __builtin_amdgcn_rcpf(c.w);
    return make_float2(__builtin_fmaf(c.x * r, V.hW, V.hW), __builtin_fmaf(c.y * r, V.hH, V.hH));
}

// Window position of a vertex of an interior draw from the draw's prescaled rows (see above).
__device__ __forceinline__ float2 fast_window_prescaled(const float* R, const float* Aw, float vx, float vy, float vz)
{
    const float X = row_dot(R + 0, vx, vy, vz);
    const float Y = row_dot(R + 4, vx, vy, vz);
    const float w = row_dot(Aw, vx, vy, vz);
    const float r = __builtin_amdgcn_rcpf(w);
    return make_float2(X * r, Y * r);
}

// True when the widened extent [xmin, xmax] x [ymin, ymax] of finite window positions provably
// holds no pixel centre of the view.  The centre of pixel p (an integer in [0, W-1]) is p + 0.5,
// so a centre lies in [min - m, max + m] iff some integer p in [0, W-1] has lo <= p <= hi,
// lo = min - m - 0.5, hi = max + m - 0.5.  The largest candidate is min(floor(hi), W-1), so one
// exists iff f = floor(hi) has f >= 0, f >= lo and lo <= W-1.  Without tiny culling only boxes
// wholly outside the view (f < 0 or lo > W-1) are rejected.
__device__ __forceinline__ bool fast_reject_extent(float xmin, float xmax, float ymin, float ymax, const ViewDesc& V,
                                                   bool tiny_cull)
{
    const float lx = xmin - (kFastMargin + 0.5f);
    const float fx = __builtin_floorf(xmax + (kFastMargin - 0.5f));
    const float ly = ymin - (kFastMargin + 0.5f);
    const float fy = __builtin_floorf(ymax + (kFastMargin - 0.5f));
    const bool outside = (fx < 0.0f) | (lx > V.wmax) | (fy < 0.0f) | (ly > V.hmax);
    const bool empty = (fx < lx) | (fy < ly);
    return outside | (tiny_cull & empty);
}

__device__ __forceinline__ bool fast_reject_box(float2 a, float2 b, float2 c, const ViewDesc& V, bool tiny_cull)
{
    return fast_reject_extent(fminf(a.x, fminf(b.x, c.x)), fmaxf(a.x, fmaxf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)),
                              fmaxf(a.y, fmaxf(b.y, c.y)), V, tiny_cull);
}

// Same for the output of fast_window, whose x is NaN for a vertex outside the fast range.
__device__ __forceinline__ bool fast_reject(float2 a, float2 b, float2 c, const ViewDesc& V, bool tiny_cull)
{
    if (__builtin_isnan(a.x) | __builtin_isnan(b.x) | __builtin_isnan(c.x)) return false;
    return fast_reject_box(a, b, c, V, tiny_cull);
}

// Undecided (triangle, draw) pairs wait in a per-wavefront ring in LDS; the wavefront drains 64 of
// them at a time with every lane busy.  Entries carry the exact clip coordinates where the lane
// has them at hand (ClipEntry: the drain then loads only the draw and its view); the strip
// kernels store ids (IdEntry) and the drain reloads the triangle, which is rare there.  Head and
// tail are wave-uniform (scalar), so no workgroup barrier is needed.
struct ClipEntry {
    float c[9];
    uint32_t draw;
    uint32_t tri;
};
struct IdEntry {
    uint32_t draw;
    uint32_t tri;
    uint32_t mesh;
};
constexpr int kRing = 128;

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact classification of one (draw, triangle) per lane with `have`, then Q2 or the small
// rasterizer.  Every lane of the wavefront takes part (the Q2 reservation is wave-wide).
template <bool STATS>
__device__ __forceinline__ void exact_route(const RasterArgs& a, bool have, const Clip (&c)[3], const ViewDesc& V,
                                            uint32_t dd, uint32_t tt, uint64_t idb, bool tiny_cull, bool early_out,
                                            StatAcc<STATS>& st)
{
    int route = kRouteNone;
    SmallTri s;
    if (have) route = classify<STATS>(c, V, a.small_px, tiny_cull, s, st);
    const unsigned long long slot = wave_reserve(route == kRouteForward, a.counters + kCntQ2);
    if (route == kRouteForward) {
        st.add(kStQ2);
        if (slot < a.q2_cap) {
            Q2Entry qe;
            qe.draw = dd;
            qe.tri = tt;
            a.q2[slot] = qe;
        } else {
            st.add(kStQ2Overflow);
        }
    }
    if (route == kRouteSmall) {
        st.add(kStS1Raster);
        raster_small<STATS>(s, idb + tt, V, early_out, st);
    }
}

// Drain ring entries [head, head + n), n <= 64, one per lane.
template <bool STATS>
__device__ __forceinline__ void drain_ring(const RasterArgs& a, const ViewDesc* __restrict__ d_views,
                                           const MeshDesc* __restrict__, const DrawDesc* __restrict__ d_draws,
                                           const ClipEntry* ring, uint32_t head, uint32_t n, bool tiny_cull,
                                           bool early_out, StatAcc<STATS>& st)
{
    const bool have = lane_id() < n;
    Clip c[3] = {};
    ViewDesc V;
    uint32_t dd = 0, tt = 0;
    uint64_t idb = 0;
    if (have) {
        const ClipEntry& e = ring[(head + lane_id()) & (kRing - 1)];
        dd = e.draw;
        tt = e.tri;
#pragma unroll
        for (int k = 0; k < 3; ++k) c[k] = Clip{e.c[3 * k], e.c[3 * k + 1], e.c[3 * k + 2]};
        const DrawDesc& D = d_draws[dd];
        V = d_views[D.view & kDrawViewMask];
        idb = D.id_base;
    }
    exact_route<STATS>(a, have, c, V, dd, tt, idb, tiny_cull, early_out, st);
}

template <bool STATS>
__device__ __forceinline__ void drain_ring(const RasterArgs& a, const ViewDesc* __restrict__ d_views,
                                           const MeshDesc* __restrict__ d_meshes, const DrawDesc* __restrict__ d_draws,
                                           const IdEntry* ring, uint32_t head, uint32_t n, bool tiny_cull,
                                           bool early_out, StatAcc<STATS>& st)
{
    const bool have = lane_id() < n;
    Clip c[3] = {};
    ViewDesc V;
    uint32_t dd = 0, tt = 0;
    uint64_t idb = 0;
    if (have) {
        const IdEntry e = ring[(head + lane_id()) & (kRing - 1)];
        dd = e.draw;
        tt = e.tri;
        const DrawDesc& D = d_draws[dd];
        const MeshDesc& M = d_meshes[e.mesh];
        uint32_t iv[3];
        mesh_triangle(M, tt, iv);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float q[3];
            mesh_vertex(M, iv[k], q);
            c[k] = transform(D.A, q[0], q[1], q[2]);
        }
        V = d_views[D.view & kDrawViewMask];
        idb = D.id_base;
    }
    exact_route<STATS>(a, have, c, V, dd, tt, idb, tiny_cull, early_out, st);
}

// The vertex of triangle a missing from triangle b; true when exactly one is.
__device__ __forceinline__ bool one_missing(const uint32_t (&a)[3], const uint32_t (&b)[3], uint32_t& out)
{
    bool m[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) m[j] = (a[j] != b[0]) & (a[j] != b[1]) & (a[j] != b[2]);
    out = m[0] ? a[0] : (m[1] ? a[1] : a[2]);
    return (int)m[0] + (int)m[1] + (int)m[2] == 1;
}

__device__ __forceinline__ bool in_tri(uint32_t v, const uint32_t (&t)[3]) { return (v == t[0]) | (v == t[1]) | (v == t[2]); }

// Vertex sequence v[0..S+1] with triangle k = {v[k], v[k+1], v[k+2]} as a set, for S consecutive
// triangles each sharing an edge with the next (a strip: rows of a grid, bands of a sphere).
// Returns false when the triangles do not form one; v is then unspecified.
template <int S>
__device__ __forceinline__ bool build_strip(const uint32_t (&t)[S][3], uint32_t (&v)[S + 2])
{
    static_assert(S == 2 || S == 4 || S == 8, "strips of 2, 4 or 8 triangles");
    bool ok = true;
    uint32_t out[S], nw[S];
#pragma unroll
    for (int k = 0; k + 1 < S; ++k) ok &= one_missing(t[k], t[k + 1], out[k]);
#pragma unroll
    for (int k = 1; k < S; ++k) ok &= one_missing(t[k], t[k - 1], nw[k]);
    if constexpr (S == 2) {
        v[0] = out[0];
        v[1] = out[0] == t[0][0] ? t[0][1] : (out[0] == t[0][1] ? t[0][2] : t[0][0]);
        v[2] = out[0] == t[0][0] ? t[0][2] : (out[0] == t[0][1] ? t[0][0] : t[0][1]);
        v[3] = nw[1];
    } else {
        // v_k is the vertex of triangle k that triangle k + 1 lacks (k <= S - 2); the last three are
        // the vertices that triangles S - 3 .. S - 1 add to their predecessors
#pragma unroll
        for (int k = 0; k + 1 < S; ++k) v[k] = out[k];
        v[S - 1] = nw[S - 3];
        v[S] = nw[S - 2];
        v[S + 1] = nw[S - 1];
    }
    // every triangle is exactly its three sequence vertices, all distinct
#pragma unroll
    for (int k = 0; k < S; ++k)
        ok &= in_tri(v[k], t[k]) & in_tri(v[k + 1], t[k]) & in_tri(v[k + 2], t[k]) & (v[k] != v[k + 1]) &
              (v[k] != v[k + 2]) & (v[k + 1] != v[k + 2]);
    return ok;
}

// The same test on the union box of N finite window positions.
template <int N>
__device__ __forceinline__ bool fast_reject_union(const float2 (&w)[N], const ViewDesc& V, bool tiny_cull)
{
    float x0 = w[0].x, x1 = w[0].x, y0 = w[0].y, y1 = w[0].y;
#pragma unroll
    for (int i = 1; i < N; ++i) {
        x0 = fminf(x0, w[i].x);
        x1 = fmaxf(x1, w[i].x);
        y0 = fminf(y0, w[i].y);
        y1 = fmaxf(y1, w[i].y);
    }
    return fast_reject_extent(x0, x1, y0, y1, V, tiny_cull);
}

// Clip-plane bits of a fast_window<true> output: exact for a vertex outside the fast range; for a
// finite position only the bits its distance past a view border proves (the position is within
// kFastMargin of the exact one, and w > 0, so past W means x > w).
__device__ __forceinline__ uint32_t window_bits(float2 v, const ViewDesc& V)
{
    if (__builtin_isnan(v.x)) return __builtin_bit_cast(uint32_t, v.y);
    return (uint32_t)(v.x > (V.wmax + 1.0f) + kFastMargin) | (uint32_t)(v.x < -kFastMargin) << 1 |
           (uint32_t)(v.y > (V.hmax + 1.0f) + kFastMargin) << 2 | (uint32_t)(v.y < -kFastMargin) << 3;
}

// The union test of a strip's N window positions; with BITS (positions from fast_window<true>) a
// strip with a vertex outside the fast range is still rejected when all N vertices share a
// clip-plane bit.
template <int N, bool BITS>
__device__ __forceinline__ bool fast_reject_strip(const float2 (&w)[N], bool any_nan, const ViewDesc& V, bool tiny_cull)
{
    if constexpr (BITS) {
        if (any_nan) {
            uint32_t bits = window_bits(w[0], V);
#pragma unroll
            for (int i = 1; i < N; ++i) bits &= window_bits(w[i], V);
            return bits != 0u;
        }
    }
    return !any_nan && fast_reject_union<N>(w, V, tiny_cull);
}

// Strip spheres.  Before a strip of an interior draw is projected vertex by vertex, it is tested
// through a bounding sphere (c, r) of its vertices, computed once per work item in object space.
// For a vertex v = c + d, |d| <= r, with a = (row x'')[0..2] and b = (row w)[0..2] of the draw,
//   x(v) - x(c) = ((a - x(c) b) . d) / (w(c) + b . d),  so  |x(v) - x(c)| <= |a - x(c) b| r / (w(c) - |b| r)
// (and likewise y), provided w(c) - |b| r > 0; the test requires at least w(c) / 2.  The box
// x(c) +- that bound, widened by the per-draw slack the host derived for the binary32 error of the
// projected centre and of the box arithmetic (DrawDesc::slack), holds every exact window position of
// the strip's vertices up to kFastMargin, so the extent test of the union box applies to it.  The
// radius itself is inflated by 2^-10 in relative terms, which covers the few roundings in r, the
// norms, the reciprocal and the products below.  A rejected strip covers no pixel centre.
// A strip whose union box may hold a pixel centre, waiting for its per-triangle tests: the
// window positions of its N vertices for one draw, the draw and its first triangle.
template <int N>
struct StripEntry {
    float2 w[N];
    uint32_t draw, tri;
    uint32_t even;                // bit k: triangle k's own vertex order is an even permutation of
                                  // strip vertices k, k + 1, k + 2 (same winding)
};

// Provably back-facing from fast window positions p0, p1, p2 (in the strip's vertex order, `even`
// when that order has the triangle's own winding): each fast position is within m = kFastMargin of
// its snapped position, so the snapped signed area differs from the one of the fast positions by at
// most 2m(|a.x| + |a.y| + |b.x| + |b.y|) + 8m^2 (a = p1 - p0, b = p2 - p0); the binary32 evaluation
// adds at most 5u(|a.x b.y| + |a.y b.x|), bounded here by 2^-20 times that sum, and the bound's own
// roundings are covered by the factor 1 + 2^-16.  A negative snapped area is culled in every stage,
// so the triangle covers nothing.  NaN positions (outside the fast range) never pass.
__device__ __forceinline__ bool fast_back_facing(float2 p0, float2 p1, float2 p2, bool even)
{
    const float ax = p1.x - p0.x, ay = p1.y - p0.y, bx = p2.x - p0.x, by = p2.y - p0.y;
    const float P = ax * by, Q = ay * bx;
    const float A = even ? P - Q : Q - P;
    const float m = kFastMargin;
    const float B = (2.0f * m) * ((__builtin_fabsf(ax) + __builtin_fabsf(ay)) + (__builtin_fabsf(bx) + __builtin_fabsf(by))) +
                    8.0f * m * m + (1.0f / 1048576.0f) * (__builtin_fabsf(P) + __builtin_fabsf(Q));
    return A < -(B * (1.0f + 1.0f / 65536.0f));
}

// A (draw, lane) pair of the stage-1 strip path whose sphere test could not reject the strip of
// that lane of the wavefront: it waits in LDS for the union-box and per-triangle tests.
struct StripPair {
    uint32_t draw, lane;
};

// What the sphere test reads of a draw and its view (one record, so one batch of loads per draw).
struct SphereDraw {
    float Rx[4], Ry[4], Aw[4];
    float wnorm, slack, wmax, hmax;
    uint32_t view;
};

__device__ __forceinline__ SphereDraw sphere_draw(const DrawDesc* __restrict__ d_draws, uint32_t d)
{
    const DrawDesc& D = d_draws[d];
    SphereDraw s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        s.Rx[k] = D.R[k];
        s.Ry[k] = D.R[4 + k];
        s.Aw[k] = D.A[8 + k];
    }
    s.wnorm = D.wnorm;
    s.slack = D.slack;
    s.view = D.view;
    s.wmax = D.wmax;
    s.hmax = D.hmax;
    return s;
}

__device__ __forceinline__ bool sphere_reject(const SphereDraw& D, const float (&c)[3], float r, bool tiny_cull)
{
    const float* Rx = D.Rx;
    const float* Ry = D.Ry;
    const float* Aw = D.Aw;
    const float w = row_dot(Aw, c[0], c[1], c[2]);
    const float rw = __builtin_amdgcn_rcpf(w);
    const float xc = row_dot(Rx, c[0], c[1], c[2]) * rw;
    const float yc = row_dot(Ry, c[0], c[1], c[2]) * rw;
    const float ex0 = __builtin_fmaf(-xc, Aw[0], Rx[0]), ex1 = __builtin_fmaf(-xc, Aw[1], Rx[1]),
                ex2 = __builtin_fmaf(-xc, Aw[2], Rx[2]);
    const float ey0 = __builtin_fmaf(-yc, Aw[0], Ry[0]), ey1 = __builtin_fmaf(-yc, Aw[1], Ry[1]),
                ey2 = __builtin_fmaf(-yc, Aw[2], Ry[2]);
    const float nx = __builtin_amdgcn_sqrtf(__builtin_fmaf(ex2, ex2, __builtin_fmaf(ex1, ex1, ex0 * ex0)));
    const float ny = __builtin_amdgcn_sqrtf(__builtin_fmaf(ey2, ey2, __builtin_fmaf(ey1, ey1, ey0 * ey0)));
    const float den = __builtin_fmaf(-D.wnorm, r, w);
    const float t = r * __builtin_amdgcn_rcpf(den);
    const float rx = __builtin_fmaf(nx, t, D.slack), ry = __builtin_fmaf(ny, t, D.slack);
    // the extent test of fast_reject_extent on the box xc +- rx, yc +- ry, without branches
    const float lx = (xc - rx) - (kFastMargin + 0.5f);
    const float fx = __builtin_floorf((xc + rx) + (kFastMargin - 0.5f));
    const float ly = (yc - ry) - (kFastMargin + 0.5f);
    const float fy = __builtin_floorf((yc + ry) + (kFastMargin - 0.5f));
    const bool outside = (fx < 0.0f) | (lx > D.wmax) | (fy < 0.0f) | (ly > D.hmax);
    const bool empty = (fx < lx) | (fy < ly);
    return (den >= 0.5f * w) & (outside | (tiny_cull & empty));
}

// Object-space bounding sphere of N points: their mean (a convex combination, so it lies inside
// the mesh's bounding sphere like the points, where the host's per-draw bounds hold) and the largest
// distance to it, inflated by 2^-10 (see sphere_reject).
template <int N>
__device__ __forceinline__ void strip_sphere(const float (&q)[N][3], float (&c)[3], float& r)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float sum = q[0][j];
#pragma unroll
        for (int i = 1; i < N; ++i) sum += q[i][j];
        c[j] = sum * (1.0f / (float)N);
    }
    float r2 = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float d0 = q[i][0] - c[0], d1 = q[i][1] - c[1], d2 = q[i][2] - c[2];
        r2 = fmaxf(r2, __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0)));
    }
    r = __builtin_amdgcn_sqrtf(r2) * (1.0f + 1.0f / 1024.0f);
}

template <int BLOCK, int TPT, bool STRIPS, bool STATS, int CMP, bool SPH>
__global__ void __launch_bounds__(BLOCK) stage1_fast_kernel(RasterArgs a, CURAST_DESC_PARAMS)
{
    static_assert(!STRIPS || TPT == 2 || TPT == 4 || TPT == 8, "strips of 2, 4 or 8 triangles per lane");
    static_assert(STRIPS || !SPH, "strip spheres need strips");
    constexpr int WAVES = BLOCK / 64;
    using Entry = typename std::conditional<STRIPS, IdEntry, ClipEntry>::type;
    constexpr int NV = TPT + 2;   // vertices of a strip
    __shared__ Entry s_ring[WAVES][kRing];
    // Strips that a per-draw test could not reject gather in LDS, 64 at a time, so that their
    // per-triangle tests run with every lane busy instead of on the few failing lanes of a draw.
    // Union-box strips keep their window positions (StripRing).  Sphere strips (SPH) keep (draw,
    // lane) pairs and every lane's strip vertices for the work item, so the lane that drains a pair
    // projects another lane's strip (StripStore).
    struct StripRing {
        StripEntry<NV> e[kRing];
    };
    struct StripStore {
        float q[64][3 * NV];
        StripPair ring[kRing];
    };
    using StripLds =
        typename std::conditional<!STRIPS, char, typename std::conditional<SPH, StripStore, StripRing>::type>::type;
    __shared__ StripLds s_strip[WAVES];
    StripLds& slds = s_strip[threadIdx.x >> 6];
    uint32_t shead = 0, stail = 0;   // wave-uniform (union-box strips)
    const FrameHeader hdr = *d_hdr;
    uint64_t first, total;
    work_range(hdr, a.part, first, total);
    const uint32_t n_segs = uni(hdr.n_segs);
    const uint32_t dpi = uni(hdr.draws_per_item);
    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    const bool tiny_cull = !(a.flags & kFlagNoTinyCull);
    Entry* ring = s_ring[threadIdx.x >> 6];
    uint32_t head = 0, tail = 0;   // wave-uniform
    StatAcc<STATS> st;
    // append (draw d, triangle t) where `need`; fill(e) writes the rest of the entry
    auto push = [&](bool need, uint32_t d, uint32_t t, auto&& fill) __attribute__((always_inline)) {
        const unsigned long long m = __ballot(need);
        if (m) {
            if (need) {
                Entry& e = ring[(tail + rank_in(m)) & (kRing - 1)];
                e.draw = d;
                e.tri = t;
                fill(e);
            }
            tail += (uint32_t)__popcll(m);
            if (tail - head >= 64) {
                wave_lds_sync();
                drain_ring<STATS>(a, d_views, d_meshes, d_draws, ring, head, 64, tiny_cull, early_out, st);
                head += 64;
                wave_lds_sync();
            }
        }
    };
    auto count = [&](bool valid, bool rejected) {
        if (valid) {
            st.add(kStTriDraws);
            if (rejected) st.add(kStCulledTiny);
        }
    };
    // window position of one vertex and the per-triangle test, for interior draws (prescaled rows,
    // no range tests) or general ones (exact transform, range tests, NaN for an undecidable vertex)
    // clip-plane bits for strips in the kernels without strip spheres (the union-box strips, whose
    // launches see general draws of meshes reaching past the view: many views of a large mesh)
    constexpr bool BITS = STRIPS && !SPH;
    auto window = [&](auto interior_tag, const DrawDesc& D, const ViewDesc& V, const float* q) -> float2 {
        if constexpr (decltype(interior_tag)::value) return fast_window_prescaled(D.R, D.A + 8, q[0], q[1], q[2]);
        else return fast_window<BITS>(transform(D.A, q[0], q[1], q[2]), V);
    };
    auto reject = [&](auto interior_tag, float2 x, float2 y, float2 z, const ViewDesc& V) -> bool {
        if constexpr (decltype(interior_tag)::value) return fast_reject_box(x, y, z, V, tiny_cull);
        else return fast_reject(x, y, z, V, tiny_cull);
    };
    // per-triangle tests of n gathered union-box strips, one strip per lane; survivors go to the
    // exact path
    auto drain_strips = [&](uint32_t n) __attribute__((always_inline)) {
        if constexpr (STRIPS && !SPH) {
            const uint32_t lane = threadIdx.x & 63;
            const bool have = lane < n;
            const StripEntry<NV> e = slds.e[(shead + lane) & (kRing - 1)];
            const uint32_t dd = have ? e.draw : 0u;
            const DrawDesc& D = d_draws[dd];
            const ViewDesc V = d_views[D.view & kDrawViewMask];
            const bool interior = (D.view & kDrawInterior) != 0;
            const uint32_t dmesh = D.mesh;
            auto fill_mesh = [&](IdEntry& x) { x.mesh = dmesh; };
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                const bool rej = interior ? fast_reject_box(e.w[k], e.w[k + 1], e.w[k + 2], V, tiny_cull)
                                          : fast_reject(e.w[k], e.w[k + 1], e.w[k + 2], V, tiny_cull);
                const bool back = !rej && fast_back_facing(e.w[k], e.w[k + 1], e.w[k + 2], (e.even >> k) & 1u);
                if (have && rej) st.add(kStCulledTiny);
                if (have && back) st.add(kStCulledBack);
                push(have && !rej && !back, dd, e.tri + (uint32_t)k, fill_mesh);
            }
        }
    };
    // the union-box and per-triangle tests of n gathered (draw, lane) pairs of sphere strips, one per
    // lane: the lane projects the strip of lane `src` of its wavefront for draw `dd` (interior or
    // general); survivors go to the exact path
    auto drain_pairs = [&](uint32_t head, uint32_t n, uint64_t tb, uint32_t mesh_id, uint32_t d_any)
        __attribute__((always_inline)) {
        if constexpr (SPH) {
            const uint32_t lane = threadIdx.x & 63;
            const bool have = lane < n;
            const StripPair e = slds.ring[(head + lane) & (kRing - 1)];
            const uint32_t dd = have ? e.draw : d_any;
            const uint32_t src = have ? e.lane : 0u;
            const DrawDesc& D = d_draws[dd];
            const ViewDesc V = d_views[D.view & kDrawViewMask];
            const bool interior = (D.view & kDrawInterior) != 0;
            float2 w[NV];
            bool any_nan = false;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const float* qq = &slds.q[src][3 * i];
                const float q0 = qq[0], q1 = qq[1], q2 = qq[2];
                w[i] = interior ? fast_window_prescaled(D.R, D.A + 8, q0, q1, q2)
                                : fast_window(transform(D.A, q0, q1, q2), V);
                any_nan |= __builtin_isnan(w[i].x);
            }
            const bool all_out = !any_nan && fast_reject_union<NV>(w, V, tiny_cull);
            if (have) {
                if (all_out) st.add(kStCulledTiny, TPT);
                else st.add(kStStripPass);
            }
            const bool pass = have && !all_out;
            const uint32_t tri0 =
                (uint32_t)(tb * (uint64_t)(BLOCK * TPT) + (uint64_t)(((threadIdx.x & ~63u) + src) * TPT));
            auto fill_mesh = [&](IdEntry& x) { x.mesh = mesh_id; };
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                const bool rej = interior ? fast_reject_box(w[k], w[k + 1], w[k + 2], V, tiny_cull)
                                          : fast_reject(w[k], w[k + 1], w[k + 2], V, tiny_cull);
                if (pass && rej) st.add(kStCulledTiny);
                push(pass && !rej, dd, tri0 + (uint32_t)k, fill_mesh);
            }
        }
    };
    for (uint64_t b = first + blockIdx.x; b < total; b += gridDim.x) {
        const WorkItem wi = locate_work(d_segs, n_segs, dpi, b);
        const uint64_t tb = wi.tri_batch;
        const uint32_t d0 = wi.d0, d1 = wi.d1;
        const MeshDesc mesh = d_meshes[wi.mesh];
        // issue every index load before any use (memory parallelism); with STRIPS lane l owns
        // triangles TPT l .. TPT l + TPT - 1 of the batch, else l + k BLOCK
        uint32_t vi[TPT][3];
        bool valid[TPT];
        uint32_t tri[TPT];
        // compressed indices: the bit offset of the work item's first triangle once per wavefront
        // (64-bit), the lane's triangles relative to it (32-bit); an invalid lane reads the item's
        // first triangle, which exists
        const uint64_t t0 = tb * (uint64_t)(BLOCK * TPT);
        const uint64_t ubit = CMP == 1 ? 3u * t0 * (uint64_t)mesh.idx_bits : 0u;
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const uint32_t j = STRIPS ? threadIdx.x * TPT + k : k * BLOCK + threadIdx.x;
            const uint64_t t = t0 + j;
            tri[k] = (uint32_t)t;
            valid[k] = t < mesh.T;
            if constexpr (CMP == 1)
                packed_triangle_at(mesh, ubit >> 5, (uint32_t)(ubit & 31u) + (valid[k] ? 3u * j * mesh.idx_bits : 0u),
                                   vi[k]);
            else
                mesh_triangle<CMP>(mesh, valid[k] ? t : 0, vi[k]);
        }
#pragma unroll
        for (int k = 0; k < TPT; ++k)
            valid[k] = valid[k] && vi[k][0] < mesh.V && vi[k][1] < mesh.V && vi[k][2] < mesh.V;
        if constexpr (STRIPS) {
            auto fill_id = [&](IdEntry& e) { e.mesh = wi.mesh; };
            // strip mode when every lane with a valid triangle has TPT valid triangles forming a
            // strip: TPT + 2 window positions per draw, and one test of their union box rejects
            // all TPT triangles at once (it holds each triangle's box)
            uint32_t sv[TPT + 2];
            bool all_valid = true, any_valid = false;
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                all_valid &= valid[k];
                any_valid |= valid[k];
            }
            const bool lane_strip = build_strip<TPT>(vi, sv) && all_valid;
            // winding of each strip triangle against its own vertex order (union-box strips)
            uint32_t even = 0;
            if constexpr (!SPH) {
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    const uint32_t a0 = vi[k][0], a1 = vi[k][1];
                    const bool ev = (a0 == sv[k] && a1 == sv[k + 1]) || (a0 == sv[k + 1] && a1 == sv[k + 2]) ||
                                    (a0 == sv[k + 2] && a1 == sv[k]);
                    even |= (uint32_t)ev << k;
                }
            }
            if (__ballot(!any_valid || lane_strip) == __ballot(1)) {
                float q[TPT + 2][3];
#pragma unroll
                for (int i = 0; i < TPT + 2; ++i) {
                    mesh_vertex<CMP>(mesh, any_valid ? sv[i] : 0u, q[i]);
                }
                if constexpr (SPH) {
                    // this lane's strip vertices, for the lane that drains one of its (draw, lane) pairs
                    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
                    for (int i = 0; i < NV; ++i) {
                        slds.q[lane][3 * i] = q[i][0];
                        slds.q[lane][3 * i + 1] = q[i][1];
                        slds.q[lane][3 * i + 2] = q[i][2];
                    }
                    float sc[3], sr;
                    strip_sphere<NV>(q, sc, sr);
                    uint32_t phead = 0, ptail = 0;   // wave-uniform
                    // pairs of draws dbase + j for the set bits j of `bits` go to the ring, a few rounds of
                    // compaction per 32 draws instead of one per draw
                    auto flush = [&](uint32_t bits, uint32_t dbase) __attribute__((always_inline)) {
                        while (__ballot(bits != 0u)) {
                            const bool has = bits != 0u;
                            const uint32_t j = has ? (uint32_t)__builtin_ctz(bits) : 0u;
                            bits &= bits - 1u;
                            const unsigned long long m = __ballot(has);
                            if (has) {
                                StripPair& pe = slds.ring[(ptail + rank_in(m)) & (kRing - 1)];
                                pe.draw = dbase + j;
                                pe.lane = lane;
                            }
                            ptail += (uint32_t)__popcll(m);
                            if (ptail - phead >= 64) {
                                wave_lds_sync();
                                drain_pairs(phead, 64, tb, wi.mesh, d0);
                                phead += 64;
                                wave_lds_sync();
                            }
                        }
                    };
#pragma unroll 1
                    for (uint32_t dc = d0; dc < d1; dc += 32) {
                        const uint32_t dn = min(32u, d1 - dc);
                        uint32_t bits = 0;
#pragma unroll 1
                        for (uint32_t j = 0; j < dn; ++j) {
                            const uint32_t d = dc + j;
                            const DrawDesc& D = d_draws[d];
                            // the view word with the sphere test's fields: one batch of scalar loads per draw
                            const SphereDraw sd = sphere_draw(d_draws, d);
                            bool pass;
                            if (sd.view & kDrawInterior) {
                                // the strip's bounding sphere first (see sphere_reject)
                                pass = any_valid && !sphere_reject(sd, sc, sr, tiny_cull);
                                if (any_valid && pass) st.add(kStSpherePass);
                            } else {
                                const ViewDesc V = d_views[D.view & kDrawViewMask];
                                // the box around the strip's TPT + 2 window positions holds each triangle's box
                                auto body = [&](auto tag) {
                                    constexpr bool INTERIOR = decltype(tag)::value;
                                    float2 w[NV];
                                    bool any_nan = false;
#pragma unroll
                                    for (int i = 0; i < NV; ++i) {
                                        w[i] = window(tag, D, V, q[i]);
                                        if constexpr (!INTERIOR) any_nan |= __builtin_isnan(w[i].x);
                                    }
                                    return !any_nan && fast_reject_union<NV>(w, V, tiny_cull);
                                };
                                const bool all_out =
                                    (D.view & kDrawInterior) ? body(std::true_type{}) : body(std::false_type{});
                                pass = any_valid && !all_out;
                            }
                            if (any_valid) {
                                st.add(kStTriDraws, TPT);
                                st.add(kStStripDraws);
                                if (!pass) st.add(kStCulledTiny, TPT);
                            }
                            bits |= (uint32_t)pass << j;
                        }
                        flush(bits, dc);
                    }
                    wave_lds_sync();
                    if (ptail != phead) drain_pairs(phead, ptail - phead, tb, wi.mesh, d0);
                    wave_lds_sync();
                } else {
#pragma unroll 1
                    for (uint32_t d = d0; d < d1; ++d) {
                        const DrawDesc& D = d_draws[d];
                        const ViewDesc V = d_views[D.view & kDrawViewMask];
                        auto body = [&](auto tag) {
                            constexpr bool INTERIOR = decltype(tag)::value;
                            float2 w[TPT + 2];
                            bool any_nan = false;
#pragma unroll
                            for (int i = 0; i < TPT + 2; ++i) {
                                w[i] = window(tag, D, V, q[i]);
                                if constexpr (!INTERIOR) any_nan |= __builtin_isnan(w[i].x);
                            }
                            const bool all_out = fast_reject_strip<TPT + 2, BITS>(w, any_nan, V, tiny_cull);
                            if (any_valid) {
                                st.add(kStTriDraws, TPT);
                                st.add(kStStripDraws);
                                if (all_out) st.add(kStCulledTiny, TPT);
                                else st.add(kStStripPass);
                            }
                            const bool pass = any_valid && !all_out;
                            const unsigned long long m = __ballot(pass);
                            if (m) {
                                if (pass) {
                                    StripEntry<TPT + 2>& se = slds.e[(stail + rank_in(m)) & (kRing - 1)];
#pragma unroll
                                    for (int i = 0; i < TPT + 2; ++i) se.w[i] = w[i];
                                    se.draw = d;
                                    se.tri = tri[0];
                                    se.even = even;
                                }
                                stail += (uint32_t)__popcll(m);
                                if (stail - shead >= 64) {
                                    wave_lds_sync();
                                    drain_strips(64);
                                    shead += 64;
                                    wave_lds_sync();
                                }
                            }
                        };
                        if (D.view & kDrawInterior) body(std::true_type{});
                        else body(std::false_type{});
                    }
                }
                continue;
            }
            // not a strip everywhere: one triangle at a time over all draws (its index, validity
            // and id picked by value, so the per-lane arrays stay in registers)
#pragma unroll 1
            for (int k = 0; k < TPT; ++k) {
                uint32_t i3[3] = {vi[0][0], vi[0][1], vi[0][2]};
                bool vk = valid[0];
                uint32_t tk = tri[0];
#pragma unroll
                for (int j = 1; j < TPT; ++j) {
                    const uint32_t a0 = vi[j][0], a1 = vi[j][1], a2 = vi[j][2], tj = tri[j];
                    const bool vj = valid[j];
                    i3[0] = k == j ? a0 : i3[0];
                    i3[1] = k == j ? a1 : i3[1];
                    i3[2] = k == j ? a2 : i3[2];
                    vk = k == j ? vj : vk;
                    tk = k == j ? tj : tk;
                }
                float p[9];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    float src[3];
                    mesh_vertex<CMP>(mesh, vk ? i3[v] : 0u, src);
                    p[3 * v + 0] = src[0];
                    p[3 * v + 1] = src[1];
                    p[3 * v + 2] = src[2];
                }
#pragma unroll 1
                for (uint32_t d = d0; d < d1; ++d) {
                    const DrawDesc& D = d_draws[d];
                    const ViewDesc V = d_views[D.view & kDrawViewMask];
                    auto body = [&](auto tag) {
                        const bool rej = reject(tag, window(tag, D, V, p), window(tag, D, V, p + 3),
                                                window(tag, D, V, p + 6), V);
                        count(vk, rej);
                        push(vk && !rej, d, tk, fill_id);
                    };
                    if (D.view & kDrawInterior) body(std::true_type{});
                    else body(std::false_type{});
                }
            }
        } else {
            float p[TPT][9];
#pragma unroll
            for (int k = 0; k < TPT; ++k)
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    float src[3];
                    mesh_vertex<CMP>(mesh, valid[k] ? vi[k][v] : 0u, src);
                    p[k][3 * v + 0] = src[0];
                    p[k][3 * v + 1] = src[1];
                    p[k][3 * v + 2] = src[2];
                }
#pragma unroll 1
            for (uint32_t d = d0; d < d1; ++d) {
                const DrawDesc& D = d_draws[d];
                const ViewDesc V = d_views[D.view & kDrawViewMask];
                auto body = [&](auto tag) {
                    constexpr bool INTERIOR = decltype(tag)::value;
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        // the exact clip coordinates go into the ring: general draws have them
                        // from the window computation, interior ones compute them when pushing
                        Clip c[3];
                        float2 w[3];
#pragma unroll
                        for (int v = 0; v < 3; ++v) {
                            if constexpr (INTERIOR) {
                                w[v] = window(tag, D, V, p[k] + 3 * v);
                            } else {
                                c[v] = transform(D.A, p[k][3 * v], p[k][3 * v + 1], p[k][3 * v + 2]);
                                w[v] = fast_window(c[v], V);
                            }
                        }
                        const bool rej = reject(tag, w[0], w[1], w[2], V);
                        count(valid[k], rej);
                        push(valid[k] && !rej, d, tri[k], [&](ClipEntry& e) {
#pragma unroll
                            for (int v = 0; v < 3; ++v) {
                                const Clip cv = INTERIOR ? transform(D.A, p[k][3 * v], p[k][3 * v + 1], p[k][3 * v + 2])
                                                         : c[v];
                                e.c[3 * v] = cv.x;
                                e.c[3 * v + 1] = cv.y;
                                e.c[3 * v + 2] = cv.w;
                            }
                        });
                    }
                };
                if (D.view & kDrawInterior) body(std::true_type{});
                else body(std::false_type{});
            }
        }
    }
    if constexpr (STRIPS && !SPH) {
        if (stail != shead) {
            wave_lds_sync();
            drain_strips(stail - shead);
            shead = stail;
        }
    }
    if (tail != head) {
        wave_lds_sync();
        drain_ring<STATS>(a, d_views, d_meshes, d_draws, ring, head, tail - head, tiny_cull, early_out, st);
    }
    st.flush(a.stats);
}

// ----------------------------------------------------------------------------------------------
// Stage 1 with vertex sharing, for triangles drawn many times (instances x views).  One wavefront
// per workgroup: it deduplicates the vertex indices of its 64*TPT triangles in an LDS hash table
// once per work item, then for every draw transforms each unique vertex once (window positions in
// LDS) and tests each triangle from those.  The arithmetic of the fast test is the same as in
// stage1_fast_kernel; undecided (triangle, draw) pairs go through the exact path after reloading
// the triangle (rare for dense meshes).  Vertex reuse through shared memory is named as future
// work in the paper's conclusion.
// ----------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t vertex_hash(uint32_t v, int bits) { return (v * 2654435761u) >> (32 - bits); }

template <int TPT, bool STATS>
__global__ void __launch_bounds__(64) stage1_share_kernel(RasterArgs a, CURAST_DESC_PARAMS)
{
    constexpr int NT = 64 * TPT;                       // triangles per work item
    constexpr int NI = 3 * NT;                         // vertex references
    constexpr int RS = 3 * TPT;                        // rounds of 64 unique vertices at most
    constexpr int HBITS = TPT == 1 ? 8 : TPT == 2 ? 9 : 10;
    constexpr int HT = 1 << HBITS;                     // load factor <= 3/4
    constexpr uint32_t kFree = 0xFFFFFFFFu;
    __shared__ uint32_t s_key[HT];
    __shared__ uint16_t s_val[HT];
    __shared__ uint32_t s_uniq[NI];
    __shared__ float2 s_win[NI];
    __shared__ IdEntry s_ring[kRing];
    __shared__ uint32_t s_nu;
    const FrameHeader hdr = *d_hdr;
    uint64_t first, total;
    work_range(hdr, a.part, first, total);
    const uint32_t n_segs = uni(hdr.n_segs);
    const uint32_t dpi = uni(hdr.draws_per_item);
    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    const bool tiny_cull = !(a.flags & kFlagNoTinyCull);
    const uint32_t lane = threadIdx.x;
    uint32_t head = 0, tail = 0;
    StatAcc<STATS> st;
    for (uint64_t b = first + blockIdx.x; b < total; b += gridDim.x) {
        const WorkItem wi = locate_work(d_segs, n_segs, dpi, b);
        const uint64_t tb = wi.tri_batch;
        const uint32_t d0 = wi.d0, d1 = wi.d1;
        const MeshDesc mesh = d_meshes[wi.mesh];
        uint32_t vi[TPT][3], dv[TPT][3], tri[TPT];
        bool valid[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const uint64_t t = tb * (uint64_t)NT + (uint64_t)(k * 64) + lane;
            tri[k] = (uint32_t)t;
            valid[k] = t < mesh.T;
            mesh_triangle(mesh, valid[k] ? t : 0, vi[k]);
        }
        for (int i = lane; i < HT; i += 64) s_key[i] = kFree;
        if (lane == 0) s_nu = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            valid[k] = valid[k] && vi[k][0] < mesh.V && vi[k][1] < mesh.V && vi[k][2] < mesh.V;
            if (!valid[k]) continue;
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                uint32_t h = vertex_hash(vi[k][v], HBITS);
                while (true) {
                    const uint32_t prev = atomicCAS(&s_key[h], kFree, vi[k][v]);
                    if (prev == kFree) {
                        const uint32_t dn = atomicAdd(&s_nu, 1u);
                        s_val[h] = (uint16_t)dn;
                        s_uniq[dn] = vi[k][v];
                        break;
                    }
                    if (prev == vi[k][v]) break;
                    h = (h + 1) & (HT - 1);
                }
            }
        }
        __syncthreads();
        const uint32_t nu = uni(s_nu);
#pragma unroll
        for (int k = 0; k < TPT; ++k)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                dv[k][v] = 0;
                if (valid[k]) {
                    uint32_t h = vertex_hash(vi[k][v], HBITS);
                    while (s_key[h] != vi[k][v]) h = (h + 1) & (HT - 1);
                    dv[k][v] = s_val[h];
                }
            }
        float pu[RS][3];
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const uint32_t u = lane + 64 * r;
            mesh_vertex(mesh, u < nu ? s_uniq[u] : 0u, pu[r]);
        }
#pragma unroll 1
        for (uint32_t d = d0; d < d1; ++d) {
            const DrawDesc D = d_draws[d];
            const ViewDesc V = d_views[D.view & kDrawViewMask];
            const bool interior = (D.view & kDrawInterior) != 0;
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                if (64 * r >= (int)nu) break;                // uniform
                const uint32_t u = lane + 64 * r;
                const Clip c = transform(D.A, pu[r][0], pu[r][1], pu[r][2]);
                const float2 w = interior ? fast_window_interior(c, V) : fast_window(c, V);
                if (u < nu) s_win[u] = w;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                bool need = false;
                if (valid[k]) {
                    st.add(kStTriDraws);
                    need = !fast_reject(s_win[dv[k][0]], s_win[dv[k][1]], s_win[dv[k][2]], V, tiny_cull);
                    if (!need) st.add(kStCulledTiny);
                }
                const unsigned long long m = __ballot(need);
                if (m) {
                    if (need) {
                        IdEntry& e = s_ring[(tail + rank_in(m)) & (kRing - 1)];
                        e.draw = d;
                        e.tri = tri[k];
                        e.mesh = wi.mesh;
                    }
                    tail += (uint32_t)__popcll(m);
                    if (tail - head >= 64) {
                        __syncthreads();
                        drain_ring<STATS>(a, d_views, d_meshes, d_draws, s_ring, head, 64, tiny_cull, early_out, st);
                        head += 64;
                        __syncthreads();
                    }
                }
            }
            __syncthreads();
        }
    }
    if (tail != head) {
        __syncthreads();
        drain_ring<STATS>(a, d_views, d_meshes, d_draws, s_ring, head, tail - head, tiny_cull, early_out, st);
    }
    st.flush(a.stats);
}

// Stage-1 overflow pass: when more triangles were forwarded than Q2 holds, every forwarded
// triangle is rasterized here by one thread (those that did fit are drawn twice; the minimum is
// idempotent).  Exits at once when nothing overflowed.
__global__ void __launch_bounds__(256) stage1_overflow_kernel(RasterArgs a, CURAST_DESC_PARAMS)
{
    if (a.counters[kCntQ2] <= a.q2_cap) return;
    const FrameHeader hdr = *d_hdr;
    uint64_t first, total;
    work_range(hdr, a.part, first, total);
    const uint32_t n_segs = uni(hdr.n_segs);
    const uint32_t dpi = uni(hdr.draws_per_item);

    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    const bool tiny_cull = !(a.flags & kFlagNoTinyCull);
    StatAcc<false> st;
    for (uint64_t b = first + blockIdx.x; b < total; b += gridDim.x) {
        const WorkItem wi = locate_work(d_segs, n_segs, dpi, b);
        const uint64_t tb = wi.tri_batch;
        const uint32_t d0 = wi.d0, d1 = wi.d1;
        const MeshDesc mesh = d_meshes[wi.mesh];
        const uint32_t bt = wi.batch_tris;
        for (uint32_t tt = threadIdx.x; tt < bt; tt += blockDim.x) {
            const uint64_t t = tb * bt + tt;
            if (t >= mesh.T) break;
            uint32_t iv[3];
            mesh_triangle(mesh, t, iv);
            if (iv[0] >= mesh.V || iv[1] >= mesh.V || iv[2] >= mesh.V) continue;
            float p[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) mesh_vertex(mesh, iv[k], p[k]);
            for (uint32_t d = d0; d < d1; ++d) {
                const DrawDesc D = d_draws[d];
                const ViewDesc V = d_views[D.view & kDrawViewMask];
                const Clip c[3] = {transform(D.A, p[0][0], p[0][1], p[0][2]), transform(D.A, p[1][0], p[1][1], p[1][2]),
                                   transform(D.A, p[2][0], p[2][1], p[2][2])};
                SmallTri s;
                if (classify<false>(c, V, a.small_px, tiny_cull, s, st) == kRouteForward)
                    raster_any_thread(c, D.id_base + t, V, early_out);
            }
        }
    }
}

// ----------------------------------------------------------------------------------------------
// One wavefront rasterizes a general triangle over its clamped box, visiting only blocks of 64
// pixels that can hold a covered pixel centre.  The box is cut into blocks as square as its
// shape allows (8 x 8, or 1/2/4 wide for narrow boxes, 1/2/4 high for flat ones).  First every
// lane tests one block: an edge function is affine, so its maximum over the block's pixel
// centres sits at one corner (the left or right column as the edge's dy is positive or not, the
// top or bottom row as its dx is positive or not); a block whose maximum E_k + bias_k is
// negative for some edge holds no covered centre.  The test is exact (int64), so skipping such
// blocks changes nothing.  Then the wave visits the remaining blocks one by one, one pixel per
// lane, with the usual per-pixel test.
// ----------------------------------------------------------------------------------------------
template <class Stats>
__device__ __forceinline__ void raster_wave_blocks(const Tri64& t, uint64_t id, unsigned long long* vis, int32_t W,
                                                   bool early_out, uint32_t lane, Stats& st)
{
    const uint32_t bw = (uint32_t)(t.px1 - t.px0 + 1), bh = (uint32_t)(t.py1 - t.py0 + 1);
    uint32_t lbw;   // log2 of the block width; the block is 64 pixels
    if (bw >= 8 && bh >= 8) lbw = 3;
    else if (bw < 8) lbw = bw <= 1 ? 0 : bw <= 2 ? 1 : bw <= 4 ? 2 : 3;
    else lbw = bh <= 1 ? 6 : bh <= 2 ? 5 : bh <= 4 ? 4 : 3;
    const uint32_t BW = 1u << lbw, lbh = 6 - lbw;
    const uint32_t nbx = (bw + BW - 1) >> lbw, nby = (bh + (1u << lbh) - 1) >> lbh;
    const uint32_t nblocks = nbx * nby;
    for (uint32_t base = 0; base < nblocks; base += 64) {
        const uint32_t j = base + lane;
        bool cand = false;
        if (j < nblocks) {
            const uint32_t by = j / nbx, bx = j - by * nbx;
            const int32_t x0 = t.px0 + (int32_t)(bx << lbw), y0 = t.py0 + (int32_t)(by << lbh);
            const int32_t x1 = min(x0 + (int32_t)BW - 1, t.px1), y1 = min(y0 + (1 << lbh) - 1, t.py1);
            cand = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int32_t cx = t.dy[k] > 0 ? x0 : x1;
                const int32_t cy = t.dx[k] > 0 ? y1 : y0;
                cand = cand && edge64(t, k, cx, cy) + t.bias[k] >= 0;
            }
        }
        unsigned long long mask = __ballot(cand);
        while (mask) {
            const uint32_t jb = base + (uint32_t)__builtin_ctzll(mask);
            mask &= mask - 1;
            const uint32_t by = jb / nbx, bx = jb - by * nbx;
            const int32_t px = t.px0 + (int32_t)((bx << lbw) + (lane & (BW - 1)));
            const int32_t py = t.py0 + (int32_t)((by << lbh) + (lane >> lbw));
            if (px <= t.px1 && py <= t.py1 && raster_pixel64(t, px, py, id, vis, W, early_out)) st.add(kStFragments);
        }
    }
}

// ----------------------------------------------------------------------------------------------
// Stage 2: the wavefront rasterizes forwarded triangles one at a time (Sec. 4.2), after setting up
// 64 of them in parallel
// ----------------------------------------------------------------------------------------------
// Snapped polygon of one forwarded triangle (3 vertices, or up to 8 after clipping), in LDS.
struct S2Poly {
    int32_t X[8], Y[8];
    float zI[8];
    uint64_t id;
    uint32_t np, view;
};

template <bool STATS>
__global__ void __launch_bounds__(256) stage2_kernel(RasterArgs a)
{
    // Each wavefront takes 64 queue entries at a time.  Every lane sets up one of them (descriptor,
    // index and vertex loads, transform, clip, snap: 64 dependent load chains in flight at once)
    // and leaves the snapped polygon in LDS; then the whole wavefront rasterizes the 64 polygons
    // one after the other.
    __shared__ S2Poly s_poly[4][64];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wslot = threadIdx.x >> 6;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const unsigned long long n = min(a.counters[kCntQ2], (unsigned long long)a.q2_cap);
    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    StatAcc<STATS> st;
    for (unsigned long long base = (unsigned long long)wave * 64; base < n; base += (unsigned long long)nwaves * 64) {
        S2Poly& mine = s_poly[wslot][lane];
        const unsigned long long e = base + lane;
        uint32_t np = 0;
        if (e < n) {
            const Q2Entry q = a.q2[e];
            const DrawDesc& D = a.draws[q.draw];
            const uint32_t view = D.view & kDrawViewMask;
            const ViewDesc& V = a.views[view];
            const MeshDesc& M = a.meshes[D.mesh];
            Clip c[3];
            uint32_t iv[3];
            mesh_triangle(M, q.tri, iv);
            for (int k = 0; k < 3; ++k) {
                float qv[3];
                mesh_vertex(M, iv[k], qv);
                c[k] = transform(D.A, qv[0], qv[1], qv[2]);
            }
            const float hW = V.hW, hH = V.hH;
            if (outside_guard(c[0], V.near_plane) || outside_guard(c[1], V.near_plane) ||
                outside_guard(c[2], V.near_plane)) {
                Clip poly[8];
                np = (uint32_t)clip_triangle(c, V.near_plane, poly);
                for (uint32_t k = 0; k < np; ++k) snap_vertex(poly[k], hW, hH, mine.X[k], mine.Y[k], mine.zI[k]);
            } else {
                np = 3;
                for (int k = 0; k < 3; ++k) snap_vertex(c[k], hW, hH, mine.X[k], mine.Y[k], mine.zI[k]);
            }
            mine.id = D.id_base + q.tri;
            mine.view = view;
        }
        mine.np = np;
        wave_lds_sync();
        for (uint32_t l = 0; l < 64; ++l) {
            const S2Poly& P = s_poly[wslot][l];
            const uint32_t npl = __builtin_amdgcn_readfirstlane(P.np);
            if (npl < 3) continue;
            const uint32_t view = __builtin_amdgcn_readfirstlane(P.view);
            const ViewDesc V = a.views[view];
            const uint64_t id = P.id;
            for (uint32_t j = 1; j + 1 < npl; ++j) {
                const int32_t tx[3] = {P.X[0], P.X[j], P.X[j + 1]}, ty[3] = {P.Y[0], P.Y[j], P.Y[j + 1]};
                const float tz[3] = {P.zI[0], P.zI[j], P.zI[j + 1]};
                Tri64 tri;
                if (!setup_tri64(tx, ty, tz, V.W, V.H, tri)) continue;
                const uint32_t bw = (uint32_t)(tri.px1 - tri.px0 + 1);
                const uint64_t cnt = (uint64_t)bw * (uint64_t)(tri.py1 - tri.py0 + 1);
                bool in_place = cnt <= a.medium_px;
                if (!in_place) {
                    const uint32_t tx0 = tri.px0 / kTileSize, tx1 = tri.px1 / kTileSize;
                    const uint32_t ty0 = tri.py0 / kTileSize, ty1 = tri.py1 / kTileSize;
                    const uint32_t ntx = tx1 - tx0 + 1;
                    const uint64_t ntiles = (uint64_t)ntx * (uint64_t)(ty1 - ty0 + 1);
                    unsigned long long rec = 0, qbase = 0;
                    if (lane == 0) {
                        rec = atomicAdd(a.counters + kCntLarge, 1ull);
                        qbase = atomicAdd(a.counters + kCntQ3, (unsigned long long)ntiles);
                    }
                    rec = __shfl(rec, 0);
                    qbase = __shfl(qbase, 0);
                    const bool ok = rec < a.large_cap && qbase + ntiles <= a.q3_cap;
                    if (ok) {
                        if (lane == 0) {
                            LargeTri r;
                            for (int k = 0; k < 3; ++k) {
                                r.X[k] = tx[k];
                                r.Y[k] = ty[k];
                                r.zI[k] = tz[k];
                            }
                            r.view = view;
                            r.id = id;
                            a.large[rec] = r;
                        }
                        const uint32_t view_ntx = (uint32_t)(V.W + kTileSize - 1) / kTileSize;
                        for (uint64_t i = lane; i < ntiles; i += 64) {
                            Q3Entry qe;
                            qe.rec = (uint32_t)rec;
                            qe.tx = (uint16_t)(tx0 + (uint32_t)(i % ntx));
                            qe.ty = (uint16_t)(ty0 + (uint32_t)(i / ntx));
                            a.q3[qbase + i] = qe;
                            atomicAdd(a.tile_count + V.tile_base + (uint32_t)qe.ty * view_ntx + qe.tx, 1u);
                        }
                        if (lane == 0) st.add(kStQ3, (uint32_t)ntiles);
                    } else {
                        // the reserved range may start inside the queue: mark those slots empty
                        for (uint64_t i = lane; i < ntiles && qbase + i < a.q3_cap; i += 64) {
                            Q3Entry qe;
                            qe.rec = kNullRecord;
                            qe.tx = 0;
                            qe.ty = 0;
                            a.q3[qbase + i] = qe;
                        }
                        if (lane == 0) st.add(kStQ3Overflow);
                        in_place = true;
                    }
                }
                if (in_place) {
                    if (lane == 0) st.add(kStS2Raster);
                    raster_wave_blocks(tri, id, V.vis, V.W, early_out, lane, st);
                }
            }
        }
        wave_lds_sync();   // the polygons are read by every lane before the next round overwrites them
    }
    st.flush(a.stats);
}

// ----------------------------------------------------------------------------------------------
// Stage 3: one workgroup of 256 lanes per 64x64 tile part (Sec. 4.3); lane l covers column l % 64
// and every fourth row from l / 64.
// ----------------------------------------------------------------------------------------------
template <bool STATS>
__global__ void __launch_bounds__(256) stage3_kernel(RasterArgs a)
{
    const unsigned long long n = min(a.counters[kCntQ3], (unsigned long long)a.q3_cap);
    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    const int32_t col = threadIdx.x & 63;
    const int32_t row0 = threadIdx.x >> 6;
    StatAcc<STATS> st;
    for (unsigned long long e = blockIdx.x; e < n; e += gridDim.x) {
        const Q3Entry q = a.q3[e];
        if (q.rec == kNullRecord) continue;
        const LargeTri r = a.large[q.rec];
        const ViewDesc V = a.views[r.view];
        Tri64 tri;
        if (!setup_tri64(r.X, r.Y, r.zI, V.W, V.H, tri)) continue;
        const int32_t px = (int32_t)q.tx * kTileSize + col;
        const int32_t y0 = max(tri.py0, (int32_t)q.ty * kTileSize);
        const int32_t y1 = min(tri.py1, (int32_t)q.ty * kTileSize + kTileSize - 1);
        if (px < tri.px0 || px > tri.px1) continue;
        int32_t py = (int32_t)q.ty * kTileSize + row0;
        while (py < y0) py += 4;
        for (; py <= y1; py += 4)
            if (raster_pixel64(tri, px, py, r.id, V.vis, V.W, early_out)) st.add(kStFragments);
    }
    st.flush(a.stats);
}

// ----------------------------------------------------------------------------------------------
// Stage 3 binned by screen tile.  The parts stage 2 produced are grouped by 64x64 tile (count,
// scan, scatter); then one workgroup per non-empty tile walks all parts of its bin.  Lane l owns
// the 16 pixels (l % 64, l / 64 + 4k) of the tile and keeps their running minimum keys in
// registers, so the parts of one tile need no atomics at all and the tile costs one global 64-bit
// atomic minimum per covered pixel however many large triangles overlap it.
// ----------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) tile_scan_kernel(RasterArgs a)
{
    __shared__ uint32_t s_part[1024];
    __shared__ uint32_t s_carry;
    const uint32_t n = a.hdr->n_tiles;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < n ? a.tile_count[i] : 0u;
        s_part[threadIdx.x] = v;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {           // inclusive Hillis-Steele scan
            const uint32_t add = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0u;
            __syncthreads();
            s_part[threadIdx.x] += add;
            __syncthreads();
        }
        const uint32_t carry = s_carry;
        if (i < n) a.tile_offset[i] = carry + s_part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = carry + s_part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.tile_offset[n] = s_carry;
}

__global__ void __launch_bounds__(256) tile_scatter_kernel(RasterArgs a, const ViewDesc* __restrict__ d_views)
{
    const unsigned long long n = min(a.counters[kCntQ3], (unsigned long long)a.q3_cap);
    for (unsigned long long e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const Q3Entry q = a.q3[e];
        if (q.rec == kNullRecord) continue;
        const ViewDesc& V = d_views[a.large[q.rec].view];
        const uint32_t t = V.tile_base + (uint32_t)q.ty * ((uint32_t)(V.W + kTileSize - 1) / kTileSize) + q.tx;
        const uint32_t left = atomicSub(a.tile_count + t, 1u);    // left..1: a distinct slot per part
        a.q3_binned[a.tile_offset[t] + left - 1] = q.rec;
    }
}

template <bool STATS>
__global__ void __launch_bounds__(256) stage3_tile_kernel(RasterArgs a, const ViewDesc* __restrict__ d_views)
{
    const uint32_t n_tiles = a.hdr->n_tiles;
    const uint32_t nv = a.hdr->n_views;
    const bool early_out = !(a.flags & kFlagNoEarlyOut);
    const int32_t col = threadIdx.x & 63;
    const int32_t row0 = threadIdx.x >> 6;
    StatAcc<STATS> st;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint32_t begin = a.tile_offset[t], end = a.tile_offset[t + 1];
        if (begin == end) continue;
        // the view that owns tile t (views are few: linear scan of their tile bases)
        uint32_t v = 0;
        while (v + 1 < nv && d_views[v + 1].tile_base <= t) ++v;
        const ViewDesc V = d_views[v];
        const uint32_t ntx = (uint32_t)(V.W + kTileSize - 1) / kTileSize;
        const uint32_t local = t - V.tile_base;
        const int32_t px = (int32_t)(local % ntx) * kTileSize + col;
        const int32_t py0 = (int32_t)(local / ntx) * kTileSize + row0;
        unsigned long long best[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) best[k] = kEmptyKey;
        for (uint32_t j = begin; j < end; ++j) {
            const LargeTri r = a.large[a.q3_binned[j]];
            Tri64 tri;
            if (!setup_tri64(r.X, r.Y, r.zI, V.W, V.H, tri)) continue;
            if (px < tri.px0 || px > tri.px1) continue;
            // edge values at (px, py0), stepped by four rows
            int64_t e[3];
            const int64_t step[3] = {(int64_t)tri.dx[0] * 1024, (int64_t)tri.dx[1] * 1024, (int64_t)tri.dx[2] * 1024};
#pragma unroll
            for (int k = 0; k < 3; ++k) e[k] = edge64(tri, k, px, py0);
            const float area_f = (float)tri.area;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int32_t py = py0 + 4 * k;
                if (py >= tri.py0 && py <= tri.py1 &&
                    ((e[0] + tri.bias[0]) | (e[1] + tri.bias[1]) | (e[2] + tri.bias[2])) >= 0) {
                    const float depth = frag_depth((float)e[0], (float)e[1], (float)e[2], tri.zI, area_f);
                    const unsigned long long key = make_key(depth, r.id);
                    best[k] = key < best[k] ? key : best[k];
                    st.add(kStFragments);
                }
                e[0] += step[0];
                e[1] += step[1];
                e[2] += step[2];
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int32_t py = py0 + 4 * k;
            if (best[k] != kEmptyKey && px < V.W && py < V.H)
                write_fragment(V.vis + (size_t)py * (size_t)V.W + (size_t)px, best[k], early_out);
        }
    }
    st.flush(a.stats);
}

// ----------------------------------------------------------------------------------------------
// Launch wrappers
// ----------------------------------------------------------------------------------------------
hipError_t launch_clear(const RasterArgs& a, uint32_t grid, hipStream_t s)
{
    clear_kernel<<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int BLOCK, int TPT>
static hipError_t stage1_dispatch(const RasterArgs& a, bool stats, uint32_t grid, hipStream_t s)
{
    if (stats) stage1_kernel<BLOCK, TPT, true><<<grid, BLOCK, 0, s>>>(a, CURAST_DESC_ARGS(a));
    else stage1_kernel<BLOCK, TPT, false><<<grid, BLOCK, 0, s>>>(a, CURAST_DESC_ARGS(a));
    return hipGetLastError();
}

template <int BLOCK>
static hipError_t stage1_tpt(const RasterArgs& a, uint32_t tpt, bool stats, uint32_t grid, hipStream_t s)
{
    switch (tpt) {
    case 1: return stage1_dispatch<BLOCK, 1>(a, stats, grid, s);
    case 2: return stage1_dispatch<BLOCK, 2>(a, stats, grid, s);
    case 4: return stage1_dispatch<BLOCK, 4>(a, stats, grid, s);
    case 8: return stage1_dispatch<BLOCK, 8>(a, stats, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage1(const RasterArgs& a, uint32_t block, uint32_t tpt, bool stats, uint32_t grid, hipStream_t s)
{
    switch (block) {
    case 64: return stage1_tpt<64>(a, tpt, stats, grid, s);
    case 128: return stage1_tpt<128>(a, tpt, stats, grid, s);
    case 256: return stage1_tpt<256>(a, tpt, stats, grid, s);
    case 512: return stage1_tpt<512>(a, tpt, stats, grid, s);
    default: return hipErrorInvalidValue;
    }
}

// Launches whose meshes are all plain or all compressed use a kernel without the per-mesh
// compression branch (Sec. 4.6 notes the same for its kernels); mixed launches decide per mesh.
template <int BLOCK, int TPT, bool STRIPS, bool SPH>
static hipError_t stage1_fast_dispatch(const RasterArgs& a, bool stats, uint32_t grid, hipStream_t s)
{
    // the statistics variants (a measurement aid) decide per mesh, which is right for any launch
    const bool any = (a.compressed_parts >> a.part) & 1u, all = (a.compressed_parts >> (a.part + 8)) & 1u;
    if (stats) stage1_fast_kernel<BLOCK, TPT, STRIPS, true, -1, SPH><<<grid, BLOCK, 0, s>>>(a, CURAST_DESC_ARGS(a));
    else if (all) stage1_fast_kernel<BLOCK, TPT, STRIPS, false, 1, SPH><<<grid, BLOCK, 0, s>>>(a, CURAST_DESC_ARGS(a));
    else if (any) stage1_fast_kernel<BLOCK, TPT, STRIPS, false, -1, SPH><<<grid, BLOCK, 0, s>>>(a, CURAST_DESC_ARGS(a));
    else stage1_fast_kernel<BLOCK, TPT, STRIPS, false, 0, SPH><<<grid, BLOCK, 0, s>>>(a, CURAST_DESC_ARGS(a));
    return hipGetLastError();
}

template <int BLOCK, int TPT>
static hipError_t stage1_fast_strips(const RasterArgs& a, bool strips, bool spheres, bool stats, uint32_t grid,
                                     hipStream_t s)
{
    if (!strips) return stage1_fast_dispatch<BLOCK, TPT, false, false>(a, stats, grid, s);
    return spheres ? stage1_fast_dispatch<BLOCK, TPT, true, true>(a, stats, grid, s)
                   : stage1_fast_dispatch<BLOCK, TPT, true, false>(a, stats, grid, s);
}

template <int BLOCK>
static hipError_t stage1_fast_tpt(const RasterArgs& a, uint32_t tpt, bool strips, bool spheres, bool stats,
                                  uint32_t grid, hipStream_t s)
{
    switch (tpt) {
    case 1: return stage1_fast_dispatch<BLOCK, 1, false, false>(a, stats, grid, s);
    case 2: return stage1_fast_strips<BLOCK, 2>(a, strips, spheres, stats, grid, s);
    case 4: return stage1_fast_strips<BLOCK, 4>(a, strips, spheres, stats, grid, s);
    case 8: return stage1_fast_strips<BLOCK, 8>(a, strips, spheres, stats, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage1_fast(const RasterArgs& a, uint32_t block, uint32_t tpt, bool strips, bool spheres, bool stats,
                              uint32_t grid, hipStream_t s)
{
    switch (block) {
    case 64: return stage1_fast_tpt<64>(a, tpt, strips, spheres, stats, grid, s);
    case 128: return stage1_fast_tpt<128>(a, tpt, strips, spheres, stats, grid, s);
    case 256: return stage1_fast_tpt<256>(a, tpt, strips, spheres, stats, grid, s);
    case 512: return stage1_fast_tpt<512>(a, tpt, strips, spheres, stats, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int TPT>
static hipError_t stage1_share_dispatch(const RasterArgs& a, bool stats, uint32_t grid, hipStream_t s)
{
    if (stats) stage1_share_kernel<TPT, true><<<grid, 64, 0, s>>>(a, CURAST_DESC_ARGS(a));
    else stage1_share_kernel<TPT, false><<<grid, 64, 0, s>>>(a, CURAST_DESC_ARGS(a));
    return hipGetLastError();
}

hipError_t launch_stage1_share(const RasterArgs& a, uint32_t tpt, bool stats, uint32_t grid, hipStream_t s)
{
    switch (tpt) {
    case 1: return stage1_share_dispatch<1>(a, stats, grid, s);
    case 2: return stage1_share_dispatch<2>(a, stats, grid, s);
    case 4: return stage1_share_dispatch<4>(a, stats, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage1_overflow(const RasterArgs& a, uint32_t grid, hipStream_t s)
{
    stage1_overflow_kernel<<<grid, 256, 0, s>>>(a, CURAST_DESC_ARGS(a));
    return hipGetLastError();
}

hipError_t launch_stage2(const RasterArgs& a, uint32_t grid, bool stats, hipStream_t s)
{
    if (stats) stage2_kernel<true><<<grid, 256, 0, s>>>(a);
    else stage2_kernel<false><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_stage3_binned(const RasterArgs& a, uint32_t grid, bool stats, hipStream_t s)
{
    tile_scan_kernel<<<1, 1024, 0, s>>>(a);
    tile_scatter_kernel<<<grid, 256, 0, s>>>(a, a.views);
    if (stats) stage3_tile_kernel<true><<<grid, 256, 0, s>>>(a, a.views);
    else stage3_tile_kernel<false><<<grid, 256, 0, s>>>(a, a.views);
    return hipGetLastError();
}

hipError_t launch_stage3(const RasterArgs& a, uint32_t grid, bool stats, hipStream_t s)
{
    if (stats) stage3_kernel<true><<<grid, 256, 0, s>>>(a);
    else stage3_kernel<false><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace curast

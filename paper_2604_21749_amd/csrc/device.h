// Device-side arithmetic of the rasterizer (gfx950).  Compiled with -ffp-contract=off and
// correctly rounded fp32 division, so every float operation below is one IEEE binary32
// round-to-nearest-even step unless written as __builtin_fmaf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace curast {

// Caller buffers (vertices, indices, visibility buffers) are global memory; pointers fetched from
// descriptors are generic to the compiler, which would emit flat accesses.  These casts give it
// the address space so it emits global loads, stores and atomics.
#if defined(__HIP_DEVICE_COMPILE__)
#define CURAST_GLOBAL __attribute__((address_space(1)))
#else
#define CURAST_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ const CURAST_GLOBAL T* gl(const T* p)
{
    return (const CURAST_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ CURAST_GLOBAL T* gl(T* p)
{
    return (CURAST_GLOBAL T*)p;
}

struct Clip {                 // clip-space vertex: x, y and the positive view depth w
    float x, y, w;
};

// ----------------------------------------------------------------------------------------------
// Mesh geometry access, plain or compressed (Sec. 4.6).  Packed index i occupies bits
// [i b, (i + 1) b) of a little-endian stream of 32-bit words.  The 3 b bits of a triangle are
// read with one load of the 2 words (b <= 11) or 4 words (b > 11) from the word holding its first
// bit; the stream carries three words of padding so that this stays inside it.  The 6 bytes of a
// quantized vertex are read with one 8-byte load from the 4-byte boundary at or below them (the
// positions carry one padding element); a component decodes as fmaf(q, step, lo).
// ----------------------------------------------------------------------------------------------
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// Bits [s, s + 32) of the 128-bit little-endian value w0..w3, for s < 96.
__device__ __forceinline__ uint32_t window_bits(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t s)
{
    const uint32_t j = s >> 5;
    const uint32_t lo = j == 0 ? w0 : j == 1 ? w1 : w2;
    const uint32_t hi = j == 0 ? w1 : j == 1 ? w2 : w3;
    return __builtin_amdgcn_alignbit(hi, lo, s & 31);
}

// The three indices whose bits start at bit offset (uword words + lbit bits) of the stream:
// uword is the same for the whole wavefront (64-bit address arithmetic once per wavefront),
// lbit < 2^32 is the lane's part.
__device__ __forceinline__ void packed_triangle_at(const MeshDesc& M, uint64_t uword, uint32_t lbit, uint32_t (&v)[3])
{
    const uint32_t b = M.idx_bits;
    const CURAST_GLOBAL uint32_t* w = gl(M.idx) + uword + (lbit >> 5);
    const uint32_t o = lbit & 31;
    uint32_t w0, w1, w2 = 0, w3 = 0;
    if (b <= 11) {                            // o + 3 b <= 64: two words
        const u32x2_a4 d = *(const CURAST_GLOBAL u32x2_a4*)w;
        w0 = d.x;
        w1 = d.y;
    } else {                                  // o + 3 b <= 127: four words
        const u32x4_a4 d = *(const CURAST_GLOBAL u32x4_a4*)w;
        w0 = d.x;
        w1 = d.y;
        w2 = d.z;
        w3 = d.w;
    }
    const uint32_t mask = b >= 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = M.idx_min + (window_bits(w0, w1, w2, w3, o + k * b) & mask);
}

__device__ __forceinline__ void packed_triangle(const MeshDesc& M, uint64_t t, uint32_t (&v)[3])
{
    const uint64_t bit = 3 * t * (uint64_t)M.idx_bits;
    packed_triangle_at(M, bit >> 5, (uint32_t)bit & 31u, v);
}

// Vertex indices of triangle t (CMP: the mesh is known to be compressed; otherwise decided per
// mesh, which is uniform across the wavefront).
template <int CMP = -1>
__device__ __forceinline__ void mesh_triangle(const MeshDesc& M, uint64_t t, uint32_t (&v)[3])
{
    const bool packed = CMP < 0 ? M.idx_bits != 0 : CMP != 0;
    if (packed) {
        packed_triangle(M, t, v);
    } else {
        const CURAST_GLOBAL uint32_t* ip = gl(M.idx) + 3 * t;
        v[0] = ip[0];
        v[1] = ip[1];
        v[2] = ip[2];
    }
}

template <int CMP = -1>
__device__ __forceinline__ void mesh_vertex(const MeshDesc& M, uint32_t v, float (&p)[3])
{
    const bool packed = CMP < 0 ? M.qpos != nullptr : CMP != 0;
    if (CMP == 1) {
        // the launches specialized for compressed meshes take meshes of at most 2^29 vertices (the
        // host checks), so byte offsets stay below 2^32: 32-bit offset arithmetic from the mesh's
        // base address, the same load and decode as below
        const uint32_t e = 3u * v;
        const u32x2_a4 d =
            *(const CURAST_GLOBAL u32x2_a4*)((const CURAST_GLOBAL char*)gl(M.qpos) + (uint32_t)((e >> 1) << 2));
        const uint64_t q = ((uint64_t)d.x | ((uint64_t)d.y << 32)) >> ((e & 1u) * 16u);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[c] = __builtin_fmaf((float)(uint32_t)((q >> (16 * c)) & 0xFFFFu), M.step[c], M.lo[c]);
    } else if (packed) {
        const uint64_t e = 3 * (uint64_t)v;   // first element; the load starts at element e & ~1
        const u32x2_a4 d = *(const CURAST_GLOBAL u32x2_a4*)((const CURAST_GLOBAL uint32_t*)gl(M.qpos) + (e >> 1));
        const uint64_t q = ((uint64_t)d.x | ((uint64_t)d.y << 32)) >> ((e & 1) * 16);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[c] = __builtin_fmaf((float)(uint32_t)((q >> (16 * c)) & 0xFFFFu), M.step[c], M.lo[c]);
    } else {
        const CURAST_GLOBAL float* q = gl(M.pos) + 3 * (size_t)v;
        p[0] = q[0];
        p[1] = q[1];
        p[2] = q[2];
    }
}

// Row r of a draw matrix applied to an object-space point: fmaf(A0, vx, fmaf(A1, vy, fmaf(A2, vz, A3))).
__device__ __forceinline__ float row_dot(const float* A, float vx, float vy, float vz)
{
    return __builtin_fmaf(A[0], vx, __builtin_fmaf(A[1], vy, __builtin_fmaf(A[2], vz, A[3])));
}

__device__ __forceinline__ Clip transform(const float* A, float vx, float vy, float vz)
{
    Clip c;
    c.x = row_dot(A + 0, vx, vy, vz);
    c.y = row_dot(A + 4, vx, vy, vz);
    c.w = row_dot(A + 8, vx, vy, vz);
    return c;
}

__device__ __forceinline__ bool outside_guard(const Clip& c, float near_plane)
{
    const float g = kGuardBand * c.w;
    return c.w < near_plane || __builtin_fabsf(c.x) > g || __builtin_fabsf(c.y) > g;
}

// Distance to the clip planes in order: w >= near, x >= -16w, x <= 16w, y >= -16w, y <= 16w.
__device__ __forceinline__ float plane_distance(const Clip& c, int plane, float near_plane)
{
    const float g = kGuardBand * c.w;
    switch (plane) {
    case 0: return c.w - near_plane;
    case 1: return c.x + g;
    case 2: return g - c.x;
    case 3: return c.y + g;
    default: return g - c.y;
    }
}

// Sutherland-Hodgman clipping of a triangle (Sec. 4.2); intersections are computed from the
// inside vertex of each crossing edge, so two triangles sharing an edge produce identical points.
// Returns the polygon size (0 when nothing is left, else 3..8).
__device__ inline int clip_triangle(const Clip in[3], float near_plane, Clip poly[8])
{
    Clip tmp[8];
    Clip* src = poly;
    Clip* dst = tmp;
    src[0] = in[0];
    src[1] = in[1];
    src[2] = in[2];
    int n = 3;
#pragma unroll 1
    for (int plane = 0; plane < 5; ++plane) {
        int m = 0;
#pragma unroll 1
        for (int i = 0; i < n; ++i) {
            const Clip a = src[i];
            const Clip b = src[i + 1 < n ? i + 1 : 0];
            const float da = plane_distance(a, plane, near_plane);
            const float db = plane_distance(b, plane, near_plane);
            const bool ain = da >= 0.0f, bin = db >= 0.0f;
            if (ain) dst[m++] = a;
            if (ain != bin) {
                const Clip vi = ain ? a : b;
                const Clip vo = ain ? b : a;
                const float di = ain ? da : db;
                const float dout = ain ? db : da;
                const float t = di / (di - dout);
                Clip r;
                r.x = __builtin_fmaf(t, vo.x - vi.x, vi.x);
                r.y = __builtin_fmaf(t, vo.y - vi.y, vi.y);
                r.w = __builtin_fmaf(t, vo.w - vi.w, vi.w);
                dst[m++] = r;
            }
        }
        n = m;
        if (n < 3) return 0;
        Clip* sw = src;
        src = dst;
        dst = sw;
    }
    if (src != poly)
        for (int i = 0; i < n; ++i) poly[i] = src[i];
    return n;
}

// Window position snapped to 1/256 pixel: zI = 1/w, s = fmaf(c*zI, h, h), X = rint(256 s).
__device__ __forceinline__ void snap_vertex(const Clip& c, float hW, float hH, int32_t& X, int32_t& Y, float& zI)
{
    zI = 1.0f / c.w;
    const float sx = __builtin_fmaf(c.x * zI, hW, hW);
    const float sy = __builtin_fmaf(c.y * zI, hH, hH);
    X = (int32_t)__builtin_rintf(sx * 256.0f);
    Y = (int32_t)__builtin_rintf(sy * 256.0f);
}

// Pixel-centre range [p0, p1] of a snapped interval [lo, hi]: centres 256 p + 128.
__device__ __forceinline__ int32_t first_centre(int32_t lo) { return (lo + 127) >> 8; }
__device__ __forceinline__ int32_t last_centre(int32_t hi) { return (hi - 128) >> 8; }

// Top-left rule for edges of counter-clockwise triangles in y-up window coordinates.
__device__ __forceinline__ bool top_left(int32_t dx, int32_t dy) { return dy < 0 || (dy == 0 && dx < 0); }

__device__ __forceinline__ unsigned long long make_key(float depth, uint64_t id)
{
    const uint32_t bits = __float_as_uint(depth);
    return ((unsigned long long)(bits >> 3) << 36) | (unsigned long long)id;
}

// Depth from the three edge values (interpolated 1/w, Sec. 4.1) in the fixed operation order.
__device__ __forceinline__ float frag_depth(float e0, float e1, float e2, const float zI[3], float area_f)
{
    const float D = __builtin_fmaf(e2, zI[2], __builtin_fmaf(e1, zI[1], e0 * zI[0]));
    return area_f / D;
}

__device__ __forceinline__ void write_fragment(unsigned long long* p, unsigned long long key, bool early_out)
{
    CURAST_GLOBAL unsigned long long* g = gl(p);
    if (early_out) {
        const unsigned long long cur = *g;   // keys only decrease: a stale value is never smaller
        if (key >= cur) return;
    }
    atomicMin(g, key);
}

// General (int64) setup of a snapped triangle, used by stages 2 and 3 and the overflow paths.
struct Tri64 {
    int32_t X[3], Y[3];
    float zI[3];
    int64_t area;
    int32_t dx[3], dy[3];         // edge k runs from vertex k+1 to k+2
    int32_t bias[3];              // 0 on top-left edges, -1 elsewhere: inside iff E + bias >= 0
    int32_t px0, px1, py0, py1;   // pixel-centre box clamped to the view
};

// Returns false when the triangle covers nothing (area <= 0 or empty clamped box).
__device__ inline bool setup_tri64(const int32_t X[3], const int32_t Y[3], const float zI[3], int32_t W,
                                   int32_t H, Tri64& t)
{
    for (int k = 0; k < 3; ++k) {
        t.X[k] = X[k];
        t.Y[k] = Y[k];
        t.zI[k] = zI[k];
    }
    t.area = (int64_t)(X[1] - X[0]) * (int64_t)(Y[2] - Y[0]) - (int64_t)(Y[1] - Y[0]) * (int64_t)(X[2] - X[0]);
    if (t.area <= 0) return false;
    const int32_t minX = min(X[0], min(X[1], X[2])), maxX = max(X[0], max(X[1], X[2]));
    const int32_t minY = min(Y[0], min(Y[1], Y[2])), maxY = max(Y[0], max(Y[1], Y[2]));
    t.px0 = max(first_centre(minX), 0);
    t.px1 = min(last_centre(maxX), W - 1);
    t.py0 = max(first_centre(minY), 0);
    t.py1 = min(last_centre(maxY), H - 1);
    if (t.px0 > t.px1 || t.py0 > t.py1) return false;
    for (int k = 0; k < 3; ++k) {
        const int a = k == 2 ? 0 : k + 1;
        const int b = k == 0 ? 2 : k - 1;
        t.dx[k] = X[b] - X[a];
        t.dy[k] = Y[b] - Y[a];
        t.bias[k] = top_left(t.dx[k], t.dy[k]) ? 0 : -1;
    }
    return true;
}

// Edge value E_k at the centre of pixel (px, py).  Snapped coordinates lie in the guard band
// (|X| < 17 * 8192 * 256 < 2^26) and pixel centres below 2^22, so the differences and the edge
// vectors fit int32 and each product is one 32 x 32 -> 64-bit multiply.
__device__ __forceinline__ int64_t edge64(const Tri64& t, int k, int32_t px, int32_t py)
{
    const int a = k == 2 ? 0 : k + 1;
    const int32_t rx = 256 * px + 128 - t.X[a], ry = 256 * py + 128 - t.Y[a];
    return (int64_t)t.dx[k] * (int64_t)ry - (int64_t)t.dy[k] * (int64_t)rx;
}

// Test one pixel of a general triangle and write its fragment.
__device__ __forceinline__ bool raster_pixel64(const Tri64& t, int32_t px, int32_t py, uint64_t id,
                                               unsigned long long* vis, int32_t W, bool early_out)
{
    const int64_t e0 = edge64(t, 0, px, py);
    const int64_t e1 = edge64(t, 1, px, py);
    const int64_t e2 = edge64(t, 2, px, py);
    if (((e0 + t.bias[0]) | (e1 + t.bias[1]) | (e2 + t.bias[2])) < 0) return false;
    const float depth = frag_depth((float)e0, (float)e1, (float)e2, t.zI, (float)t.area);
    write_fragment(vis + (size_t)py * (size_t)W + (size_t)px, make_key(depth, id), early_out);
    return true;
}

}  // namespace curast

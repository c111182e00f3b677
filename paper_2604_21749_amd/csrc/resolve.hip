// Resolve kernels for gfx950 (Sec. 4.4): one lane per pixel decodes the 28-bit depth / 36-bit
// global triangle ID, finds the (mesh, instance) by binary search over the int64 exclusive
// prefix of triangle counts, reloads and re-projects the triangle, and interpolates its vertex
// attributes perspective-correctly at the pixel centre.  The paper shades in world space with a
// ray-plane intersection; the equivalent screen-space form used here is
//   b_k = q_k / (q0 + q1 + q2), q_k = lambda_k / w_k,
// lambda_k the 2-D cross products of the pixel-relative projected vertices, which stays valid for
// vertices behind the camera (the resolve uses the unclipped triangle).  The backward kernel
// differentiates that expression with visibility held fixed.
#include <hip/hip_runtime.h>

#include "device.h"

namespace curast {

struct Interp {
    float d[3][2];   // pixel-relative window positions
    float zI[3];
    float lam[3];
    float s;
    float b[3];
};

// fp32 interpolation weights in a fixed operation order (no contraction).
__device__ __forceinline__ void interp_weights(const float sx[3], const float sy[3], const float w[3], int32_t px,
                                               int32_t py, Interp& r)
{
    const float cx = (float)px + 0.5f, cy = (float)py + 0.5f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.d[k][0] = sx[k] - cx;
        r.d[k][1] = sy[k] - cy;
        r.zI[k] = 1.0f / w[k];
    }
    r.lam[0] = r.d[1][0] * r.d[2][1] - r.d[1][1] * r.d[2][0];
    r.lam[1] = r.d[2][0] * r.d[0][1] - r.d[2][1] * r.d[0][0];
    r.lam[2] = r.d[0][0] * r.d[1][1] - r.d[0][1] * r.d[1][0];
    const float q0 = r.lam[0] * r.zI[0], q1 = r.lam[1] * r.zI[1], q2 = r.lam[2] * r.zI[2];
    r.s = (q0 + q1) + q2;
    r.b[0] = q0 / r.s;
    r.b[1] = q1 / r.s;
    r.b[2] = q2 / r.s;
}

__device__ __forceinline__ void write_interp(const Interp& r, const float* a0, const float* a1, const float* a2,
                                             uint32_t C, float* o)
{
    for (uint32_t c = 0; c < C; ++c) o[c] = (r.b[0] * a0[c] + r.b[1] * a1[c]) + r.b[2] * a2[c];
}

__device__ __forceinline__ void write_zero(uint32_t C, float* o)
{
    for (uint32_t c = 0; c < C; ++c) o[c] = 0.0f;
}

// ----------------------------------------------------------------------------------------------
// Window positions of one mesh instance: pos_ss[v] = (sx, sy, w) before snapping
// ----------------------------------------------------------------------------------------------
struct ProjectArgs {
    MeshDesc mesh;                // plain or compressed positions
    float A[12];
    float hW, hH;
    float* out;
};

__global__ void __launch_bounds__(256) project_kernel(ProjectArgs a)
{
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.mesh.V) return;
    float p[3];
    mesh_vertex(a.mesh, (uint32_t)v, p);
    const Clip c = transform(a.A, p[0], p[1], p[2]);
    const float zI = 1.0f / c.w;
    a.out[3 * v + 0] = __builtin_fmaf(c.x * zI, a.hW, a.hW);
    a.out[3 * v + 1] = __builtin_fmaf(c.y * zI, a.hH, a.hH);
    a.out[3 * v + 2] = c.w;
}

// ----------------------------------------------------------------------------------------------
// Resolve of a multi-mesh, multi-instance visibility buffer
// ----------------------------------------------------------------------------------------------
constexpr uint32_t kLdsBases = 2048;   // per-mesh first IDs staged in LDS for the binary search

// The triangle of pixel p of the view (row-major index) and its interpolation weights there;
// false for an empty pixel or an invalid triangle.
struct PixelHit {
    const float* a[3];   // attribute rows of the three vertices
    float b[3];
};

// The (mesh, instance) pair and vertex indices of the triangle stored at pixel p; false for an
// empty pixel or an invalid triangle.
__device__ __forceinline__ bool pixel_triangle(const ResolveArgs& a, const uint64_t* B, const DrawDesc* __restrict__ pairs,
                                               const MeshDesc* __restrict__ meshes, uint64_t p, uint32_t& pair,
                                               uint32_t (&vi)[3])
{
    // the int64 prefix of triangle counts over (mesh, instance) pairs (Sec. 4.4) is searched at
    // mesh granularity: the instances of mesh m hold IDs B[m] + i T_m .. B[m] + (i + 1) T_m - 1,
    // so the instance is one exact integer division (the last mesh with B[m] <= id has T_m > 0)
    const uint32_t nm = a.n_meshes;
    const unsigned long long key = gl(a.vis)[p];
    const uint64_t id = key & kIdMask;
    if (key == kEmptyKey || id >= B[nm]) return false;
    uint32_t lo = 0, hi = nm;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (B[mid] <= id) lo = mid;
        else hi = mid;
    }
    const MeshDesc& M = meshes[lo];
    const uint64_t off = id - B[lo];
    const uint64_t inst = off >= M.T ? off / M.T : 0;
    mesh_triangle(M, off - inst * M.T, vi);
    pair = a.mesh_pair[lo] + (uint32_t)inst;
    return vi[0] < M.V && vi[1] < M.V && vi[2] < M.V;
}

__device__ __forceinline__ bool resolve_hit(const ResolveArgs& a, const uint64_t* B, const DrawDesc* __restrict__ pairs,
                                            const MeshDesc* __restrict__ meshes, const float* const* __restrict__ attrs,
                                            uint64_t p, PixelHit& h)
{
    uint32_t lo, vi[3];
    if (!pixel_triangle(a, B, pairs, meshes, p, lo, vi)) return false;
    const DrawDesc& D = pairs[lo];
    const MeshDesc& M = meshes[D.mesh];
    float sx[3], sy[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float q[3];
        mesh_vertex(M, vi[k], q);
        const Clip c = transform(D.A, q[0], q[1], q[2]);
        const float zI = 1.0f / c.w;
        sx[k] = __builtin_fmaf(c.x * zI, a.hW, a.hW);
        sy[k] = __builtin_fmaf(c.y * zI, a.hH, a.hH);
        w[k] = c.w;
    }
    const int32_t px = (int32_t)(p % (uint64_t)a.W), py = (int32_t)(p / (uint64_t)a.W);
    Interp r;
    interp_weights(sx, sy, w, px, py, r);
    const float* at = attrs[D.mesh];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        h.a[k] = at + (size_t)vi[k] * a.C;
        h.b[k] = r.b[k];
    }
    return true;
}

// Stage the prefix of triangle counts in LDS when it fits (all threads of the block take part).
__device__ __forceinline__ const uint64_t* stage_bases(const ResolveArgs& a, const uint64_t* __restrict__ bases,
                                                       uint64_t* s_bases)
{
    const bool staged = a.n_meshes <= kLdsBases;
    if (staged) {
        for (uint32_t i = threadIdx.x; i <= a.n_meshes; i += blockDim.x) s_bases[i] = bases[i];
        __syncthreads();
    }
    return staged ? s_bases : bases;
}

__global__ void __launch_bounds__(256) resolve_kernel(ResolveArgs a, const uint64_t* __restrict__ bases,
                                                      const DrawDesc* __restrict__ pairs,
                                                      const MeshDesc* __restrict__ meshes,
                                                      const float* const* __restrict__ attrs)
{
    __shared__ uint64_t s_bases[kLdsBases + 1];
    const uint64_t* B = stage_bases(a, bases, s_bases);
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t npix = (uint64_t)a.W * (uint64_t)a.H;
    if (p >= npix) return;
    float* o = a.out + p * a.C;
    PixelHit h;
    if (!resolve_hit(a, B, pairs, meshes, attrs, p, h)) {
        write_zero(a.C, o);
        return;
    }
    for (uint32_t c = 0; c < a.C; ++c) o[c] = (h.b[0] * h.a[0][c] + h.b[1] * h.a[1][c]) + h.b[2] * h.a[2][c];
}

// Supersampled resolve: the view holds ss x ss samples per output pixel (a visibility buffer of
// ss W_out x ss H_out); each lane resolves the samples of one output pixel, sums them in fp32 row
// by row (empty samples add 0) and scales by 1 / ss^2 (exact).
constexpr uint32_t kMaxChannels = 16;

__global__ void __launch_bounds__(256) resolve_ss_kernel(ResolveArgs a, const uint64_t* __restrict__ bases,
                                                         const DrawDesc* __restrict__ pairs,
                                                         const MeshDesc* __restrict__ meshes,
                                                         const float* const* __restrict__ attrs)
{
    __shared__ uint64_t s_bases[kLdsBases + 1];
    const uint64_t* B = stage_bases(a, bases, s_bases);
    const uint32_t k = a.ss;
    const uint32_t Wo = (uint32_t)a.W / k, Ho = (uint32_t)a.H / k;
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint64_t)Wo * Ho) return;
    const uint32_t px = (uint32_t)(p % Wo), py = (uint32_t)(p / Wo);
    float acc[kMaxChannels];
#pragma unroll
    for (uint32_t c = 0; c < kMaxChannels; ++c) acc[c] = 0.0f;
    for (uint32_t sy = 0; sy < k; ++sy)
        for (uint32_t sx = 0; sx < k; ++sx) {
            const uint64_t q = (uint64_t)(py * k + sy) * (uint64_t)a.W + (px * k + sx);
            PixelHit h;
            if (!resolve_hit(a, B, pairs, meshes, attrs, q, h)) continue;
#pragma unroll
            for (uint32_t c = 0; c < kMaxChannels; ++c)
                if (c < a.C) acc[c] += (h.b[0] * h.a[0][c] + h.b[1] * h.a[1][c]) + h.b[2] * h.a[2][c];
        }
    const float scale = 1.0f / (float)(k * k);
    float* o = a.out + p * a.C;
#pragma unroll
    for (uint32_t c = 0; c < kMaxChannels; ++c)
        if (c < a.C) o[c] = acc[c] * scale;
}

// ----------------------------------------------------------------------------------------------
// Textured resolve (Sec. 4.4, "Shading and Mip Mapping").  Rays through the pixel and its right,
// top and top-right neighbours hit the triangle's plane; their barycentrics are solved in clip
// space (the world-to-clip map is affine, so they equal the world-space ones, and no vertex is
// divided by its w):
//   n = ((sx - W/2) / (W/2), (sy - H/2) / (H/2)),  a_k = fmaf(-n.x, w_k, x_k),  c_k likewise,
//   e = a x c,  s = (e0 + e1) + e2,  uv = ((e0 uv0 + e1 uv1) + e2 uv2) / s.
// lod = log2 of the larger UV extent of the four hits in texels, clamped to the chain; the colour
// is the trilinear, wrap-around sample at the pixel's own hit.
// ----------------------------------------------------------------------------------------------
__device__ __forceinline__ float4 bilinear(const TexDesc& T, uint32_t l, float u, float v)
{
    const uint32_t wl = max(1u, T.w >> l), hl = max(1u, T.h >> l);
    const CURAST_GLOBAL uint32_t* L = gl(T.texels) + T.off[l];
    const float fu = u - floorf(u), fv = v - floorf(v);
    const float x = fu * (float)wl - 0.5f, y = fv * (float)hl - 0.5f;
    const float x0 = floorf(x), y0 = floorf(y);
    const float ax = x - x0, ay = y - y0;
    // x0 lies in [-1, wl - 1] and y0 in [-1, hl - 1]; the clamps only guard the addressing
    const int32_t ix = (int32_t)x0, iy = (int32_t)y0;
    const uint32_t i0 = min(ix < 0 ? wl - 1 : (uint32_t)ix, wl - 1), i1 = ix + 1 >= (int32_t)wl ? 0u : (uint32_t)(ix + 1);
    const uint32_t j0 = min(iy < 0 ? hl - 1 : (uint32_t)iy, hl - 1), j1 = iy + 1 >= (int32_t)hl ? 0u : (uint32_t)(iy + 1);
    const uint32_t t00 = L[(size_t)j0 * wl + i0], t10 = L[(size_t)j0 * wl + min(i1, wl - 1)];
    const uint32_t t01 = L[(size_t)min(j1, hl - 1) * wl + i0], t11 = L[(size_t)min(j1, hl - 1) * wl + min(i1, wl - 1)];
    const float k = 1.0f / 255.0f;
    float r[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float c00 = (float)((t00 >> (8 * c)) & 0xFFu) * k, c10 = (float)((t10 >> (8 * c)) & 0xFFu) * k;
        const float c01 = (float)((t01 >> (8 * c)) & 0xFFu) * k, c11 = (float)((t11 >> (8 * c)) & 0xFFu) * k;
        const float r0 = c00 + ax * (c10 - c00);
        const float r1 = c01 + ax * (c11 - c01);
        r[c] = r0 + ay * (r1 - r0);
    }
    return make_float4(r[0], r[1], r[2], r[3]);
}

__global__ void __launch_bounds__(256) resolve_textured_kernel(ResolveArgs a, const uint64_t* __restrict__ bases,
                                                               const DrawDesc* __restrict__ pairs,
                                                               const MeshDesc* __restrict__ meshes,
                                                               const float* const* __restrict__ uvs,
                                                               const TexDesc* __restrict__ texs)
{
    __shared__ uint64_t s_bases[kLdsBases + 1];
    const uint64_t* B = stage_bases(a, bases, s_bases);
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint64_t)a.W * (uint64_t)a.H) return;
    CURAST_GLOBAL float4* o = (CURAST_GLOBAL float4*)gl(a.out) + p;
    uint32_t pr, vi[3];
    if (!pixel_triangle(a, B, pairs, meshes, p, pr, vi)) {
        *o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    const DrawDesc& D = pairs[pr];
    const MeshDesc& M = meshes[D.mesh];
    float cx[3], cy[3], cw[3], tu[3], tv[3];
    const CURAST_GLOBAL float* uv = gl(uvs[D.mesh]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float q[3];
        mesh_vertex(M, vi[k], q);
        const Clip c = transform(D.A, q[0], q[1], q[2]);
        cx[k] = c.x;
        cy[k] = c.y;
        cw[k] = c.w;
        tu[k] = uv[2 * (size_t)vi[k]];
        tv[k] = uv[2 * (size_t)vi[k] + 1];
    }
    const int32_t px = (int32_t)(p % (uint64_t)a.W), py = (int32_t)(p / (uint64_t)a.W);
    float su[4], sv[4];
    bool finite = true;
#pragma unroll
    for (int smp = 0; smp < 4; ++smp) {
        const float sx = (float)px + ((smp & 1) ? 1.5f : 0.5f), sy = (float)py + ((smp & 2) ? 1.5f : 0.5f);
        const float nx = (sx - a.hW) / a.hW, ny = (sy - a.hH) / a.hH;
        float e_a[3], e_c[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            e_a[k] = __builtin_fmaf(-nx, cw[k], cx[k]);
            e_c[k] = __builtin_fmaf(-ny, cw[k], cy[k]);
        }
        const float e0 = e_a[1] * e_c[2] - e_a[2] * e_c[1];
        const float e1 = e_a[2] * e_c[0] - e_a[0] * e_c[2];
        const float e2 = e_a[0] * e_c[1] - e_a[1] * e_c[0];
        const float s = (e0 + e1) + e2;
        su[smp] = ((e0 * tu[0] + e1 * tu[1]) + e2 * tu[2]) / s;
        sv[smp] = ((e0 * tv[0] + e1 * tv[1]) + e2 * tv[2]) / s;
        finite = finite && __builtin_isfinite(su[smp]) && __builtin_isfinite(sv[smp]);
    }
    if (!__builtin_isfinite(su[0]) || !__builtin_isfinite(sv[0])) {
        *o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    const TexDesc& T = texs[D.mesh];
    const float top = (float)(T.levels - 1);
    float lod = top;
    if (finite) {
        float umin = su[0], umax = su[0], vmin = sv[0], vmax = sv[0];
#pragma unroll
        for (int smp = 1; smp < 4; ++smp) {
            umin = fminf(umin, su[smp]);
            umax = fmaxf(umax, su[smp]);
            vmin = fminf(vmin, sv[smp]);
            vmax = fmaxf(vmax, sv[smp]);
        }
        const float du = (umax - umin) * (float)T.w, dv = (vmax - vmin) * (float)T.h;
        lod = log2f(fmaxf(du, dv));
        lod = lod > 0.0f ? lod : 0.0f;
        lod = lod > top ? top : lod;
    }
    const uint32_t l0 = (uint32_t)floorf(lod);
    const float t = lod - (float)l0;
    float4 c = bilinear(T, l0, su[0], sv[0]);
    if (t > 0.0f && l0 + 1 < T.levels) {
        const float4 c1 = bilinear(T, l0 + 1, su[0], sv[0]);
        c.x = c.x + t * (c1.x - c.x);
        c.y = c.y + t * (c1.y - c.y);
        c.z = c.z + t * (c1.z - c.z);
        c.w = c.w + t * (c1.w - c.w);
    }
    *o = c;
}

// Level l + 1 of a chain from level l: per-channel rounded mean of a 2 x 2 block, coordinates
// clamped to level l.
__global__ void __launch_bounds__(256) mip_kernel(const uint32_t* __restrict__ src, uint32_t pw, uint32_t ph,
                                                  uint32_t* __restrict__ dst, uint32_t cw, uint32_t ch)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)cw * ch) return;
    const uint32_t x = (uint32_t)(i % cw), y = (uint32_t)(i / cw);
    const uint32_t x0 = 2 * x, y0 = 2 * y, x1 = min(2 * x + 1, pw - 1), y1 = min(2 * y + 1, ph - 1);
    const CURAST_GLOBAL uint32_t* S = gl(src);
    const uint32_t q0 = S[(size_t)y0 * pw + x0], q1 = S[(size_t)y0 * pw + x1];
    const uint32_t q2 = S[(size_t)y1 * pw + x0], q3 = S[(size_t)y1 * pw + x1];
    uint32_t out = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t sum = 2 + ((q0 >> (8 * c)) & 0xFFu) + ((q1 >> (8 * c)) & 0xFFu) + ((q2 >> (8 * c)) & 0xFFu) +
                             ((q3 >> (8 * c)) & 0xFFu);
        out |= (sum >> 2) << (8 * c);
    }
    gl(dst)[i] = out;
}

// ----------------------------------------------------------------------------------------------
// Screen-space (differentiable) resolve of one mesh and its backward pass
// ----------------------------------------------------------------------------------------------
__device__ __forceinline__ bool screen_tri(const ScreenArgs& a, uint64_t p, uint32_t vi[3])
{
    const unsigned long long key = a.vis[p];
    if (key == kEmptyKey) return false;
    const uint64_t id = key & kIdMask;
    if (id < a.id_base || id - a.id_base >= a.T) return false;
    const uint64_t t = id - a.id_base;
    vi[0] = a.idx[3 * t];
    vi[1] = a.idx[3 * t + 1];
    vi[2] = a.idx[3 * t + 2];
    return vi[0] < a.V && vi[1] < a.V && vi[2] < a.V;
}

__global__ void __launch_bounds__(256) resolve_screen_kernel(ScreenArgs a)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint64_t)a.W * (uint64_t)a.H) return;
    float* o = a.out + p * a.C;
    uint32_t vi[3];
    if (!screen_tri(a, p, vi)) {
        write_zero(a.C, o);
        return;
    }
    float sx[3], sy[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sx[k] = a.pos_ss[3 * (size_t)vi[k]];
        sy[k] = a.pos_ss[3 * (size_t)vi[k] + 1];
        w[k] = a.pos_ss[3 * (size_t)vi[k] + 2];
    }
    Interp r;
    interp_weights(sx, sy, w, (int32_t)(p % (uint64_t)a.W), (int32_t)(p / (uint64_t)a.W), r);
    write_interp(r, a.attrs + (size_t)vi[0] * a.C, a.attrs + (size_t)vi[1] * a.C, a.attrs + (size_t)vi[2] * a.C, a.C, o);
}

// Backward with visibility held fixed.  The chain rule of one pixel has cancelling terms
// (G_j - sum_k G_k b_k, the cross-product partials of sliver triangles), so it is evaluated in
// fp64 from the fp32 inputs and each contribution is rounded once into the fp32 atomic sums:
//   dL/da_k = g b_k;  G_k = g . a_k;  dL/dq_j = (G_j - sum_k G_k b_k) / s;
//   dL/dlambda_j = dL/dq_j zI_j;  dL/dw_j = -(dL/dq_j lambda_j) zI_j^2;
//   lambda_0 = d1 x d2, lambda_1 = d2 x d0, lambda_2 = d0 x d1 with d_k = s_k - pixel centre.
//
// Workgroups take 16 x 16 pixel tiles: neighbouring pixels reach neighbouring vertices of a dense
// mesh, so the atomics a workgroup issues close together in time fall on fewer cache lines.  The
// atomics themselves are performed at the memory side, one request per cache-line sector and
// instruction, so each wavefront stages the rows its 64 pixels add to (3 vertices x (C + 3) values)
// in LDS and issues them with neighbouring lanes on neighbouring components of one row: the three
// adds of a row then travel as one request instead of three (C <= kBwdStageC; more channels take
// one atomic per lane and value).
constexpr uint32_t kBwdStageC = 4;

// The fp64 terms of one pixel's chain rule, from the fp32 window positions (sx, sy, w) of its
// triangle's vertices and the pixel (x, y).
struct BwdTerms {
    double d[3][2];   // pixel-relative positions
    double zI[3];
    double lam[3];
    double b[3];
    double inv_sum;   // 1 / (q0 + q1 + q2)
};

__device__ __forceinline__ void bwd_terms(const float (&sx)[3], const float (&sy)[3], const float (&w)[3], uint32_t x,
                                          uint32_t y, BwdTerms& t)
{
    const double cx = (double)x + 0.5, cy = (double)y + 0.5;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t.d[k][0] = (double)sx[k] - cx;
        t.d[k][1] = (double)sy[k] - cy;
        t.zI[k] = 1.0 / (double)w[k];
    }
    t.lam[0] = t.d[1][0] * t.d[2][1] - t.d[1][1] * t.d[2][0];
    t.lam[1] = t.d[2][0] * t.d[0][1] - t.d[2][1] * t.d[0][0];
    t.lam[2] = t.d[0][0] * t.d[1][1] - t.d[0][1] * t.d[1][0];
    const double q[3] = {t.lam[0] * t.zI[0], t.lam[1] * t.zI[1], t.lam[2] * t.zI[2]};
    t.inv_sum = 1.0 / (q[0] + q[1] + q[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) t.b[k] = q[k] * t.inv_sum;
}

// Gradients to (sx, sy, w) of the three vertices from G_k = g . a_k, each rounded once to fp32.
__device__ __forceinline__ void bwd_pos(const BwdTerms& t, const double (&G)[3], float (&gpos)[3][3])
{
    const double Gb = G[0] * t.b[0] + G[1] * t.b[1] + G[2] * t.b[2];
    double L[3], dw[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double Q = (G[j] - Gb) * t.inv_sum;
        L[j] = Q * t.zI[j];
        dw[j] = -(Q * t.lam[j]) * t.zI[j] * t.zI[j];
    }
    const double gx[3] = {L[2] * t.d[1][1] - L[1] * t.d[2][1], L[0] * t.d[2][1] - L[2] * t.d[0][1],
                          L[1] * t.d[0][1] - L[0] * t.d[1][1]};
    const double gy[3] = {L[1] * t.d[2][0] - L[2] * t.d[1][0], L[2] * t.d[0][0] - L[0] * t.d[2][0],
                          L[0] * t.d[1][0] - L[1] * t.d[0][0]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        gpos[k][0] = (float)gx[k];
        gpos[k][1] = (float)gy[k];
        gpos[k][2] = (float)dw[k];
    }
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(256) resolve_backward_kernel(ScreenArgs a)
{
    __shared__ uint32_t s_vid[4][192];
    __shared__ float s_att[4][192 * kBwdStageC];
    __shared__ float s_pos[4][192 * 3];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool staged = a.C <= kBwdStageC;
    const uint32_t tiles_x = ((uint32_t)a.W + 15u) / 16u;
    const uint32_t x = (blockIdx.x % tiles_x) * 16u + (threadIdx.x & 15u);
    const uint32_t y = (blockIdx.x / tiles_x) * 16u + (threadIdx.x >> 4);
    const uint64_t p = (uint64_t)y * (uint64_t)a.W + x;
    uint32_t vi[3] = {~0u, ~0u, ~0u};
    const bool have = x < (uint32_t)a.W && y < (uint32_t)a.H && screen_tri(a, p, vi);
    BwdTerms t = {};
    double G[3] = {0.0, 0.0, 0.0};
    if (have) {
        float sx[3], sy[3], w[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            sx[k] = a.pos_ss[3 * (size_t)vi[k]];
            sy[k] = a.pos_ss[3 * (size_t)vi[k] + 1];
            w[k] = a.pos_ss[3 * (size_t)vi[k] + 2];
        }
        bwd_terms(sx, sy, w, x, y, t);
    }
    // attribute gradients g b_k, and G_k = g . a_k
    const float* g = a.grad_out + (have ? p : 0) * a.C;
    for (uint32_t c = 0; c < a.C; ++c) {
        const double gc = have ? (double)g[c] : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (have) G[k] += gc * (double)a.attrs[(size_t)vi[k] * a.C + c];
            const float v = (float)(gc * t.b[k]);
            if (staged) s_att[wave][(3 * lane + k) * a.C + c] = v;
            else if (have) unsafeAtomicAdd(a.grad_attr + (size_t)vi[k] * a.C + c, v);
        }
    }
    // position gradients
    float gpos[3][3] = {};
    if (a.grad_pos && have) bwd_pos(t, G, gpos);
    if (!staged) {
        if (a.grad_pos && have)
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j) unsafeAtomicAdd(a.grad_pos + 3 * (size_t)vi[k] + j, gpos[k][j]);
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s_vid[wave][3 * lane + k] = have ? vi[k] : ~0u;
#pragma unroll
        for (int j = 0; j < 3; ++j) s_pos[wave][(3 * lane + k) * 3 + j] = gpos[k][j];
    }
    wave_sync();
    // item it = (row, component) in row-major order, row = 3 lane + k of the staging lane
    const uint32_t n_att = 192u * a.C;
    for (uint32_t it = lane; it < n_att; it += 64u) {
        const uint32_t row = it / a.C;
        const uint32_t v = s_vid[wave][row];
        if (v != ~0u) unsafeAtomicAdd(a.grad_attr + (size_t)v * a.C + (it - row * a.C), s_att[wave][it]);
    }
    if (a.grad_pos)
        for (uint32_t it = lane; it < 576u; it += 64u) {
            const uint32_t row = it / 3u;
            const uint32_t v = s_vid[wave][row];
            if (v != ~0u) unsafeAtomicAdd(a.grad_pos + 3 * (size_t)v + (it - 3u * row), s_pos[wave][it]);
        }
}

// Backward of the multi-mesh resolve (resolve_kernel) with visibility held fixed: one lane per
// pixel finds the (mesh, instance) and triangle as the forward does, projects its three vertices
// with the same fp32 operations, and applies the chain rule above; attribute gradients of every
// instance of a mesh add into the mesh's rows, position gradients (to the unsnapped window
// positions of one-instance meshes) where the mesh has a gradient buffer.  One atomic per value.
__global__ void __launch_bounds__(256) resolve_backward_meshes_kernel(ResolveArgs a, const uint64_t* __restrict__ bases,
                                                                      const DrawDesc* __restrict__ pairs,
                                                                      const MeshDesc* __restrict__ meshes,
                                                                      const float* const* __restrict__ attrs)
{
    __shared__ uint64_t s_bases[kLdsBases + 1];
    const uint64_t* B = stage_bases(a, bases, s_bases);
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint64_t)a.W * (uint64_t)a.H) return;
    uint32_t pair, vi[3];
    if (!pixel_triangle(a, B, pairs, meshes, p, pair, vi)) return;
    const DrawDesc& D = pairs[pair];
    const uint32_t m = D.mesh;
    const MeshDesc& M = meshes[m];
    float sx[3], sy[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float q[3];
        mesh_vertex(M, vi[k], q);
        const Clip c = transform(D.A, q[0], q[1], q[2]);
        const float zI = 1.0f / c.w;
        sx[k] = __builtin_fmaf(c.x * zI, a.hW, a.hW);
        sy[k] = __builtin_fmaf(c.y * zI, a.hH, a.hH);
        w[k] = c.w;
    }
    const uint32_t x = (uint32_t)(p % (uint64_t)a.W), y = (uint32_t)(p / (uint64_t)a.W);
    BwdTerms t;
    bwd_terms(sx, sy, w, x, y, t);
    const float* at = attrs[m];
    float* ga = a.grad_attrs[m];
    float* gp = a.grad_pos ? a.grad_pos[m] : nullptr;
    const float* g = a.grad_out + p * a.C;
    double G[3] = {0.0, 0.0, 0.0};
    for (uint32_t c = 0; c < a.C; ++c) {
        const double gc = (double)g[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            G[k] += gc * (double)at[(size_t)vi[k] * a.C + c];
            if (ga) unsafeAtomicAdd(ga + (size_t)vi[k] * a.C + c, (float)(gc * t.b[k]));
        }
    }
    if (gp) {
        float gpos[3][3];
        bwd_pos(t, G, gpos);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) unsafeAtomicAdd(gp + 3 * (size_t)vi[k] + j, gpos[k][j]);
    }
}

// ----------------------------------------------------------------------------------------------
// Launch wrappers
// ----------------------------------------------------------------------------------------------
static uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + 255) / 256); }

hipError_t launch_project(const MeshDesc& mesh, const float A[12], float hW, float hH, float* out, hipStream_t s)
{
    ProjectArgs a;
    a.mesh = mesh;
    for (int i = 0; i < 12; ++i) a.A[i] = A[i];
    a.hW = hW;
    a.hH = hH;
    a.out = out;
    if (mesh.V == 0) return hipSuccess;
    project_kernel<<<blocks_for(mesh.V), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_resolve(const ResolveArgs& a, hipStream_t s)
{
    if (a.ss > 1) {
        const uint64_t out_pixels = (uint64_t)(a.W / a.ss) * (uint64_t)(a.H / a.ss);
        resolve_ss_kernel<<<blocks_for(out_pixels), 256, 0, s>>>(a, a.bases, a.pairs, a.meshes, a.attrs);
    } else {
        resolve_kernel<<<blocks_for((uint64_t)a.W * (uint64_t)a.H), 256, 0, s>>>(a, a.bases, a.pairs, a.meshes,
                                                                                 a.attrs);
    }
    return hipGetLastError();
}

hipError_t launch_resolve_textured(const ResolveArgs& a, hipStream_t s)
{
    resolve_textured_kernel<<<blocks_for((uint64_t)a.W * (uint64_t)a.H), 256, 0, s>>>(a, a.bases, a.pairs, a.meshes,
                                                                                      a.attrs, a.tex);
    return hipGetLastError();
}

// Levels 1 .. levels - 1 from level 0, one launch per level (each reads the previous one).
hipError_t launch_build_mips(uint32_t* texels, uint32_t w, uint32_t h, uint32_t levels, hipStream_t s)
{
    uint64_t off = 0;
    for (uint32_t l = 0; l + 1 < levels; ++l) {
        const uint32_t pw = max(1u, w >> l), ph = max(1u, h >> l), cw = max(1u, w >> (l + 1)), ch = max(1u, h >> (l + 1));
        uint32_t* src = texels + off;
        off += (uint64_t)pw * ph;
        mip_kernel<<<blocks_for((uint64_t)cw * ch), 256, 0, s>>>(src, pw, ph, texels + off, cw, ch);
    }
    return hipGetLastError();
}

hipError_t launch_resolve_screen(const ScreenArgs& a, hipStream_t s)
{
    resolve_screen_kernel<<<blocks_for((uint64_t)a.W * (uint64_t)a.H), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_resolve_backward(const ScreenArgs& a, hipStream_t s)
{
    const uint32_t tiles = (((uint32_t)a.W + 15u) / 16u) * (((uint32_t)a.H + 15u) / 16u);
    resolve_backward_kernel<<<tiles, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_resolve_backward_meshes(const ResolveArgs& a, hipStream_t s)
{
    resolve_backward_meshes_kernel<<<blocks_for((uint64_t)a.W * (uint64_t)a.H), 256, 0, s>>>(a, a.bases, a.pairs,
                                                                                             a.meshes, a.attrs);
    return hipGetLastError();
}

}  // namespace curast

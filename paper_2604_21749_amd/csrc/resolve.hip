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
constexpr uint32_t kLdsBases = 2048;   // prefix entries staged in LDS for the binary search

// The triangle of pixel p of the view (row-major index) and its interpolation weights there;
// false for an empty pixel or an invalid triangle.
struct PixelHit {
    const float* a[3];   // attribute rows of the three vertices
    float b[3];
};

__device__ __forceinline__ bool resolve_hit(const ResolveArgs& a, const uint64_t* B, const DrawDesc* __restrict__ pairs,
                                            const MeshDesc* __restrict__ meshes, const float* const* __restrict__ attrs,
                                            uint64_t p, PixelHit& h)
{
    const uint32_t np = a.n_pairs;
    const unsigned long long key = gl(a.vis)[p];
    const uint64_t id = key & kIdMask;
    if (key == kEmptyKey || id >= B[np]) return false;
    uint32_t lo = 0, hi = np;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (B[mid] <= id) lo = mid;
        else hi = mid;
    }
    const DrawDesc& D = pairs[lo];
    const MeshDesc& M = meshes[D.mesh];
    const uint64_t t = id - B[lo];
    uint32_t vi[3];
    mesh_triangle(M, t, vi);
    if (vi[0] >= M.V || vi[1] >= M.V || vi[2] >= M.V) return false;
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
    const bool staged = a.n_pairs <= kLdsBases;
    if (staged) {
        for (uint32_t i = threadIdx.x; i <= a.n_pairs; i += blockDim.x) s_bases[i] = bases[i];
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
__global__ void __launch_bounds__(256) resolve_backward_kernel(ScreenArgs a)
{
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint64_t)a.W * (uint64_t)a.H) return;
    uint32_t vi[3];
    if (!screen_tri(a, p, vi)) return;
    const double cx = (double)(p % (uint64_t)a.W) + 0.5, cy = (double)(p / (uint64_t)a.W) + 0.5;
    double d[3][2], zI[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k][0] = (double)a.pos_ss[3 * (size_t)vi[k]] - cx;
        d[k][1] = (double)a.pos_ss[3 * (size_t)vi[k] + 1] - cy;
        zI[k] = 1.0 / (double)a.pos_ss[3 * (size_t)vi[k] + 2];
    }
    const double lam[3] = {d[1][0] * d[2][1] - d[1][1] * d[2][0], d[2][0] * d[0][1] - d[2][1] * d[0][0],
                           d[0][0] * d[1][1] - d[0][1] * d[1][0]};
    const double q[3] = {lam[0] * zI[0], lam[1] * zI[1], lam[2] * zI[2]};
    const double sum = q[0] + q[1] + q[2];
    const double b[3] = {q[0] / sum, q[1] / sum, q[2] / sum};
    const float* g = a.grad_out + p * a.C;
    double G[3] = {0.0, 0.0, 0.0};
    for (uint32_t c = 0; c < a.C; ++c) {
        const double gc = g[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            G[k] += gc * (double)a.attrs[(size_t)vi[k] * a.C + c];
            unsafeAtomicAdd(a.grad_attr + (size_t)vi[k] * a.C + c, (float)(gc * b[k]));
        }
    }
    if (!a.grad_pos) return;
    const double Gb = G[0] * b[0] + G[1] * b[1] + G[2] * b[2];
    double L[3], dw[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double Q = (G[j] - Gb) / sum;
        L[j] = Q * zI[j];
        dw[j] = -(Q * lam[j]) * zI[j] * zI[j];
    }
    const double gx[3] = {L[2] * d[1][1] - L[1] * d[2][1], L[0] * d[2][1] - L[2] * d[0][1], L[1] * d[0][1] - L[0] * d[1][1]};
    const double gy[3] = {L[1] * d[2][0] - L[2] * d[1][0], L[2] * d[0][0] - L[0] * d[2][0], L[0] * d[1][0] - L[1] * d[0][0]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        unsafeAtomicAdd(a.grad_pos + 3 * (size_t)vi[k] + 0, (float)gx[k]);
        unsafeAtomicAdd(a.grad_pos + 3 * (size_t)vi[k] + 1, (float)gy[k]);
        unsafeAtomicAdd(a.grad_pos + 3 * (size_t)vi[k] + 2, (float)dw[k]);
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

hipError_t launch_resolve_screen(const ScreenArgs& a, hipStream_t s)
{
    resolve_screen_kernel<<<blocks_for((uint64_t)a.W * (uint64_t)a.H), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_resolve_backward(const ScreenArgs& a, hipStream_t s)
{
    resolve_backward_kernel<<<blocks_for((uint64_t)a.W * (uint64_t)a.H), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace curast

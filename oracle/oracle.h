/*
 * CPU oracle for the brute-force visibility-buffer rasterizer (CuRast, Schuetz et al.).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this library:
 * it exists so that tests, the smoke check and the benchmark's CPU baseline can compare the GPU
 * kernels against a plain, slow, obviously correct definition of the result.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * What it computes (the plain definition the GPU path must reach exactly):
 *   for every pixel, the minimum 64-bit key (depth28 << 36 | global triangle ID) over every
 *   fragment of every triangle of every mesh instance (Sec. 3.1 atomicMin visibility, Sec. 4.1
 *   key layout, Sec. 4 global triangle IDs), where a fragment exists when the pixel centre is
 *   inside the triangle under fixed-point coverage rules.  Stages, thresholds and culling in the
 *   GPU path are speed-ups that must not change this result.
 *
 * Arithmetic (both sides implement it independently; every float op is IEEE binary32 round-to-
 * nearest-even, compiled with -ffp-contract=off; fmaf is the fused operation, used only where
 * written):
 *   draw matrix  A = VP * X for the x, y, w rows of the view-projection (row 2 unused):
 *                A[r][c] = (VP[r][0]*X[0][c] + VP[r][1]*X[1][c]) + VP[r][2]*X[2][c]   (c < 3)
 *                A[r][3] = ((VP[r][0]*X[0][3] + VP[r][1]*X[1][3]) + VP[r][2]*X[2][3]) + VP[r][3]
 *   vertex       c_r = fmaf(A[r][0], vx, fmaf(A[r][1], vy, fmaf(A[r][2], vz, A[r][3])))
 *   no fragments if every w < near
 *   clip         if any w < near or |x| > 16w or |y| > 16w: Sutherland-Hodgman against
 *                w >= near, x >= -16w, x <= 16w, y >= -16w, y <= 16w (in that order), each
 *                intersection computed from the inside vertex: t = d_in / (d_in - d_out),
 *                v = fmaf(t, out - in, in); fan (q0, qj, qj+1) of the result
 *   snap         zI = 1/w, sx = fmaf(x*zI, W/2, W/2), sy likewise; X = rint(sx*256), Y = rint(sy*256)
 *   setup        area = (X1-X0)(Y2-Y0) - (Y1-Y0)(X2-X0) (int64); area <= 0: no fragments
 *   coverage     sample of pixel (px, py) at (256px+128, 256py+128); edge k from v(k+1) to v(k+2),
 *                E_k = dx*(Py - Y(k+1)) - dy*(Px - X(k+1)); inside iff every E_k > 0 or
 *                E_k == 0 on a top-left edge (dy < 0, or dy == 0 and dx < 0); y is up, row 0 bottom
 *   depth        D = fmaf((float)E2, zI2, fmaf((float)E1, zI1, (float)E0 * zI0)); depth = (float)area / D
 *   key          ((bits(depth) >> 3) << 36) | ID, ID = exclusive prefix of triangle counts over
 *                all (mesh, instance) pairs in mesh-major order, plus the triangle index
 *   clear value  all ones
 *
 * Resolve (fp32, Sec. 4.4): per pixel decode the ID, find the (mesh, instance) by binary search
 * over the int64 prefix array, recompute the three original vertices, unsnapped screen positions
 * s_k, d_k = s_k - (px + 0.5, py + 0.5), lambda_0 = d1 x d2, lambda_1 = d2 x d0, lambda_2 = d0 x d1,
 * q_k = lambda_k * zI_k, s = (q0 + q1) + q2, b_k = q_k / s, out = (b0 a0 + b1 a1) + b2 a2.
 * Empty pixels resolve to 0.
 *
 * Every function returns 0 on success and a negative value on invalid arguments.
 */
#ifndef CURAST_ORACLE_H
#define CURAST_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    const float* pos;      /* [V][3] object-space positions */
    uint32_t V;
    const uint32_t* idx;   /* [T][3] vertex indices */
    uint64_t T;
    const float* inst;     /* [N][12] row-major 3x4 object-to-world, or NULL for identity (N = 1) */
    uint32_t N;
} orc_mesh;

typedef struct {
    float vp[16];          /* row-major view-projection; rows 0, 1, 3 used */
    float near_plane;
    int32_t width, height;
} orc_view;

/* Number of (mesh, instance) pairs, and their exclusive prefix of triangle counts
   (bases must hold pairs + 1 entries; the last one is the total). */
int64_t orc_num_pairs(const orc_mesh* meshes, uint32_t M);
int orc_id_bases(const orc_mesh* meshes, uint32_t M, int64_t* bases);

/* Global ID -> (mesh, instance, local triangle) by binary search over the prefix array. */
int orc_decode_id(const orc_mesh* meshes, uint32_t M, const int64_t* bases, int64_t id,
                  uint32_t* mesh, uint32_t* inst, uint64_t* tri);

/* Visibility buffer [H][W] (row 0 = bottom).  nthreads <= 0 uses all cores.  Triangle ranges
   are split over threads, each with a private buffer, merged by elementwise minimum. */
int orc_rasterize(const orc_mesh* meshes, uint32_t M, const orc_view* view, uint64_t* vis, int nthreads);

/* Only the (mesh, instance) pairs in [pair_begin, pair_end) and triangles [tri_begin, tri_end)
   of each (used to time a bounded sample of a large workload). */
int orc_rasterize_range(const orc_mesh* meshes, uint32_t M, const orc_view* view,
                        int64_t pair_begin, int64_t pair_end, uint64_t tri_begin, uint64_t tri_end,
                        uint64_t* vis, int nthreads);

/* Per-pixel counts of front-facing (area > 0) and back-facing (area < 0, tested as the reversed
   triangle) coverage, with no depth test: pins the fill rule (watertightness invariants). */
int orc_coverage_counts(const orc_mesh* meshes, uint32_t M, const orc_view* view,
                        uint32_t* front, uint32_t* back);

/* Independent brute-force transcription: every pixel against every triangle, no bounding box. */
int orc_rasterize_brute(const orc_mesh* meshes, uint32_t M, const orc_view* view, uint64_t* vis);

/* Compressed geometry (Sec. 4.6): binary32 quantization of positions to 16 bits relative to lo with
 * scale (float)(1 / (double)step) (0 for step 0), and the decoding fmaf(q, step, lo). */
int orc_quantize_positions(const float* pos, uint32_t V, const float lo[3], const float step[3], uint16_t* out);
int orc_decode_positions(const uint16_t* q, uint32_t V, const float lo[3], const float step[3], float* out);

/* Textures (Sec. 4.4, "Shading and Mip Mapping"): RGBA8 mip chains, level l is
 * max(1, width >> l) x max(1, height >> l) texels, levels concatenated from level 0. */
typedef struct {
    const uint32_t* texels;
    uint32_t width, height, levels;
} orc_texture;

/* Words of a chain (0 if the sizes are not powers of two in [1, 16384] or levels is out of
 * range); the 2x2 box-filtered chain (rounded mean, coordinates clamped) from level 0; one
 * trilinear wrap-around sample; the level of detail of four UV hits (see texture.c). */
uint64_t orc_texture_texels(uint32_t width, uint32_t height, uint32_t levels);
int orc_build_mips(uint32_t* texels, uint32_t width, uint32_t height, uint32_t levels);
void orc_sample_trilinear(const orc_texture* tex, float u, float v, float lod, float out[4]);
float orc_texture_lod(const orc_texture* tex, const float u[4], const float v[4], int finite);

/* Textured resolve: out [H][W][4] RGBA; uvs[m] is mesh m's [V][2], textures[m] its texture. */
int orc_resolve_textured(const orc_mesh* meshes, uint32_t M, const orc_view* view, const uint64_t* vis,
                         const float* const* uvs, const orc_texture* textures, float* out, int nthreads);

/* Unsnapped screen positions (sx, sy, w) of every vertex of one mesh instance: [V][3]. */
int orc_project(const orc_mesh* mesh, uint32_t instance, const orc_view* view, float* pos_ss);

/* fp32 resolve of a visibility buffer: out [H][W][C]; attrs[m] is mesh m's [V][C]. */
int orc_resolve(const orc_mesh* meshes, uint32_t M, const orc_view* view, const uint64_t* vis,
                const float* const* attrs, uint32_t C, float* out, int nthreads);

/* fp32 resolve of one mesh from given screen positions pos_ss [V][3] = (sx, sy, w); pixels whose
   ID lies outside [id_base, id_base + T) resolve to 0. */
int orc_resolve_screen(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                       int64_t id_base, const float* pos_ss, uint32_t V, const float* attrs,
                       uint32_t C, float* out);

/* fp64 versions for gradient checks. */
int orc_resolve_screen_f64(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                           int64_t id_base, const double* pos_ss, uint32_t V, const double* attrs,
                           uint32_t C, double* out);

/* Analytic fp64 gradient of L = sum_p sum_c grad_out[p][c] * out[p][c] (i.e. the chain rule with
   a given upstream gradient) with visibility held fixed; accumulates into grad_attr [V][C] and
   grad_pos [V][3] (either may be NULL). */
int orc_resolve_screen_backward_f64(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx,
                                    uint64_t T, int64_t id_base, const double* pos_ss, uint32_t V,
                                    const double* attrs, uint32_t C, const double* grad_out,
                                    double* grad_attr, double* grad_pos);

/* Central finite differences of the squared-error loss L = sum_p sum_c (out - target)^2 with
   respect to pos_ss[v][j] for the listed vertices, evaluated in fp64 over the pixels whose
   visible triangle uses v (visibility fixed).  order4 = 0: (L(+e) - L(-e)) / 2e; order4 = 1:
   the fourth-order central stencil (4 D(e) - D(2e)) / 3 of the same differences.  fd [n][3]. */
int orc_fd_pos_grad_l2(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                       int64_t id_base, const double* pos_ss, uint32_t V, const double* attrs,
                       uint32_t C, const double* target, const uint32_t* verts, uint32_t n,
                       double eps, int order4, double* fd);

#ifdef __cplusplus
}
#endif
#endif

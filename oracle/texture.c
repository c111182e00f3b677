/*
 * Oracle textured resolve (test infrastructure only, see oracle.h).
 *
 * Sec. 4.4, "Shading and Mip Mapping": for each covered pixel, cast rays through the pixel and
 * its right, top and top-right neighbours, intersect them with the plane of the pixel's
 * triangle, interpolate (or extrapolate) the vertex UVs at the four hits, take the UV extent in
 * texels as the footprint and its log2 as the mip level, and sample the texture at the pixel's
 * own hit.  The hit barycentrics are solved in clip space, where the ray through window point
 * (sx, sy) is {x - n.x w = 0, y - n.y w = 0}: the world-to-clip map is affine, so the
 * barycentrics of the intersection are the same as in world space, and no vertex is divided by
 * its w (vertices behind the camera need no special case).
 *
 * Textures are RGBA8 mip chains, levels concatenated; level l is max(1, w >> l) by
 * max(1, h >> l).  Every step below is one binary32 operation in the written order.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ID_MASK ((((uint64_t)1) << 36) - 1)
#define EMPTY (~(uint64_t)0)

void orc_internal_draw_matrix(const float vp[16], const float* inst, float A[3][4]);
void orc_internal_transform(const float A[3][4], const float* p, float out[3]);

static uint32_t level_dim(uint32_t d, uint32_t l) { return (d >> l) ? (d >> l) : 1u; }

static int is_pow2(uint32_t d) { return d && !(d & (d - 1)); }

static uint32_t max_levels(uint32_t w, uint32_t h)
{
    uint32_t m = w > h ? w : h, n = 1;
    while (m > 1) { m >>= 1; ++n; }
    return n;
}

uint64_t orc_texture_texels(uint32_t w, uint32_t h, uint32_t levels)
{
    if (!is_pow2(w) || !is_pow2(h) || w > 16384 || h > 16384 || levels < 1 || levels > max_levels(w, h)) return 0;
    uint64_t n = 0;
    for (uint32_t l = 0; l < levels; ++l) n += (uint64_t)level_dim(w, l) * level_dim(h, l);
    return n;
}

static uint64_t level_offset(uint32_t w, uint32_t h, uint32_t l)
{
    uint64_t n = 0;
    for (uint32_t j = 0; j < l; ++j) n += (uint64_t)level_dim(w, j) * level_dim(h, j);
    return n;
}

int orc_build_mips(uint32_t* texels, uint32_t w, uint32_t h, uint32_t levels)
{
    if (!texels || !orc_texture_texels(w, h, levels)) return -1;
    for (uint32_t l = 0; l + 1 < levels; ++l) {
        const uint32_t pw = level_dim(w, l), ph = level_dim(h, l);
        const uint32_t cw = level_dim(w, l + 1), ch = level_dim(h, l + 1);
        const uint32_t* src = texels + level_offset(w, h, l);
        uint32_t* dst = texels + level_offset(w, h, l + 1);
        for (uint32_t j = 0; j < ch; ++j)
            for (uint32_t i = 0; i < cw; ++i) {
                const uint32_t x0 = 2 * i, y0 = 2 * j;
                const uint32_t x1 = 2 * i + 1 < pw ? 2 * i + 1 : pw - 1;
                const uint32_t y1 = 2 * j + 1 < ph ? 2 * j + 1 : ph - 1;
                const uint32_t q[4] = {src[(size_t)y0 * pw + x0], src[(size_t)y0 * pw + x1], src[(size_t)y1 * pw + x0],
                                       src[(size_t)y1 * pw + x1]};
                uint32_t out = 0;
                for (int c = 0; c < 4; ++c) {
                    uint32_t sum = 2;
                    for (int k = 0; k < 4; ++k) sum += (q[k] >> (8 * c)) & 0xFFu;
                    out |= (sum >> 2) << (8 * c);
                }
                dst[(size_t)j * cw + i] = out;
            }
    }
    return 0;
}

/* One level, bilinear, wrap-around. */
static void bilinear(const orc_texture* T, uint32_t l, float u, float v, float out[4])
{
    const uint32_t wl = level_dim(T->width, l), hl = level_dim(T->height, l);
    const uint32_t* L = T->texels + level_offset(T->width, T->height, l);
    const float fu = u - floorf(u), fv = v - floorf(v);
    const float x = fu * (float)wl - 0.5f, y = fv * (float)hl - 0.5f;
    const float x0 = floorf(x), y0 = floorf(y);
    const float ax = x - x0, ay = y - y0;
    /* x0 lies in [-1, wl - 1] and y0 in [-1, hl - 1] */
    const int64_t ix = (int64_t)x0, iy = (int64_t)y0;
    const uint32_t i0 = (uint32_t)((ix + (int64_t)wl) % (int64_t)wl), i1 = (uint32_t)((ix + 1) % (int64_t)wl);
    const uint32_t j0 = (uint32_t)((iy + (int64_t)hl) % (int64_t)hl), j1 = (uint32_t)((iy + 1) % (int64_t)hl);
    const uint32_t t00 = L[(size_t)j0 * wl + i0], t10 = L[(size_t)j0 * wl + i1];
    const uint32_t t01 = L[(size_t)j1 * wl + i0], t11 = L[(size_t)j1 * wl + i1];
    const float k = 1.0f / 255.0f;
    for (int c = 0; c < 4; ++c) {
        const float c00 = (float)((t00 >> (8 * c)) & 0xFFu) * k, c10 = (float)((t10 >> (8 * c)) & 0xFFu) * k;
        const float c01 = (float)((t01 >> (8 * c)) & 0xFFu) * k, c11 = (float)((t11 >> (8 * c)) & 0xFFu) * k;
        const float r0 = c00 + ax * (c10 - c00);
        const float r1 = c01 + ax * (c11 - c01);
        out[c] = r0 + ay * (r1 - r0);
    }
}

void orc_sample_trilinear(const orc_texture* T, float u, float v, float lod, float out[4])
{
    const float top = (float)(T->levels - 1);
    if (!(lod > 0.0f)) lod = 0.0f;   /* also NaN */
    if (lod > top) lod = top;
    const uint32_t l0 = (uint32_t)floorf(lod);
    const float t = lod - (float)l0;
    bilinear(T, l0, u, v, out);
    if (t > 0.0f && l0 + 1 < T->levels) {
        float hi[4];
        bilinear(T, l0 + 1, u, v, hi);
        for (int c = 0; c < 4; ++c) out[c] = out[c] + t * (hi[c] - out[c]);
    }
}

/* UV of the ray through window point (sx, sy) hitting the plane of clip-space vertices cl[k]
 * (x, y, w); returns 0 when either coordinate is not finite. */
static int ray_uv(const float cl[3][3], const float* uv[3], float sx, float sy, float hW, float hH, float* u,
                  float* v)
{
    const float nx = (sx - hW) / hW, ny = (sy - hH) / hH;
    float a[3], c[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = fmaf(-nx, cl[k][2], cl[k][0]);
        c[k] = fmaf(-ny, cl[k][2], cl[k][1]);
    }
    const float e0 = a[1] * c[2] - a[2] * c[1];
    const float e1 = a[2] * c[0] - a[0] * c[2];
    const float e2 = a[0] * c[1] - a[1] * c[0];
    const float s = (e0 + e1) + e2;
    *u = ((e0 * uv[0][0] + e1 * uv[1][0]) + e2 * uv[2][0]) / s;
    *v = ((e0 * uv[0][1] + e1 * uv[1][1]) + e2 * uv[2][1]) / s;
    return isfinite(*u) && isfinite(*v);
}

float orc_texture_lod(const orc_texture* T, const float u[4], const float v[4], int finite)
{
    const float top = (float)(T->levels - 1);
    if (!finite) return top;
    float umin = u[0], umax = u[0], vmin = v[0], vmax = v[0];
    for (int j = 1; j < 4; ++j) {
        umin = fminf(umin, u[j]);
        umax = fmaxf(umax, u[j]);
        vmin = fminf(vmin, v[j]);
        vmax = fmaxf(vmax, v[j]);
    }
    const float du = (umax - umin) * (float)T->width, dv = (vmax - vmin) * (float)T->height;
    float lod = log2f(fmaxf(du, dv));
    if (!(lod > 0.0f)) lod = 0.0f;
    if (lod > top) lod = top;
    return lod;
}

typedef struct {
    const orc_mesh* meshes;
    const orc_view* view;
    const uint64_t* vis;
    const float* const* uvs;
    const orc_texture* tex;
    float* out;
    const int64_t* bases;
    const uint32_t* pair_mesh;
    int64_t npairs;
    float (*A)[3][4];
    int32_t y0, y1;
} tjob;

static void* textured_rows(void* arg)
{
    const tjob* j = (const tjob*)arg;
    const int32_t W = j->view->width;
    const float hW = 0.5f * (float)j->view->width, hH = 0.5f * (float)j->view->height;
    static const float off[4][2] = {{0.5f, 0.5f}, {1.5f, 0.5f}, {0.5f, 1.5f}, {1.5f, 1.5f}};
    for (int32_t py = j->y0; py < j->y1; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const size_t p = (size_t)py * (size_t)W + (size_t)px;
            float* o = j->out + 4 * p;
            memset(o, 0, 4 * sizeof(float));
            const uint64_t key = j->vis[p];
            if (key == EMPTY) continue;
            const int64_t id = (int64_t)(key & ID_MASK);
            if (id >= j->bases[j->npairs]) continue;
            int64_t lo = 0, hi = j->npairs;
            while (hi - lo > 1) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (j->bases[mid] <= id) lo = mid; else hi = mid;
            }
            const uint32_t m = j->pair_mesh[lo];
            const orc_mesh* me = &j->meshes[m];
            const uint64_t t = (uint64_t)(id - j->bases[lo]);
            float cl[3][3];
            const float* uv[3];
            int bad = 0;
            for (int k = 0; k < 3; ++k) {
                const uint32_t vi = me->idx[3 * t + (uint64_t)k];
                if (vi >= me->V) { bad = 1; break; }
                orc_internal_transform(j->A[lo], me->pos + 3 * (size_t)vi, cl[k]);
                uv[k] = j->uvs[m] + 2 * (size_t)vi;
            }
            if (bad) continue;
            float u[4], v[4];
            int finite = 1;
            for (int s = 0; s < 4; ++s)
                finite &= ray_uv(cl, uv, (float)px + off[s][0], (float)py + off[s][1], hW, hH, &u[s], &v[s]);
            if (!isfinite(u[0]) || !isfinite(v[0])) continue;
            orc_sample_trilinear(&j->tex[m], u[0], v[0], orc_texture_lod(&j->tex[m], u, v, finite), o);
        }
    return NULL;
}

int orc_resolve_textured(const orc_mesh* meshes, uint32_t M, const orc_view* view, const uint64_t* vis,
                         const float* const* uvs, const orc_texture* textures, float* out, int nthreads)
{
    if (!view || !vis || !uvs || !textures || !out || view->width <= 0 || view->height <= 0) return -1;
    for (uint32_t m = 0; m < M; ++m)
        if (!textures[m].texels || !orc_texture_texels(textures[m].width, textures[m].height, textures[m].levels))
            return -1;
    const int64_t np = orc_num_pairs(meshes, M);
    int64_t* bases = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np + 1));
    uint32_t* pm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(np + 1));
    float(*A)[3][4] = malloc(sizeof(float[3][4]) * (size_t)(np + 1));
    if (!bases || !pm || !A) { free(bases); free(pm); free(A); return -2; }
    orc_id_bases(meshes, M, bases);
    int64_t p = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const uint32_t n = meshes[m].inst ? meshes[m].N : 1;
        for (uint32_t i = 0; i < n; ++i, ++p) {
            pm[p] = m;
            orc_internal_draw_matrix(view->vp, meshes[m].inst ? meshes[m].inst + 12 * (size_t)i : NULL, A[p]);
        }
    }
    int nt = nthreads > 0 ? nthreads : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > view->height) nt = view->height;
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    tjob* jobs = (tjob*)calloc((size_t)nt, sizeof(tjob));
    for (int t = 0; t < nt; ++t) {
        tjob jb = {meshes, view, vis, uvs, textures, out, bases, pm, np, A,
                   (int32_t)((int64_t)view->height * t / nt), (int32_t)((int64_t)view->height * (t + 1) / nt)};
        jobs[t] = jb;
        if (t) pthread_create(&th[t], NULL, textured_rows, &jobs[t]);
    }
    textured_rows(&jobs[0]);
    for (int t = 1; t < nt; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    free(bases);
    free(pm);
    free(A);
    return 0;
}

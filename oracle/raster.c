/*
 * Oracle rasterization: the plain definition of the visibility buffer (test infrastructure only,
 * see oracle.h).  One triangle at a time, every pixel centre of its bounding box, int64 edge
 * functions, elementwise minimum of 64-bit keys.  No stages, no queues, no culling beyond what
 * the definition itself implies.
 *
 * Paper passages followed:
 *   Sec. 3.1   64-bit atomicMin of (depth bits << 32 | payload): the closest fragment wins.
 *   Sec. 4     global triangle ID = exclusive prefix sum of triangle counts per mesh/instance.
 *   Sec. 4.1   view-space transform and projection vector (Eqs. 1-2); frustum, tiny-triangle and
 *              backface culling; bounding-box traversal; 28-bit depth (sign and 3 low mantissa
 *              bits dropped) above a 36-bit triangle ID; perspective-correct depth from
 *              interpolated 1/z.
 *   Sec. 4.2   Sutherland-Hodgman clipping of triangles that cross the near plane.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GUARD 16.0f                         /* guard band: |x|, |y| <= 16 w needs no clipping */
#define ID_MASK ((((uint64_t)1) << 36) - 1)

typedef struct { float x, y, w; } cvert;              /* clip-space vertex */
typedef struct { int64_t X, Y; float zI; } svert;      /* snapped window vertex, 1/256 px */

typedef struct {
    int32_t W, H;
    float hW, hH, near_plane;
} vctx;

static vctx make_vctx(const orc_view* v)
{
    vctx c;
    c.W = v->width;
    c.H = v->height;
    c.hW = 0.5f * (float)v->width;
    c.hH = 0.5f * (float)v->height;
    c.near_plane = v->near_plane;
    return c;
}

static int view_ok(const orc_view* v)
{
    return v && v->width > 0 && v->height > 0 && v->width <= 16384 && v->height <= 16384 &&
           v->near_plane > 0.0f && isfinite(v->near_plane);
}

/* A = VP * X restricted to the x, y and w rows of VP; X is 3x4 row-major (identity if NULL). */
static void draw_matrix(const float vp[16], const float* inst, float A[3][4])
{
    static const float ident[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    const float* X = inst ? inst : ident;
    static const int rows[3] = {0, 1, 3};
    for (int k = 0; k < 3; ++k) {
        const float* r = vp + 4 * rows[k];
        for (int c = 0; c < 3; ++c) {
            float t = r[0] * X[0 * 4 + c];
            t = t + r[1] * X[1 * 4 + c];
            t = t + r[2] * X[2 * 4 + c];
            A[k][c] = t;
        }
        float t = r[0] * X[0 * 4 + 3];
        t = t + r[1] * X[1 * 4 + 3];
        t = t + r[2] * X[2 * 4 + 3];
        A[k][3] = t + r[3];
    }
}

static cvert transform(const float A[3][4], const float* p)
{
    cvert o;
    o.x = fmaf(A[0][0], p[0], fmaf(A[0][1], p[1], fmaf(A[0][2], p[2], A[0][3])));
    o.y = fmaf(A[1][0], p[0], fmaf(A[1][1], p[1], fmaf(A[1][2], p[2], A[1][3])));
    o.w = fmaf(A[2][0], p[0], fmaf(A[2][1], p[1], fmaf(A[2][2], p[2], A[2][3])));
    return o;
}

/* Signed distance of v to clip plane `plane` (0 near, 1 left, 2 right, 3 bottom, 4 top). */
static float plane_dist(cvert v, int plane, float near_plane)
{
    switch (plane) {
    case 0: return v.w - near_plane;
    case 1: return v.x + GUARD * v.w;
    case 2: return GUARD * v.w - v.x;
    case 3: return v.y + GUARD * v.w;
    default: return GUARD * v.w - v.y;
    }
}

static int needs_clip(const cvert c[3], float near_plane)
{
    for (int k = 0; k < 3; ++k) {
        if (c[k].w < near_plane) return 1;
        if (fabsf(c[k].x) > GUARD * c[k].w) return 1;
        if (fabsf(c[k].y) > GUARD * c[k].w) return 1;
    }
    return 0;
}

/* Sutherland-Hodgman against the five planes in order; returns the vertex count (0 or >= 3). */
static int clip_polygon(const cvert tri[3], float near_plane, cvert out[8])
{
    cvert a[8], b[8];
    int n = 3;
    memcpy(a, tri, sizeof(cvert) * 3);
    for (int plane = 0; plane < 5; ++plane) {
        int m = 0;
        for (int i = 0; i < n; ++i) {
            cvert p = a[i], q = a[(i + 1) % n];
            float dp = plane_dist(p, plane, near_plane);
            float dq = plane_dist(q, plane, near_plane);
            int pin = dp >= 0.0f, qin = dq >= 0.0f;
            if (pin) b[m++] = p;
            if (pin != qin) {
                cvert vi = pin ? p : q, vo = pin ? q : p;
                float di = pin ? dp : dq, dout = pin ? dq : dp;
                float t = di / (di - dout);
                cvert r;
                r.x = fmaf(t, vo.x - vi.x, vi.x);
                r.y = fmaf(t, vo.y - vi.y, vi.y);
                r.w = fmaf(t, vo.w - vi.w, vi.w);
                b[m++] = r;
            }
        }
        n = m;
        if (n < 3) return 0;
        memcpy(a, b, sizeof(cvert) * (size_t)n);
    }
    memcpy(out, a, sizeof(cvert) * (size_t)n);
    return n;
}

static int snap(cvert v, const vctx* vc, svert* s)
{
    float zI = 1.0f / v.w;
    float sx = fmaf(v.x * zI, vc->hW, vc->hW);
    float sy = fmaf(v.y * zI, vc->hH, vc->hH);
    float fx = rintf(sx * 256.0f), fy = rintf(sy * 256.0f);
    if (!(fabsf(fx) < 1073741824.0f) || !(fabsf(fy) < 1073741824.0f)) return 0; /* non-finite input */
    s->X = (int64_t)fx;
    s->Y = (int64_t)fy;
    s->zI = zI;
    return 1;
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int is_top_left(int64_t dx, int64_t dy)
{
    return dy < 0 || (dy == 0 && dx < 0);
}

static uint64_t make_key(float depth, uint64_t id)
{
    uint32_t bits;
    memcpy(&bits, &depth, 4);
    return ((uint64_t)(bits >> 3) << 36) | (id & ID_MASK);
}

/* Rasterize one snapped triangle into vis (minimum). */
static void raster_snapped(const svert v[3], uint64_t id, const vctx* vc, uint64_t* vis)
{
    int64_t area = (v[1].X - v[0].X) * (v[2].Y - v[0].Y) - (v[1].Y - v[0].Y) * (v[2].X - v[0].X);
    if (area <= 0) return;                                      /* back-facing or degenerate */
    int64_t minX = v[0].X, maxX = v[0].X, minY = v[0].Y, maxY = v[0].Y;
    for (int k = 1; k < 3; ++k) {
        if (v[k].X < minX) minX = v[k].X;
        if (v[k].X > maxX) maxX = v[k].X;
        if (v[k].Y < minY) minY = v[k].Y;
        if (v[k].Y > maxY) maxY = v[k].Y;
    }
    /* pixel centres 256*p + 128 inside [min, max]: p in [ceil((min-128)/256), floor((max-128)/256)] */
    int64_t px0 = -floor_div(128 - minX, 256), px1 = floor_div(maxX - 128, 256);
    int64_t py0 = -floor_div(128 - minY, 256), py1 = floor_div(maxY - 128, 256);
    if (px0 < 0) px0 = 0;
    if (py0 < 0) py0 = 0;
    if (px1 > vc->W - 1) px1 = vc->W - 1;
    if (py1 > vc->H - 1) py1 = vc->H - 1;
    if (px0 > px1 || py0 > py1) return;

    int64_t dx[3], dy[3];
    int tl[3];
    for (int k = 0; k < 3; ++k) {
        const svert* a = &v[(k + 1) % 3];
        const svert* b = &v[(k + 2) % 3];
        dx[k] = b->X - a->X;
        dy[k] = b->Y - a->Y;
        tl[k] = is_top_left(dx[k], dy[k]);
    }
    const float farea = (float)area;
    for (int64_t py = py0; py <= py1; ++py) {
        const int64_t Py = 256 * py + 128;
        for (int64_t px = px0; px <= px1; ++px) {
            const int64_t Px = 256 * px + 128;
            const size_t p = (size_t)py * (size_t)vc->W + (size_t)px;
            int64_t E[3];
            int inside = 1;
            for (int k = 0; k < 3; ++k) {
                const svert* a = &v[(k + 1) % 3];
                E[k] = dx[k] * (Py - a->Y) - dy[k] * (Px - a->X);
                if (!(E[k] > 0 || (E[k] == 0 && tl[k]))) inside = 0;
            }
            if (!inside) continue;
            float D = fmaf((float)E[2], v[2].zI, fmaf((float)E[1], v[1].zI, (float)E[0] * v[0].zI));
            float depth = farea / D;
            uint64_t key = make_key(depth, id);
            if (key < vis[p]) vis[p] = key;
        }
    }
}

/* Full per-triangle definition: near rejection, clipping, fan, snapping, rasterization. */
static void raster_triangle(const cvert c[3], uint64_t id, const vctx* vc, uint64_t* vis)
{
    if (c[0].w < vc->near_plane && c[1].w < vc->near_plane && c[2].w < vc->near_plane) return;
    if (!needs_clip(c, vc->near_plane)) {
        svert s[3];
        for (int k = 0; k < 3; ++k)
            if (!snap(c[k], vc, &s[k])) return;
        raster_snapped(s, id, vc, vis);
        return;
    }
    cvert poly[8];
    int n = clip_polygon(c, vc->near_plane, poly);
    if (n < 3) return;
    svert sp[8];
    for (int k = 0; k < n; ++k)
        if (!snap(poly[k], vc, &sp[k])) return;
    for (int j = 1; j + 1 < n; ++j) {
        svert s[3] = {sp[0], sp[j], sp[j + 1]};
        raster_snapped(s, id, vc, vis);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* (mesh, instance) pairs and global IDs                                                      */
/* ------------------------------------------------------------------------------------------ */
int64_t orc_num_pairs(const orc_mesh* meshes, uint32_t M)
{
    int64_t n = 0;
    for (uint32_t m = 0; m < M; ++m) n += meshes[m].inst ? meshes[m].N : 1;
    return n;
}

int orc_id_bases(const orc_mesh* meshes, uint32_t M, int64_t* bases)
{
    if (!meshes && M) return -1;
    int64_t acc = 0, p = 0;
    for (uint32_t m = 0; m < M; ++m) {
        uint32_t n = meshes[m].inst ? meshes[m].N : 1;
        for (uint32_t i = 0; i < n; ++i) {
            bases[p++] = acc;
            acc += (int64_t)meshes[m].T;
        }
    }
    bases[p] = acc;
    return 0;
}

int orc_decode_id(const orc_mesh* meshes, uint32_t M, const int64_t* bases, int64_t id,
                  uint32_t* mesh, uint32_t* inst, uint64_t* tri)
{
    int64_t np = orc_num_pairs(meshes, M);
    if (np == 0 || id < 0 || id >= bases[np]) return -1;
    /* largest pair index p with bases[p] <= id, among pairs with triangles */
    int64_t lo = 0, hi = np; /* invariant: bases[lo] <= id < bases[hi] */
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (bases[mid] <= id) lo = mid; else hi = mid;
    }
    int64_t p = 0;
    for (uint32_t m = 0; m < M; ++m) {
        int64_t n = meshes[m].inst ? meshes[m].N : 1;
        if (lo < p + n) {
            *mesh = m;
            *inst = (uint32_t)(lo - p);
            *tri = (uint64_t)(id - bases[lo]);
            return 0;
        }
        p += n;
    }
    return -1;
}

/* ------------------------------------------------------------------------------------------ */
/* Threaded driver                                                                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    uint32_t mesh;
    float A[3][4];
    int64_t base;
    uint64_t t0, t1;   /* triangle range of this pair that is processed */
    uint64_t work0;    /* flattened work offset */
} pair_t;

typedef struct {
    const orc_mesh* meshes;
    const pair_t* pairs;
    int64_t npairs;
    const vctx* vc;
    uint64_t w0, w1;
    uint64_t* vis;
} job_t;

static void* worker(void* arg)
{
    job_t* j = (job_t*)arg;
    for (int64_t p = 0; p < j->npairs; ++p) {
        const pair_t* pr = &j->pairs[p];
        uint64_t cnt = pr->t1 - pr->t0;
        uint64_t a = pr->work0, b = pr->work0 + cnt;
        if (b <= j->w0 || a >= j->w1) continue;
        uint64_t s = (j->w0 > a ? j->w0 : a) - a + pr->t0;
        uint64_t e = (j->w1 < b ? j->w1 : b) - a + pr->t0;
        const orc_mesh* me = &j->meshes[pr->mesh];
        for (uint64_t t = s; t < e; ++t) {
            cvert c[3];
            for (int k = 0; k < 3; ++k) {
                uint32_t vi = me->idx[3 * t + (uint64_t)k];
                if (vi >= me->V) goto next;     /* out-of-range index: no fragments */
                c[k] = transform(pr->A, me->pos + 3 * (uint64_t)vi);
            }
            raster_triangle(c, (uint64_t)pr->base + t, j->vc, j->vis);
        next:;
        }
    }
    return NULL;
}

static int resolve_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

static int run(const orc_mesh* meshes, uint32_t M, const orc_view* view, int64_t pb, int64_t pe, uint64_t tb, uint64_t te, uint64_t* vis, int nthreads)
{
    if (!view_ok(view) || !vis || (M && !meshes)) return -1;
    vctx vc = make_vctx(view);
    size_t npix = (size_t)vc.W * (size_t)vc.H;
    for (size_t i = 0; i < npix; ++i) vis[i] = ~(uint64_t)0;
    int64_t np = orc_num_pairs(meshes, M);
    if (pe > np) pe = np;
    if (pb < 0) pb = 0;
    if (pe <= pb) return 0;
    pair_t* pairs = (pair_t*)calloc((size_t)(pe - pb), sizeof(pair_t));
    if (!pairs) return -2;
    int64_t p = 0, base = 0, k = 0;
    uint64_t work = 0;
    for (uint32_t m = 0; m < M; ++m) {
        uint32_t n = meshes[m].inst ? meshes[m].N : 1;
        for (uint32_t i = 0; i < n; ++i, ++p) {
            if (p >= pb && p < pe) {
                pair_t* pr = &pairs[k++];
                pr->mesh = m;
                draw_matrix(view->vp, meshes[m].inst ? meshes[m].inst + 12 * (size_t)i : NULL, pr->A);
                pr->base = base;
                pr->t0 = tb < meshes[m].T ? tb : meshes[m].T;
                pr->t1 = te < meshes[m].T ? te : meshes[m].T;
                if (pr->t1 < pr->t0) pr->t1 = pr->t0;
                pr->work0 = work;
                work += pr->t1 - pr->t0;
            }
            base += (int64_t)meshes[m].T;
        }
    }
    int nt = resolve_threads(nthreads);
    if ((uint64_t)nt > work) nt = work ? (int)work : 1;
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    job_t* jobs = (job_t*)calloc((size_t)nt, sizeof(job_t));
    uint64_t** bufs = (uint64_t**)calloc((size_t)nt, sizeof(uint64_t*));
    int rc = 0;
    if (!th || !jobs || !bufs) { rc = -2; goto done; }
    for (int t = 0; t < nt; ++t) {
        jobs[t].meshes = meshes;
        jobs[t].pairs = pairs;
        jobs[t].npairs = k;
        jobs[t].vc = &vc;
        jobs[t].w0 = work * (uint64_t)t / (uint64_t)nt;
        jobs[t].w1 = work * (uint64_t)(t + 1) / (uint64_t)nt;
        if (t == 0) {
            jobs[t].vis = vis;
        } else {
            bufs[t] = (uint64_t*)malloc(npix * sizeof(uint64_t));
            if (!bufs[t]) { rc = -2; nt = t; break; }
            for (size_t i = 0; i < npix; ++i) bufs[t][i] = ~(uint64_t)0;
            jobs[t].vis = bufs[t];
        }
    }
    if (rc == 0) {
        for (int t = 1; t < nt; ++t) pthread_create(&th[t], NULL, worker, &jobs[t]);
        worker(&jobs[0]);
        for (int t = 1; t < nt; ++t) pthread_join(th[t], NULL);
        for (int t = 1; t < nt; ++t)
            for (size_t i = 0; i < npix; ++i)
                if (bufs[t][i] < vis[i]) vis[i] = bufs[t][i];
    }
done:
    if (bufs)
        for (int t = 0; t < nt; ++t) free(bufs[t]);
    free(bufs);
    free(jobs);
    free(th);
    free(pairs);
    return rc;
}

int orc_rasterize(const orc_mesh* meshes, uint32_t M, const orc_view* view, uint64_t* vis, int nthreads)
{
    return run(meshes, M, view, 0, INT64_MAX, 0, UINT64_MAX, vis, nthreads);
}

int orc_rasterize_range(const orc_mesh* meshes, uint32_t M, const orc_view* view,
                        int64_t pair_begin, int64_t pair_end, uint64_t tri_begin, uint64_t tri_end,
                        uint64_t* vis, int nthreads)
{
    return run(meshes, M, view, pair_begin, pair_end, tri_begin, tri_end, vis, nthreads);
}

/* ------------------------------------------------------------------------------------------ */
/* Coverage counting (fill-rule pins)                                                         */
/* ------------------------------------------------------------------------------------------ */
static void count_snapped(const svert v[3], const vctx* vc, uint32_t* front, uint32_t* back)
{
    int64_t area = (v[1].X - v[0].X) * (v[2].Y - v[0].Y) - (v[1].Y - v[0].Y) * (v[2].X - v[0].X);
    if (area == 0) return;
    svert u[3] = {v[0], v[1], v[2]};
    uint32_t* cnt = front;
    if (area < 0) {           /* test the reversed (counter-clockwise) triangle */
        u[1] = v[2];
        u[2] = v[1];
        cnt = back;
    }
    int64_t minX = u[0].X, maxX = u[0].X, minY = u[0].Y, maxY = u[0].Y;
    for (int k = 1; k < 3; ++k) {
        if (u[k].X < minX) minX = u[k].X;
        if (u[k].X > maxX) maxX = u[k].X;
        if (u[k].Y < minY) minY = u[k].Y;
        if (u[k].Y > maxY) maxY = u[k].Y;
    }
    int64_t px0 = -floor_div(128 - minX, 256), px1 = floor_div(maxX - 128, 256);
    int64_t py0 = -floor_div(128 - minY, 256), py1 = floor_div(maxY - 128, 256);
    if (px0 < 0) px0 = 0;
    if (py0 < 0) py0 = 0;
    if (px1 > vc->W - 1) px1 = vc->W - 1;
    if (py1 > vc->H - 1) py1 = vc->H - 1;
    for (int64_t py = py0; py <= py1; ++py)
        for (int64_t px = px0; px <= px1; ++px) {
            int64_t Px = 256 * px + 128, Py = 256 * py + 128;
            int inside = 1;
            for (int k = 0; k < 3; ++k) {
                const svert* a = &u[(k + 1) % 3];
                const svert* b = &u[(k + 2) % 3];
                int64_t dx = b->X - a->X, dy = b->Y - a->Y;
                int64_t E = dx * (Py - a->Y) - dy * (Px - a->X);
                if (!(E > 0 || (E == 0 && is_top_left(dx, dy)))) inside = 0;
            }
            if (inside) cnt[(size_t)py * (size_t)vc->W + (size_t)px] += 1;
        }
}

int orc_coverage_counts(const orc_mesh* meshes, uint32_t M, const orc_view* view,
                        uint32_t* front, uint32_t* back)
{
    if (!view_ok(view) || !front || !back) return -1;
    vctx vc = make_vctx(view);
    size_t npix = (size_t)vc.W * (size_t)vc.H;
    memset(front, 0, npix * sizeof(uint32_t));
    memset(back, 0, npix * sizeof(uint32_t));
    for (uint32_t m = 0; m < M; ++m) {
        uint32_t n = meshes[m].inst ? meshes[m].N : 1;
        for (uint32_t i = 0; i < n; ++i) {
            float A[3][4];
            draw_matrix(view->vp, meshes[m].inst ? meshes[m].inst + 12 * (size_t)i : NULL, A);
            for (uint64_t t = 0; t < meshes[m].T; ++t) {
                cvert c[3];
                int bad = 0;
                for (int k = 0; k < 3; ++k) {
                    const uint32_t vi = meshes[m].idx[3 * t + (uint64_t)k];
                    if (vi >= meshes[m].V) bad = 1;     /* out-of-range index: no fragments (R14) */
                    else c[k] = transform(A, meshes[m].pos + 3 * (uint64_t)vi);
                }
                if (bad) continue;
                if (c[0].w < vc.near_plane && c[1].w < vc.near_plane && c[2].w < vc.near_plane) continue;
                cvert poly[8];
                int nv;
                if (needs_clip(c, vc.near_plane)) {
                    nv = clip_polygon(c, vc.near_plane, poly);
                } else {
                    memcpy(poly, c, sizeof(cvert) * 3);
                    nv = 3;
                }
                if (nv < 3) continue;
                svert sp[8];
                int ok = 1;
                for (int k = 0; k < nv; ++k) ok &= snap(poly[k], &vc, &sp[k]);
                if (!ok) continue;
                for (int j = 1; j + 1 < nv; ++j) {
                    svert s[3] = {sp[0], sp[j], sp[j + 1]};
                    count_snapped(s, &vc, front, back);
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Screen positions                                                                           */
/* ------------------------------------------------------------------------------------------ */
int orc_project(const orc_mesh* mesh, uint32_t instance, const orc_view* view, float* pos_ss)
{
    if (!mesh || !view_ok(view) || !pos_ss) return -1;
    uint32_t n = mesh->inst ? mesh->N : 1;
    if (instance >= n) return -1;
    float A[3][4];
    draw_matrix(view->vp, mesh->inst ? mesh->inst + 12 * (size_t)instance : NULL, A);
    vctx vc = make_vctx(view);
    for (uint32_t v = 0; v < mesh->V; ++v) {
        cvert c = transform(A, mesh->pos + 3 * (size_t)v);
        float zI = 1.0f / c.w;
        pos_ss[3 * (size_t)v + 0] = fmaf(c.x * zI, vc.hW, vc.hW);
        pos_ss[3 * (size_t)v + 1] = fmaf(c.y * zI, vc.hH, vc.hH);
        pos_ss[3 * (size_t)v + 2] = c.w;
    }
    return 0;
}

/* Exposed for resolve.c: the same draw-matrix and transform definitions. */
void orc_internal_draw_matrix(const float vp[16], const float* inst, float A[3][4])
{
    draw_matrix(vp, inst, A);
}

void orc_internal_transform(const float A[3][4], const float* p, float out[3])
{
    cvert c = transform(A, p);
    out[0] = c.x;
    out[1] = c.y;
    out[2] = c.w;
}

/*
 * Oracle resolve pass (test infrastructure only, see oracle.h).
 *
 * Sec. 4.4: one pixel at a time, decode the 28-bit depth / 36-bit global triangle ID, find the
 * mesh/instance by binary search over the int64 exclusive prefix of triangle counts, reload the
 * triangle and interpolate its vertex attributes.  The paper shades in world space (ray-plane
 * intersection); the screen-space form used here, barycentrics proportional to lambda_k / w_k
 * of the projected vertices, is the same perspective-correct interpolation written with the
 * already projected positions, and it stays valid for vertices behind the camera.
 *
 * The backward pass is not in the paper: with visibility held fixed, the output of a pixel is a
 * rational function of the screen positions (sx, sy, w) of its triangle's three vertices and
 * linear in their attributes; its derivatives are written out below in fp64.
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

/* fp32 barycentric interpolation at pixel (px, py) from screen positions (sx, sy, w). */
static void interp_f32(const float s[3][3], int px, int py, const float* a0, const float* a1,
                       const float* a2, uint32_t C, float* out)
{
    const float cx = (float)px + 0.5f, cy = (float)py + 0.5f;
    float dx[3], dy[3], zI[3];
    for (int k = 0; k < 3; ++k) {
        dx[k] = s[k][0] - cx;
        dy[k] = s[k][1] - cy;
        zI[k] = 1.0f / s[k][2];
    }
    float l0 = dx[1] * dy[2] - dy[1] * dx[2];
    float l1 = dx[2] * dy[0] - dy[2] * dx[0];
    float l2 = dx[0] * dy[1] - dy[0] * dx[1];
    float q0 = l0 * zI[0], q1 = l1 * zI[1], q2 = l2 * zI[2];
    float sum = (q0 + q1) + q2;
    float b0 = q0 / sum, b1 = q1 / sum, b2 = q2 / sum;
    for (uint32_t c = 0; c < C; ++c) out[c] = (b0 * a0[c] + b1 * a1[c]) + b2 * a2[c];
}

typedef struct {
    const orc_mesh* meshes;
    uint32_t M;
    const orc_view* view;
    const uint64_t* vis;
    const float* const* attrs;
    uint32_t C;
    float* out;
    const int64_t* bases;
    const uint32_t* pair_mesh;
    const uint32_t* pair_inst;
    int64_t npairs;
    float (*A)[3][4];
    int32_t y0, y1;
} rjob;

static void* resolve_rows(void* arg)
{
    rjob* j = (rjob*)arg;
    const int32_t W = j->view->width;
    const float hW = 0.5f * (float)j->view->width, hH = 0.5f * (float)j->view->height;
    for (int32_t py = j->y0; py < j->y1; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const size_t p = (size_t)py * (size_t)W + (size_t)px;
            float* o = j->out + p * j->C;
            const uint64_t key = j->vis[p];
            memset(o, 0, sizeof(float) * j->C);
            if (key == EMPTY) continue;
            const int64_t id = (int64_t)(key & ID_MASK);
            if (id >= j->bases[j->npairs]) continue;
            int64_t lo = 0, hi = j->npairs;
            while (hi - lo > 1) {
                int64_t mid = lo + (hi - lo) / 2;
                if (j->bases[mid] <= id) lo = mid; else hi = mid;
            }
            const orc_mesh* me = &j->meshes[j->pair_mesh[lo]];
            const uint64_t t = (uint64_t)(id - j->bases[lo]);
            float s[3][3];
            const float* a[3];
            int bad = 0;
            for (int k = 0; k < 3; ++k) {
                const uint32_t vi = me->idx[3 * t + (uint64_t)k];
                if (vi >= me->V) { bad = 1; break; }
                float c[3];
                orc_internal_transform(j->A[lo], me->pos + 3 * (size_t)vi, c);
                const float zI = 1.0f / c[2];
                s[k][0] = fmaf(c[0] * zI, hW, hW);
                s[k][1] = fmaf(c[1] * zI, hH, hH);
                s[k][2] = c[2];
                a[k] = j->attrs[j->pair_mesh[lo]] + (size_t)vi * j->C;
            }
            if (bad) continue;
            interp_f32(s, px, py, a[0], a[1], a[2], j->C, o);
        }
    return NULL;
}

int orc_resolve(const orc_mesh* meshes, uint32_t M, const orc_view* view, const uint64_t* vis,
                const float* const* attrs, uint32_t C, float* out, int nthreads)
{
    if (!view || !vis || !attrs || !out || C == 0 || view->width <= 0 || view->height <= 0) return -1;
    int64_t np = orc_num_pairs(meshes, M);
    int64_t* bases = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np + 1));
    uint32_t* pm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(np + 1));
    uint32_t* pi = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(np + 1));
    float(*A)[3][4] = malloc(sizeof(float[3][4]) * (size_t)(np + 1));
    if (!bases || !pm || !pi || !A) { free(bases); free(pm); free(pi); free(A); return -2; }
    orc_id_bases(meshes, M, bases);
    int64_t p = 0;
    for (uint32_t m = 0; m < M; ++m) {
        uint32_t n = meshes[m].inst ? meshes[m].N : 1;
        for (uint32_t i = 0; i < n; ++i, ++p) {
            pm[p] = m;
            pi[p] = i;
            orc_internal_draw_matrix(view->vp, meshes[m].inst ? meshes[m].inst + 12 * (size_t)i : NULL, A[p]);
        }
    }
    int nt = nthreads > 0 ? nthreads : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > view->height) nt = view->height;
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    rjob* jobs = (rjob*)calloc((size_t)nt, sizeof(rjob));
    for (int t = 0; t < nt; ++t) {
        rjob j = {meshes, M, view, vis, attrs, C, out, bases, pm, pi, np, A,
                  (int32_t)((int64_t)view->height * t / nt), (int32_t)((int64_t)view->height * (t + 1) / nt)};
        jobs[t] = j;
        if (t) pthread_create(&th[t], NULL, resolve_rows, &jobs[t]);
    }
    resolve_rows(&jobs[0]);
    for (int t = 1; t < nt; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    free(bases);
    free(pm);
    free(pi);
    free(A);
    return 0;
}

int orc_resolve_screen(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                       int64_t id_base, const float* pos_ss, uint32_t V, const float* attrs,
                       uint32_t C, float* out)
{
    if (!vis || !idx || !pos_ss || !attrs || !out || W <= 0 || H <= 0 || C == 0) return -1;
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const size_t p = (size_t)py * (size_t)W + (size_t)px;
            float* o = out + p * C;
            memset(o, 0, sizeof(float) * C);
            const uint64_t key = vis[p];
            if (key == EMPTY) continue;
            const int64_t id = (int64_t)(key & ID_MASK);
            if (id < id_base || id - id_base >= (int64_t)T) continue;
            const uint64_t t = (uint64_t)(id - id_base);
            float s[3][3];
            const float* a[3];
            int bad = 0;
            for (int k = 0; k < 3; ++k) {
                const uint32_t vi = idx[3 * t + (uint64_t)k];
                if (vi >= V) { bad = 1; break; }
                for (int c = 0; c < 3; ++c) s[k][c] = pos_ss[3 * (size_t)vi + (size_t)c];
                a[k] = attrs + (size_t)vi * C;
            }
            if (!bad) interp_f32(s, px, py, a[0], a[1], a[2], C, o);
        }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* fp64 forward, analytic backward and finite differences                                      */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    double d[3][2], zI[3], lam[3], q[3], s, b[3];
} f64pix;

static void pix_f64(const double S[3][3], int px, int py, f64pix* r)
{
    const double cx = px + 0.5, cy = py + 0.5;
    for (int k = 0; k < 3; ++k) {
        r->d[k][0] = S[k][0] - cx;
        r->d[k][1] = S[k][1] - cy;
        r->zI[k] = 1.0 / S[k][2];
    }
    r->lam[0] = r->d[1][0] * r->d[2][1] - r->d[1][1] * r->d[2][0];
    r->lam[1] = r->d[2][0] * r->d[0][1] - r->d[2][1] * r->d[0][0];
    r->lam[2] = r->d[0][0] * r->d[1][1] - r->d[0][1] * r->d[1][0];
    r->s = 0.0;
    for (int k = 0; k < 3; ++k) {
        r->q[k] = r->lam[k] * r->zI[k];
        r->s += r->q[k];
    }
    for (int k = 0; k < 3; ++k) r->b[k] = r->q[k] / r->s;
}

static int pixel_tri(const uint64_t key, const uint32_t* idx, uint64_t T, int64_t id_base,
                     uint32_t V, uint32_t vi[3])
{
    if (key == EMPTY) return 0;
    const int64_t id = (int64_t)(key & ID_MASK);
    if (id < id_base || id - id_base >= (int64_t)T) return 0;
    const uint64_t t = (uint64_t)(id - id_base);
    for (int k = 0; k < 3; ++k) {
        vi[k] = idx[3 * t + (uint64_t)k];
        if (vi[k] >= V) return 0;
    }
    return 1;
}

int orc_resolve_screen_f64(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                           int64_t id_base, const double* pos_ss, uint32_t V, const double* attrs,
                           uint32_t C, double* out)
{
    if (!vis || !idx || !pos_ss || !attrs || !out || W <= 0 || H <= 0 || C == 0) return -1;
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const size_t p = (size_t)py * (size_t)W + (size_t)px;
            double* o = out + p * C;
            for (uint32_t c = 0; c < C; ++c) o[c] = 0.0;
            uint32_t vi[3];
            if (!pixel_tri(vis[p], idx, T, id_base, V, vi)) continue;
            double S[3][3];
            for (int k = 0; k < 3; ++k)
                for (int c = 0; c < 3; ++c) S[k][c] = pos_ss[3 * (size_t)vi[k] + (size_t)c];
            f64pix r;
            pix_f64(S, px, py, &r);
            for (uint32_t c = 0; c < C; ++c)
                for (int k = 0; k < 3; ++k) o[c] += r.b[k] * attrs[(size_t)vi[k] * C + c];
        }
    return 0;
}

int orc_resolve_screen_backward_f64(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx,
                                    uint64_t T, int64_t id_base, const double* pos_ss, uint32_t V,
                                    const double* attrs, uint32_t C, const double* grad_out,
                                    double* grad_attr, double* grad_pos)
{
    if (!vis || !idx || !pos_ss || !attrs || !grad_out || W <= 0 || H <= 0 || C == 0) return -1;
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const size_t p = (size_t)py * (size_t)W + (size_t)px;
            uint32_t vi[3];
            if (!pixel_tri(vis[p], idx, T, id_base, V, vi)) continue;
            const double* g = grad_out + p * C;
            double S[3][3];
            for (int k = 0; k < 3; ++k)
                for (int c = 0; c < 3; ++c) S[k][c] = pos_ss[3 * (size_t)vi[k] + (size_t)c];
            f64pix r;
            pix_f64(S, px, py, &r);
            /* dL/da_k = g * b_k */
            if (grad_attr)
                for (int k = 0; k < 3; ++k)
                    for (uint32_t c = 0; c < C; ++c) grad_attr[(size_t)vi[k] * C + c] += g[c] * r.b[k];
            if (!grad_pos) continue;
            /* dL/db_k = G_k = sum_c g_c a_kc ; dL/dq_j = (G_j - sum_k G_k b_k) / s */
            double G[3], Gb = 0.0;
            for (int k = 0; k < 3; ++k) {
                G[k] = 0.0;
                for (uint32_t c = 0; c < C; ++c) G[k] += g[c] * attrs[(size_t)vi[k] * C + c];
                Gb += G[k] * r.b[k];
            }
            double Lm[3], dw[3];
            for (int j = 0; j < 3; ++j) {
                const double Q = (G[j] - Gb) / r.s;
                Lm[j] = Q * r.zI[j];                         /* dL/dlambda_j */
                dw[j] = -(Q * r.lam[j]) * r.zI[j] * r.zI[j];  /* dL/dw_j through zI_j = 1/w_j */
            }
            const double (*d)[2] = r.d;
            /* lambda_0 = d1 x d2, lambda_1 = d2 x d0, lambda_2 = d0 x d1 */
            double gx[3], gy[3];
            gx[0] = -Lm[1] * d[2][1] + Lm[2] * d[1][1];
            gy[0] = Lm[1] * d[2][0] - Lm[2] * d[1][0];
            gx[1] = Lm[0] * d[2][1] - Lm[2] * d[0][1];
            gy[1] = -Lm[0] * d[2][0] + Lm[2] * d[0][0];
            gx[2] = -Lm[0] * d[1][1] + Lm[1] * d[0][1];
            gy[2] = Lm[0] * d[1][0] - Lm[1] * d[0][0];
            for (int k = 0; k < 3; ++k) {
                grad_pos[3 * (size_t)vi[k] + 0] += gx[k];
                grad_pos[3 * (size_t)vi[k] + 1] += gy[k];
                grad_pos[3 * (size_t)vi[k] + 2] += dw[k];
            }
        }
    return 0;
}

static double pixel_loss(const double S[3][3], int px, int py, const double* a[3], uint32_t C,
                         const double* target)
{
    f64pix r;
    pix_f64(S, px, py, &r);
    double l = 0.0;
    for (uint32_t c = 0; c < C; ++c) {
        double o = 0.0;
        for (int k = 0; k < 3; ++k) o += r.b[k] * a[k][c];
        const double e = o - target[c];
        l += e * e;
    }
    return l;
}

int orc_fd_pos_grad_l2(const uint64_t* vis, int32_t W, int32_t H, const uint32_t* idx, uint64_t T,
                       int64_t id_base, const double* pos_ss, uint32_t V, const double* attrs,
                       uint32_t C, const double* target, const uint32_t* verts, uint32_t n,
                       double eps, int order4, double* fd)
{
    if (!vis || !idx || !pos_ss || !attrs || !target || !verts || !fd || C == 0) return -1;
    int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
    if (!slot) return -2;
    for (uint32_t v = 0; v < V; ++v) slot[v] = -1;
    for (uint32_t i = 0; i < n; ++i) {
        if (verts[i] >= V) { free(slot); return -1; }
        slot[verts[i]] = (int32_t)i;
    }
    memset(fd, 0, sizeof(double) * 3 * (size_t)n);
    for (int32_t py = 0; py < H; ++py)
        for (int32_t px = 0; px < W; ++px) {
            const size_t p = (size_t)py * (size_t)W + (size_t)px;
            uint32_t vi[3];
            if (!pixel_tri(vis[p], idx, T, id_base, V, vi)) continue;
            double S[3][3];
            const double* a[3];
            for (int k = 0; k < 3; ++k) {
                for (int c = 0; c < 3; ++c) S[k][c] = pos_ss[3 * (size_t)vi[k] + (size_t)c];
                a[k] = attrs + (size_t)vi[k] * C;
            }
            for (int k = 0; k < 3; ++k) {
                const int32_t sl = slot[vi[k]];
                if (sl < 0) continue;
                /* a vertex repeated in one (degenerate) triangle is handled once, at its first corner */
                if ((k >= 1 && vi[k] == vi[0]) || (k == 2 && vi[2] == vi[1])) continue;
                for (int c = 0; c < 3; ++c) {
                    /* central differences at +-eps and +-2eps (fourth-order stencil) */
                    double l[4];
                    static const double steps[4] = {1.0, -1.0, 2.0, -2.0};
                    for (int st = 0; st < 4; ++st) {
                        double Sx[3][3];
                        memcpy(Sx, S, sizeof S);
                        for (int kk = 0; kk < 3; ++kk)
                            if (vi[kk] == vi[k]) Sx[kk][c] += steps[st] * eps;
                        l[st] = pixel_loss(Sx, px, py, a, C, target + p * C);
                    }
                    const double d1 = (l[0] - l[1]) / (2.0 * eps);
                    const double d2 = (l[2] - l[3]) / (4.0 * eps);
                    fd[3 * (size_t)sl + (size_t)c] += order4 ? (4.0 * d1 - d2) / 3.0 : d1;
                }
            }
        }
    free(slot);
    return 0;
}

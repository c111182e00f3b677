/*
 * Brute-force transcription of the visibility-buffer definition (test infrastructure only, see
 * oracle.h).  Written separately from raster.c and sharing none of its code: every triangle is
 * tested against every pixel centre of the image, with no bounding box, no tiny-triangle test
 * and no early exits, so that comparing the two on small inputs pins raster.c's traversal and
 * bounds logic, and two independent transcriptions of the arithmetic must agree bit for bit.
 *
 * Paper passages: Sec. 3.1 (atomicMin of depth|ID keys), Sec. 4 (cumulative triangle IDs),
 * Sec. 4.1 (projection, culling, 28/36-bit key, perspective-correct depth), Sec. 4.2 (clipping).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct { float v[3]; } bv3;        /* clip-space x, y, w */

static float bdot_row(const float* r, const float* X, int c)
{
    /* ((r0*X0c + r1*X1c) + r2*X2c): the draw-matrix element order */
    float s = r[0] * X[c];
    s = s + r[1] * X[4 + c];
    s = s + r[2] * X[8 + c];
    return s;
}

static void bdraw(const float* vp, const float* inst, float A[12])
{
    float I[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    const float* X = inst ? inst : I;
    const float* rows[3] = {vp, vp + 4, vp + 12};
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) A[4 * r + c] = bdot_row(rows[r], X, c);
        A[4 * r + 3] = bdot_row(rows[r], X, 3) + rows[r][3];
    }
}

static bv3 bxf(const float A[12], const float* p)
{
    bv3 o;
    for (int r = 0; r < 3; ++r)
        o.v[r] = fmaf(A[4 * r], p[0], fmaf(A[4 * r + 1], p[1], fmaf(A[4 * r + 2], p[2], A[4 * r + 3])));
    return o;
}

/* plane distances: near, x >= -16w, x <= 16w, y >= -16w, y <= 16w */
static float bdist(const bv3* q, int k, float n)
{
    const float g = 16.0f * q->v[2];
    if (k == 0) return q->v[2] - n;
    if (k == 1) return q->v[0] + g;
    if (k == 2) return g - q->v[0];
    if (k == 3) return q->v[1] + g;
    return g - q->v[1];
}

static int bclip(bv3* poly, int n, float nearp)
{
    for (int k = 0; k < 5 && n >= 3; ++k) {
        bv3 out[8];
        int m = 0;
        for (int i = 0; i < n; ++i) {
            const bv3* a = &poly[i];
            const bv3* b = &poly[i + 1 < n ? i + 1 : 0];
            const float da = bdist(a, k, nearp), db = bdist(b, k, nearp);
            if (da >= 0.0f) out[m++] = *a;
            if ((da >= 0.0f) == (db >= 0.0f)) continue;
            const bv3* in = da >= 0.0f ? a : b;
            const bv3* ou = da >= 0.0f ? b : a;
            const float din = da >= 0.0f ? da : db;
            const float dou = da >= 0.0f ? db : da;
            const float t = din / (din - dou);
            for (int c = 0; c < 3; ++c) out[m].v[c] = fmaf(t, ou->v[c] - in->v[c], in->v[c]);
            ++m;
        }
        memcpy(poly, out, sizeof(bv3) * (size_t)m);
        n = m;
    }
    return n >= 3 ? n : 0;
}

static void bfrag(const int64_t X[3], const int64_t Y[3], const float zi[3], uint64_t id,
                  int W, int H, uint64_t* vis)
{
    const int64_t A2 = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
    if (A2 <= 0) return;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            const int64_t sx = 256 * (int64_t)px + 128, sy = 256 * (int64_t)py + 128;
            int64_t e[3];
            int ok = 1;
            for (int k = 0; k < 3; ++k) {
                const int i1 = (k + 1) % 3, i2 = (k + 2) % 3;
                const int64_t ex = X[i2] - X[i1], ey = Y[i2] - Y[i1];
                e[k] = ex * (sy - Y[i1]) - ey * (sx - X[i1]);
                const int tl = (ey < 0) || (ey == 0 && ex < 0);
                if (e[k] < 0 || (e[k] == 0 && !tl)) ok = 0;
            }
            if (!ok) continue;
            const float d = (float)A2 / fmaf((float)e[2], zi[2], fmaf((float)e[1], zi[1], (float)e[0] * zi[0]));
            uint32_t u;
            memcpy(&u, &d, sizeof u);
            const uint64_t key = ((uint64_t)(u >> 3) << 36) | (id & 0xFFFFFFFFFull);
            uint64_t* dst = &vis[(size_t)py * (size_t)W + (size_t)px];
            if (key < *dst) *dst = key;
        }
}

int orc_rasterize_brute(const orc_mesh* meshes, uint32_t M, const orc_view* view, uint64_t* vis)
{
    if (!view || !vis || view->width <= 0 || view->height <= 0 || !(view->near_plane > 0.0f)) return -1;
    const int W = view->width, H = view->height;
    const float hw = 0.5f * (float)W, hh = 0.5f * (float)H, nearp = view->near_plane;
    for (size_t i = 0; i < (size_t)W * (size_t)H; ++i) vis[i] = ~0ull;
    uint64_t base = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const orc_mesh* me = &meshes[m];
        const uint32_t ninst = me->inst ? me->N : 1;
        for (uint32_t i = 0; i < ninst; ++i, base += me->T) {
            float A[12];
            bdraw(view->vp, me->inst ? me->inst + 12 * (size_t)i : NULL, A);
            for (uint64_t t = 0; t < me->T; ++t) {
                bv3 poly[8];
                int bad = 0;
                for (int k = 0; k < 3; ++k) {
                    const uint32_t vi = me->idx[3 * t + (uint64_t)k];
                    if (vi >= me->V) bad = 1;
                    else poly[k] = bxf(A, me->pos + 3 * (size_t)vi);
                }
                if (bad) continue;
                int behind = 0, outside = 0;
                for (int k = 0; k < 3; ++k) {
                    behind += poly[k].v[2] < nearp;
                    outside |= poly[k].v[2] < nearp || fabsf(poly[k].v[0]) > 16.0f * poly[k].v[2] ||
                               fabsf(poly[k].v[1]) > 16.0f * poly[k].v[2];
                }
                if (behind == 3) continue;
                const int n = outside ? bclip(poly, 3, nearp) : 3;
                int64_t X[8], Y[8];
                float zi[8];
                int fin = 1;
                for (int k = 0; k < n; ++k) {
                    zi[k] = 1.0f / poly[k].v[2];
                    const float fx = rintf(fmaf(poly[k].v[0] * zi[k], hw, hw) * 256.0f);
                    const float fy = rintf(fmaf(poly[k].v[1] * zi[k], hh, hh) * 256.0f);
                    if (!(fabsf(fx) < 1073741824.0f && fabsf(fy) < 1073741824.0f)) fin = 0;
                    else { X[k] = (int64_t)fx; Y[k] = (int64_t)fy; }
                }
                if (!fin) continue;
                for (int j = 1; j + 1 < n; ++j) {
                    const int64_t tx[3] = {X[0], X[j], X[j + 1]}, ty[3] = {Y[0], Y[j], Y[j + 1]};
                    const float tz[3] = {zi[0], zi[j], zi[j + 1]};
                    bfrag(tx, ty, tz, base + t, W, H, vis);
                }
            }
        }
    }
    return 0;
}

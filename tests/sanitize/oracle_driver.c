/*
 * Test driver for the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built and
 * run by tests/test_sanitize_host.py; test infrastructure only).  It calls every oracle entry point
 * on small synthetic scenes, edge cases included (empty meshes, indices >= V, degenerate and
 * near-plane-crossing triangles, a 1x1 view, instanced meshes), and the argument checks with
 * invalid inputs.  It exits non-zero when a result is inconsistent; the sanitizers abort on any
 * invalid access or undefined operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}
static float frand(float lo, float hi) { return lo + (hi - lo) * (float)(rnd() >> 8) * (1.0f / 16777216.0f); }

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            fprintf(stderr, "check failed at %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

/* row-major perspective * look-at (camera at e looking at t, y up), fovy 60 degrees */
static void camera(const float e[3], const float t[3], float aspect, float vp[16])
{
    float f[3] = {t[0] - e[0], t[1] - e[1], t[2] - e[2]};
    float n = sqrtf(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int i = 0; i < 3; ++i) f[i] /= n;
    float up[3] = {0.0f, 1.0f, 0.0f};
    float s[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    n = sqrtf(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    for (int i = 0; i < 3; ++i) s[i] /= n;
    float u[3] = {s[1] * f[2] - s[2] * f[1], s[2] * f[0] - s[0] * f[2], s[0] * f[1] - s[1] * f[0]};
    float V[16] = {s[0], s[1], s[2], -(s[0] * e[0] + s[1] * e[1] + s[2] * e[2]),
                   u[0], u[1], u[2], -(u[0] * e[0] + u[1] * e[1] + u[2] * e[2]),
                   -f[0], -f[1], -f[2], (f[0] * e[0] + f[1] * e[1] + f[2] * e[2]),
                   0, 0, 0, 1};
    const float c = 1.0f / tanf(0.5f * 1.0471976f), zn = 0.05f, zf = 100.0f;
    float P[16] = {c / aspect, 0, 0, 0, 0, c, 0, 0, 0, 0, (zf + zn) / (zn - zf), 2 * zf * zn / (zn - zf), 0, 0, -1, 0};
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k) {
            float acc = 0.0f;
            for (int j = 0; j < 4; ++j) acc += P[4 * r + j] * V[4 * j + k];
            vp[4 * r + k] = acc;
        }
}

typedef struct {
    float* pos;
    uint32_t* idx;
    float* inst;
    uint32_t V, N;
    uint64_t T;
} host_mesh;

static host_mesh grid(int n, float y0, int bad)
{
    host_mesh m = {0};
    m.V = (uint32_t)(n * n);
    m.T = 2ull * (uint64_t)(n - 1) * (uint64_t)(n - 1);
    m.pos = malloc(sizeof(float) * 3 * m.V);
    m.idx = malloc(sizeof(uint32_t) * 3 * m.T);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            float* p = m.pos + 3 * (r * n + c);
            p[0] = 4.0f * c / (n - 1) - 2.0f;
            p[1] = y0 + 0.2f * sinf(0.7f * r) * cosf(0.9f * c);
            p[2] = -4.0f * r / (n - 1) - 1.0f;
        }
    uint64_t t = 0;
    for (int r = 0; r + 1 < n; ++r)
        for (int c = 0; c + 1 < n; ++c) {
            uint32_t a = r * n + c, b = a + 1, d = a + n, e = d + 1;
            uint32_t* q = m.idx + 3 * t;
            q[0] = a; q[1] = d; q[2] = b;
            q[3] = b; q[4] = d; q[5] = e;
            t += 2;
        }
    if (bad) {   /* indices >= V, a degenerate triangle, a repeated vertex */
        m.idx[0] = m.V + 5;
        m.idx[7] = 0xFFFFFFFFu;
        m.idx[9] = m.idx[10] = m.idx[11];
    }
    m.N = 1;
    return m;
}

static host_mesh soup(uint32_t T, uint32_t N)
{
    host_mesh m = {0};
    m.V = 3 * T;
    m.T = T;
    m.pos = malloc(sizeof(float) * 3 * m.V + 1);
    m.idx = malloc(sizeof(uint32_t) * 3 * m.T + 1);
    for (uint32_t i = 0; i < m.V; ++i) {
        m.pos[3 * i] = frand(-1.5f, 1.5f);
        m.pos[3 * i + 1] = frand(-1.0f, 1.0f);
        m.pos[3 * i + 2] = frand(-3.0f, 0.5f);   /* some vertices behind the camera */
        m.idx[i] = i;
    }
    m.N = N;
    m.inst = malloc(sizeof(float) * 12 * N);
    for (uint32_t k = 0; k < N; ++k) {
        float a = frand(0.0f, 6.2831853f), s = frand(0.5f, 1.5f);
        float* X = m.inst + 12 * k;
        float R[12] = {s * cosf(a), 0, s * sinf(a), frand(-0.5f, 0.5f), 0, s, 0, frand(-0.3f, 0.3f),
                       -s * sinf(a), 0, s * cosf(a), frand(-1.0f, 0.0f)};
        memcpy(X, R, sizeof R);
    }
    return m;
}

static orc_mesh as_orc(const host_mesh* h)
{
    orc_mesh m = {h->pos, h->V, h->idx, h->T, h->inst, h->N};
    return m;
}

static void scene(const orc_mesh* meshes, uint32_t M, const orc_view* view, const float* const* attrs)
{
    const int W = view->width, H = view->height;
    const size_t px = (size_t)W * H;
    uint64_t* vis = malloc(sizeof(uint64_t) * px);
    uint64_t* vis2 = malloc(sizeof(uint64_t) * px);
    uint64_t* vis3 = malloc(sizeof(uint64_t) * px);
    CHECK(orc_rasterize(meshes, M, view, vis, 1) == 0);
    CHECK(orc_rasterize(meshes, M, view, vis2, 3) == 0);
    CHECK(memcmp(vis, vis2, sizeof(uint64_t) * px) == 0);
    CHECK(orc_rasterize_brute(meshes, M, view, vis3) == 0);
    CHECK(memcmp(vis, vis3, sizeof(uint64_t) * px) == 0);
    const int64_t pairs = orc_num_pairs(meshes, M);
    CHECK(pairs >= 0);
    CHECK(orc_rasterize_range(meshes, M, view, 0, pairs, 0, UINT64_MAX, vis2, 2) == 0);
    CHECK(memcmp(vis, vis2, sizeof(uint64_t) * px) == 0);
    CHECK(orc_rasterize_range(meshes, M, view, 0, pairs, 3, 7, vis2, 1) == 0);
    uint32_t* front = malloc(sizeof(uint32_t) * px);
    uint32_t* back = malloc(sizeof(uint32_t) * px);
    CHECK(orc_coverage_counts(meshes, M, view, front, back) == 0);
    int64_t* bases = malloc(sizeof(int64_t) * (size_t)(pairs + 1));
    CHECK(orc_id_bases(meshes, M, bases) == 0);
    for (size_t p = 0; p < px; ++p) {
        if (vis[p] == UINT64_MAX) continue;
        const int64_t id = (int64_t)(vis[p] & ((1ull << 36) - 1));
        uint32_t mm, ii;
        uint64_t tt;
        CHECK(orc_decode_id(meshes, M, bases, id, &mm, &ii, &tt) == 0);
        CHECK(mm < M && ii < meshes[mm].N && tt < meshes[mm].T);
    }
    const uint32_t C = 3;
    float* out = malloc(sizeof(float) * px * C);
    CHECK(orc_resolve(meshes, M, view, vis, attrs, C, out, 2) == 0);
    for (uint32_t m = 0; m < M; ++m) {
        if (!meshes[m].V) continue;
        float* ss = malloc(sizeof(float) * 3 * meshes[m].V);
        double* ssd = malloc(sizeof(double) * 3 * meshes[m].V);
        double* ad = malloc(sizeof(double) * C * meshes[m].V);
        double* ga = calloc((size_t)C * meshes[m].V, sizeof(double));
        double* gp = calloc((size_t)3 * meshes[m].V, sizeof(double));
        double* outd = malloc(sizeof(double) * px * C);
        double* g = malloc(sizeof(double) * px * C);
        float* o32 = malloc(sizeof(float) * px * C);
        for (uint32_t i = 0; i < meshes[m].N; ++i) {
            const int64_t base = bases[orc_num_pairs(meshes, m) + i];
            CHECK(orc_project(&meshes[m], i, view, ss) == 0);
            for (uint64_t k = 0; k < 3ull * meshes[m].V; ++k) ssd[k] = ss[k];
            for (uint64_t k = 0; k < (uint64_t)C * meshes[m].V; ++k) ad[k] = attrs[m][k];
            for (size_t k = 0; k < px * C; ++k) g[k] = (double)((k * 7919u) % 13u) / 13.0 - 0.5;
            CHECK(orc_resolve_screen(vis, W, H, meshes[m].idx, meshes[m].T, base, ss, meshes[m].V, attrs[m], C, o32) == 0);
            CHECK(orc_resolve_screen_f64(vis, W, H, meshes[m].idx, meshes[m].T, base, ssd, meshes[m].V, ad, C, outd) == 0);
            CHECK(orc_resolve_screen_backward_f64(vis, W, H, meshes[m].idx, meshes[m].T, base, ssd, meshes[m].V, ad, C, g,
                                                  ga, gp) == 0);
            uint32_t verts[2] = {0, meshes[m].V - 1};
            double fd[6];
            CHECK(orc_fd_pos_grad_l2(vis, W, H, meshes[m].idx, meshes[m].T, base, ssd, meshes[m].V, ad, C, outd, verts, 2,
                                     1e-3, 1, fd) == 0);
        }
        free(ss); free(ssd); free(ad); free(ga); free(gp); free(outd); free(g); free(o32);
    }
    /* textures: one 8x4 chain per mesh, a textured resolve with planar UVs */
    const uint32_t tw = 8, th = 4, levels = 4;
    const uint64_t words = orc_texture_texels(tw, th, levels);
    CHECK(words > 0);
    uint32_t* tex = malloc(sizeof(uint32_t) * words);
    for (uint64_t k = 0; k < (uint64_t)tw * th; ++k) tex[k] = rnd();
    CHECK(orc_build_mips(tex, tw, th, levels) == 0);
    orc_texture* textures = malloc(sizeof(orc_texture) * M);
    const float** uvs = malloc(sizeof(float*) * M);
    for (uint32_t m = 0; m < M; ++m) {
        textures[m].texels = tex;
        textures[m].width = tw;
        textures[m].height = th;
        textures[m].levels = levels;
        float* uv = malloc(sizeof(float) * 2 * (meshes[m].V + 1));
        for (uint32_t v = 0; v < meshes[m].V; ++v) {
            uv[2 * v] = meshes[m].pos[3 * v];
            uv[2 * v + 1] = meshes[m].pos[3 * v + 2];
        }
        uvs[m] = uv;
    }
    float rgba[4];
    orc_sample_trilinear(&textures[0], 0.3f, -7.25f, 1.5f, rgba);
    orc_sample_trilinear(&textures[0], 1e6f, 0.5f, 40.0f, rgba);
    const float us[4] = {0.1f, 0.2f, 0.1f, 0.2f}, vs[4] = {0.5f, 0.5f, 0.6f, 0.6f};
    (void)orc_texture_lod(&textures[0], us, vs, 1);
    (void)orc_texture_lod(&textures[0], us, vs, 0);
    float* tout = malloc(sizeof(float) * px * 4);
    CHECK(orc_resolve_textured(meshes, M, view, vis, uvs, textures, tout, 2) == 0);
    for (uint32_t m = 0; m < M; ++m) free((void*)uvs[m]);
    free(uvs); free(textures); free(tex); free(tout);
    free(vis); free(vis2); free(vis3); free(front); free(back); free(bases); free(out);
}

int main(void)
{
    host_mesh g = grid(9, -0.6f, 0), gb = grid(6, -0.3f, 1), s = soup(40, 3), e = {0};
    e.N = 2;   /* an instanced mesh without triangles */
    e.inst = calloc(24, sizeof(float));
    e.inst[0] = e.inst[5] = e.inst[10] = 1.0f;
    e.inst[12] = e.inst[17] = e.inst[22] = 1.0f;
    orc_mesh meshes[4] = {as_orc(&g), as_orc(&e), as_orc(&gb), as_orc(&s)};
    float* attrs[4];
    for (int m = 0; m < 4; ++m) {
        attrs[m] = malloc(sizeof(float) * 3 * (meshes[m].V + 1));
        for (uint32_t k = 0; k < 3 * meshes[m].V; ++k) attrs[m][k] = frand(0.0f, 1.0f);
    }
    const float eye1[3] = {0.3f, 1.2f, 1.5f}, at1[3] = {0.0f, -0.5f, -2.5f};
    const float eye2[3] = {0.0f, -0.55f, -2.0f}, at2[3] = {0.5f, -0.6f, -4.0f};   /* inside the grid: near-plane crossings */
    orc_view views[3];
    camera(eye1, at1, 64.0f / 48.0f, views[0].vp);
    views[0].near_plane = 0.05f; views[0].width = 64; views[0].height = 48;
    camera(eye2, at2, 1.0f, views[1].vp);
    views[1].near_plane = 0.05f; views[1].width = 40; views[1].height = 40;
    camera(eye1, at1, 1.0f, views[2].vp);
    views[2].near_plane = 0.05f; views[2].width = 1; views[2].height = 1;
    for (int v = 0; v < 3; ++v) scene(meshes, 4, &views[v], (const float* const*)attrs);
    scene(meshes, 1, &views[0], (const float* const*)attrs);

    /* compressed positions round trip */
    const float lo[3] = {-2.0f, -1.0f, -5.0f}, step[3] = {4.0f / 65535.0f, 0.0f, 4.0f / 65535.0f};
    uint16_t* q = malloc(sizeof(uint16_t) * 3 * g.V);
    float* dec = malloc(sizeof(float) * 3 * g.V);
    CHECK(orc_quantize_positions(g.pos, g.V, lo, step, q) == 0);
    CHECK(orc_decode_positions(q, g.V, lo, step, dec) == 0);

    /* argument checks: invalid inputs return an error instead of touching memory */
    uint64_t one = 0;
    int64_t b2[2];
    CHECK(orc_rasterize(NULL, 1, &views[0], &one, 1) < 0);
    CHECK(orc_rasterize(meshes, 1, NULL, &one, 1) < 0);
    CHECK(orc_rasterize(meshes, 1, &views[0], NULL, 1) < 0);
    CHECK(orc_id_bases(NULL, 1, b2) < 0);
    CHECK(orc_texture_texels(3, 4, 1) == 0);
    CHECK(orc_texture_texels(4, 4, 9) == 0);
    orc_view bad = views[0];
    bad.width = 0;
    CHECK(orc_rasterize(meshes, 1, &bad, &one, 1) < 0);

    for (int m = 0; m < 4; ++m) free(attrs[m]);
    free(g.pos); free(g.idx); free(gb.pos); free(gb.idx); free(s.pos); free(s.idx); free(s.inst); free(e.inst);
    free(q); free(dec);
    printf("oracle driver: ok\n");
    return 0;
}

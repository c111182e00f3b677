/*
 * Test driver for the library's host-only entry points (curast_plan, curast_id_bases,
 * curast_texture_texels, curast_status_string, curast_version) under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitize_host.py from a host-only,
 * sanitized build of the library sources; test infrastructure only).  No GPU call is made: the
 * planning step validates its arguments, builds the draw list and the work items, and culls by
 * bounding sphere on the host.  Device pointers in the descriptors are never dereferenced here.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "curast.h"

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            fprintf(stderr, "check failed at %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

static void view_at(curast_view* v, float cx, float cz, int w, int h, uint64_t* dummy)
{
    /* a simple perspective looking down -z from (cx, 0.5, cz): clip x = x', y = y', w = -z' */
    memset(v, 0, sizeof *v);
    const float f = 1.7320508f;
    float vp[16] = {f * h / (float)w, 0, 0, -f * h / (float)w * cx,
                    0, f, 0, -0.5f * f,
                    0, 0, -1.001f, 0,
                    0, 0, -1, cz};
    memcpy(v->view_proj, vp, sizeof vp);
    v->near_plane = 0.05f;
    v->width = w;
    v->height = h;
    v->visbuffer = dummy;
}

int main(void)
{
    static const float fake_pos[3] = {0, 0, 0};
    static const uint32_t fake_idx[3] = {0, 0, 0};
    enum { NV = 9 };
    uint64_t dummy[NV];   /* distinct visibility-buffer handles (never dereferenced) */
    curast_view views[NV];
    for (int i = 0; i < NV; ++i) view_at(&views[i], 0.3f * i - 1.0f, 3.0f + 0.5f * i, 64 + 37 * i, 48 + 11 * i, &dummy[i]);
    views[NV - 1].width = 1;
    views[NV - 1].height = 1;

    /* meshes: plain, instanced (1000 instances, some behind the camera), empty, compressed */
    enum { NI = 1000 };
    float* inst = malloc(sizeof(float) * 12 * NI);
    for (int i = 0; i < NI; ++i) {
        float* X = inst + 12 * i;
        const float s = 0.5f + (float)(i % 7) * 0.25f;
        const float X0[12] = {s, 0, 0, (float)(i % 31) * 0.3f - 4.5f, 0, s, 0, (float)(i % 5) * 0.2f,
                              0, 0, s, (float)(i % 43) * 0.4f - 8.0f};
        memcpy(X, X0, sizeof X0);
    }
    curast_compressed cmp;
    memset(&cmp, 0, sizeof cmp);
    cmp.indices = fake_idx;
    cmp.positions = (const uint16_t*)fake_pos;
    cmp.index_bits = 20;
    for (int k = 0; k < 3; ++k) cmp.step[k] = 1.0f / 65535.0f;
    curast_mesh meshes[4];
    memset(meshes, 0, sizeof meshes);
    meshes[0].vertices = fake_pos; meshes[0].num_vertices = 1000; meshes[0].indices = fake_idx;
    meshes[0].num_triangles = 1998;
    meshes[0].bsphere[3] = 1.5f;
    meshes[1] = meshes[0];
    meshes[1].instances = inst; meshes[1].num_instances = NI;
    meshes[1].bsphere[3] = 0.2f;
    meshes[2].bsphere[3] = 1.0f;                      /* no triangles */
    meshes[3] = meshes[0];
    meshes[3].compressed = &cmp;
    meshes[3].bsphere[3] = 0.0f;                      /* unknown bound: never culled */

    const int64_t pairs = curast_id_bases(meshes, 4, NULL);
    CHECK(pairs == 1 + NI + 1 + 1);
    int64_t* bases = malloc(sizeof(int64_t) * (size_t)(pairs + 1));
    CHECK(curast_id_bases(meshes, 4, bases) == pairs);
    CHECK(bases[pairs] == (int64_t)(1998ull * (NI + 2)));
    uint8_t* visible = malloc((size_t)pairs * NV);
    uint64_t counts[4];
    curast_options opt;
    memset(&opt, 0, sizeof opt);
    for (uint32_t mode = 0; mode <= 4; ++mode) {
        opt.s1_mode = mode;
        for (uint32_t dpi = 1; dpi <= 256; dpi *= 4) {
            opt.s1_draws_per_item = dpi;
            CHECK(curast_plan(meshes, 4, views, NV, &opt, visible, bases, counts) == CURAST_OK);
            CHECK(counts[0] + counts[1] <= (uint64_t)pairs * NV);
            for (int64_t k = 0; k < pairs * NV; ++k) CHECK(visible[k] <= 2);
        }
    }
    CHECK(curast_plan(meshes, 4, views, 1, NULL, NULL, NULL, NULL) == CURAST_OK);
    CHECK(curast_plan(NULL, 0, views, 1, NULL, NULL, NULL, counts) == CURAST_OK);

    /* invalid arguments: an error status, no access out of bounds */
    CHECK(curast_plan(NULL, 2, views, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    CHECK(curast_plan(meshes, 4, NULL, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    CHECK(curast_plan(meshes, 4, views, 0, NULL, NULL, NULL, NULL) != CURAST_OK);
    curast_view bad = views[0];
    bad.width = 0;
    CHECK(curast_plan(meshes, 4, &bad, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    bad = views[0];
    bad.near_plane = 0.0f;
    CHECK(curast_plan(meshes, 4, &bad, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    bad = views[0];
    bad.view_proj[5] = NAN;
    CHECK(curast_plan(meshes, 4, &bad, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    bad = views[0];
    bad.visbuffer = NULL;
    CHECK(curast_plan(meshes, 4, &bad, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    curast_mesh bm = meshes[1];
    bm.num_instances = 0;
    CHECK(curast_plan(&bm, 1, views, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    CHECK(curast_id_bases(&bm, 1, NULL) < 0);
    bm = meshes[1];
    inst[7] = INFINITY;
    CHECK(curast_plan(&bm, 1, views, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    inst[7] = 0.0f;
    bm = meshes[0];
    bm.num_triangles = 1ull << 33;                      /* more than 2^32 - 1 triangles */
    CHECK(curast_plan(&bm, 1, views, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    bm = meshes[1];
    bm.num_triangles = 0xFFFFFFFFull;                   /* T x N beyond the 36-bit ID range */
    CHECK(curast_plan(&bm, 1, views, 1, NULL, NULL, NULL, NULL) == CURAST_E_ID_RANGE);
    CHECK(curast_id_bases(&bm, 1, NULL) == CURAST_E_ID_RANGE);
    bm = meshes[3];
    curast_compressed bc = cmp;
    bc.index_bits = 33;
    bm.compressed = &bc;
    CHECK(curast_plan(&bm, 1, views, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    bc = cmp;
    bc.step[1] = -1.0f;
    CHECK(curast_plan(&bm, 1, views, 1, NULL, NULL, NULL, NULL) != CURAST_OK);
    memset(&opt, 0, sizeof opt);
    opt.s1_mode = 9;
    CHECK(curast_plan(meshes, 4, views, 1, &opt, NULL, NULL, NULL) != CURAST_OK);
    memset(&opt, 0, sizeof opt);
    opt.s1_block = 100;
    CHECK(curast_plan(meshes, 4, views, 1, &opt, NULL, NULL, NULL) != CURAST_OK);

    CHECK(curast_texture_texels(8, 4, 4) == 8 * 4 + 4 * 2 + 2 * 1 + 1);
    CHECK(curast_texture_texels(3, 4, 1) == 0);
    CHECK(curast_texture_texels(16, 16, 6) == 0);
    for (int s = -12; s <= 1; ++s) CHECK(curast_status_string(s) != NULL);
    CHECK(curast_version() > 0);
    free(inst); free(bases); free(visible);
    printf("plan driver: ok\n");
    return 0;
}

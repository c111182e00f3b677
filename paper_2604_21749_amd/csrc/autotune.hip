// Autotuner: picks stage thresholds, workgroup sizes, work-item sizes and queue capacities by
// timing whole frames with HIP events (coordinate descent over a fixed candidate grid).  The
// paper fixes its thresholds (128 and 4096 pixels) by experiment (Sec. 4); here the experiment
// runs per device and scene class.  No option changes the visibility buffer, so tuning is safe.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/curast.h"
#include "log.h"

extern "C" int curast_internal_queue_counts(curast_ctx* ctx, uint64_t out[3]);
extern "C" int curast_internal_num_cus(const curast_ctx* ctx);
extern "C" int curast_internal_default_options(const curast_ctx* ctx, curast_options* out);

namespace {

int ilog2(uint64_t v)
{
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

std::string scene_key(const curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* views,
                      uint32_t n_views)
{
    uint64_t tris = 0, inst = 0, px = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const uint64_t n = meshes[m].instances ? meshes[m].num_instances : 1;
        tris += meshes[m].num_triangles * n;
        inst += n;
    }
    for (uint32_t v = 0; v < n_views; ++v) px += (uint64_t)views[v].width * (uint64_t)views[v].height;
    char buf[256];
    std::snprintf(buf, sizeof buf, "gfx950/cu%d/meshes%d/inst%d/views%u/tris2^%d/px2^%d", curast_internal_num_cus(ctx),
                  ilog2(M ? M : 1), ilog2(inst ? inst : 1), n_views, ilog2(tris ? tris : 1), ilog2(px ? px : 1));
    return buf;
}

struct Field {
    const char* name;
    uint32_t curast_options::*ptr;
};

const Field kFields[] = {
    {"small_px", &curast_options::small_px},
    {"medium_px", &curast_options::medium_px},
    {"s1_block", &curast_options::s1_block},
    {"s1_tris_per_thread", &curast_options::s1_tris_per_thread},
    {"s1_draws_per_item", &curast_options::s1_draws_per_item},
    {"s2_waves", &curast_options::s2_waves},
    {"s3_blocks", &curast_options::s3_blocks},
    {"q2_capacity", &curast_options::q2_capacity},
    {"q3_capacity", &curast_options::q3_capacity},
    {"large_capacity", &curast_options::large_capacity},
    {"s1_mode", &curast_options::s1_mode},
    {"s1_multi_tris_per_thread", &curast_options::s1_multi_tris_per_thread},
    {"s1_blocks_per_cu", &curast_options::s1_blocks_per_cu},
};

std::string to_json(const std::string& key, const curast_options& o)
{
    std::string s = "{\"key\": \"" + key + "\"";
    for (const Field& f : kFields) s += ", \"" + std::string(f.name) + "\": " + std::to_string(o.*(f.ptr));
    return s + "}";
}

bool from_json(const std::string& line, const std::string& key, curast_options& o)
{
    if (line.find("\"key\": \"" + key + "\"") == std::string::npos) return false;
    for (const Field& f : kFields) {
        const std::string pat = "\"" + std::string(f.name) + "\": ";
        const size_t p = line.find(pat);
        if (p == std::string::npos) return false;
        o.*(f.ptr) = (uint32_t)std::strtoul(line.c_str() + p + pat.size(), nullptr, 10);
    }
    return true;
}

// A candidate is timed on the GPU only (the library's frame events, from the first kernel of a
// frame to its last, so host planning jitter stays out), as the mean of kTuneReps frames after
// one warm-up frame, and replaces the best one only when at least 2% faster.
constexpr int kTuneReps = 5;
constexpr float kTuneGain = 0.98f;

float frame_ms(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* views, uint32_t n_views,
               hipStream_t s, int reps, int* rc)
{
    auto run = [&]() {
        return n_views == 1 ? curast_rasterize_meshes(ctx, meshes, M, views, s)
                            : curast_rasterize_batched(ctx, meshes, M, views, n_views, s);
    };
    curast_options o{};
    *rc = curast_get_options(ctx, &o);
    if (*rc) return 1e30f;
    const uint32_t flags = o.flags;
    o.flags |= CURAST_FLAG_TIMING;
    *rc = curast_set_options(ctx, &o);
    if (*rc) return 1e30f;
    *rc = run();   // warm-up (and graph capture)
    if (*rc == 0) *rc = curast_reset_stage_times(ctx);
    for (int i = 0; i < reps && *rc == 0; ++i) *rc = run();
    if (*rc == 0) *rc = hipStreamSynchronize(s) == hipSuccess ? CURAST_OK : CURAST_E_HIP;
    double ms[9] = {};
    uint64_t frames = 0;
    if (*rc == 0) *rc = curast_get_stage_times(ctx, ms, &frames);
    o.flags = flags;
    const int r2 = curast_set_options(ctx, &o);
    if (*rc == 0) *rc = r2;
    if (*rc || frames == 0) return 1e30f;
    return (float)(ms[8] / (double)frames);
}

uint32_t pow2_at_least(uint64_t v)
{
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return (uint32_t)std::min<uint64_t>(p, 1u << 30);
}

}  // namespace

extern "C" int curast_autotune(curast_ctx* ctx, const curast_mesh* meshes, uint32_t M, const curast_view* views,
                               uint32_t n_views, const char* cache_path, curast_options* chosen, void* stream)
{
    if (!ctx || !views || n_views == 0 || (M && !meshes)) return CURAST_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string key = scene_key(ctx, meshes, M, views, n_views);
    curast_options base;
    int rc = curast_get_options(ctx, &base);
    if (rc) return rc;
    const uint32_t keep_flags = base.flags;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[4096];
            curast_options o = base;
            bool hit = false;
            while (std::fgets(line, sizeof line, f))
                if (from_json(line, key, o)) hit = true;
            std::fclose(f);
            if (hit) {
                o.flags = keep_flags;
                curast::log_line("autotune: cached options for %s", key.c_str());
                rc = curast_set_options(ctx, &o);
                if (rc == CURAST_OK && chosen) curast_get_options(ctx, chosen);
                return rc;
            }
        }
    }
    // tune without statistics / timing instrumentation
    curast_options best = base;
    best.flags = keep_flags & ~(0x8u | 0x20u);
    rc = curast_set_options(ctx, &best);
    if (rc) return rc;
    float best_ms = frame_ms(ctx, meshes, M, views, n_views, s, kTuneReps, &rc);
    if (rc) return rc;
    // grow the queues to twice the observed fill when that exceeds the library defaults; never
    // shrink them below the defaults: the choice is cached for a whole scene class, and a scene of
    // the class that forwards more triangles would otherwise fall back to the one-thread overflow
    // pass (q2_overflow / q3_overflow in the statistics count such triangles)
    uint64_t fill[3];
    curast_options defaults{};
    if (curast_internal_queue_counts(ctx, fill) == CURAST_OK &&
        curast_internal_default_options(ctx, &defaults) == CURAST_OK) {
        best.q2_capacity = std::max<uint32_t>(defaults.q2_capacity, pow2_at_least(2 * fill[0] + 1));
        best.large_capacity = std::max<uint32_t>(defaults.large_capacity, pow2_at_least(2 * fill[1] + 1));
        best.q3_capacity = std::max<uint32_t>(defaults.q3_capacity, pow2_at_least(2 * fill[2] + 1));
        rc = curast_set_options(ctx, &best);
        if (rc) return rc;
        best_ms = frame_ms(ctx, meshes, M, views, n_views, s, kTuneReps, &rc);
        if (rc) return rc;
    }
    uint64_t max_draws = 0;
    for (uint32_t m = 0; m < M; ++m) max_draws = std::max<uint64_t>(max_draws, (meshes[m].instances ? meshes[m].num_instances : 1) * (uint64_t)n_views);
    const uint32_t cus = (uint32_t)curast_internal_num_cus(ctx);
    struct Axis {
        uint32_t curast_options::*ptr;
        std::vector<uint32_t> values;
    };
    std::vector<Axis> axes = {
        {&curast_options::s1_mode, {0, 1, 2, 3, 4}},
        {&curast_options::s1_block, {64, 128, 256, 512}},
        {&curast_options::s1_tris_per_thread, {1, 2, 4, 8}},
        {&curast_options::s1_blocks_per_cu, {256, 1024, 2048, 4096}},
        {&curast_options::small_px, {32, 64, 128, 256, 512}},
        {&curast_options::medium_px, {1024, 4096, 16384}},
        {&curast_options::s2_waves, {cus * 4, cus * 8, cus * 16, cus * 32}},
        {&curast_options::s3_blocks, {cus, cus * 2, cus * 4}},
    };
    if (max_draws > 1) {
        axes.push_back({&curast_options::s1_multi_tris_per_thread, {1, 2, 4, 8}});
        axes.push_back({&curast_options::s1_draws_per_item, {8, 16, 32, 64, 128, 256}});
    }
    for (int pass = 0; pass < 2; ++pass) {
        bool improved = false;
        for (const Axis& ax : axes) {
            // re-time the current best before each axis, so that one lucky measurement of it
            // does not hide a real gain further on
            if (curast_set_options(ctx, &best) == CURAST_OK) {
                int r0 = 0;
                const float again = frame_ms(ctx, meshes, M, views, n_views, s, kTuneReps, &r0);
                if (r0 == CURAST_OK) best_ms = again;
            }
            for (uint32_t v : ax.values) {
                if (best.*(ax.ptr) == v) continue;
                curast_options cand = best;
                cand.*(ax.ptr) = v;
                if (curast_set_options(ctx, &cand) != CURAST_OK) continue;
                int r2 = 0;
                const float ms = frame_ms(ctx, meshes, M, views, n_views, s, kTuneReps, &r2);
                if (r2 == CURAST_OK && ms < kTuneGain * best_ms) {
                    best = cand;
                    best_ms = ms;
                    improved = true;
                }
            }
        }
        if (!improved) break;
    }
    best.flags = keep_flags;
    rc = curast_set_options(ctx, &best);
    if (rc) return rc;
    curast::log_line("autotune: %s -> %.4f ms: %s", key.c_str(), best_ms, to_json(key, best).c_str());
    if (chosen) curast_get_options(ctx, chosen);
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s\n", to_json(key, best).c_str());
            std::fclose(f);
        }
    }
    return CURAST_OK;
}

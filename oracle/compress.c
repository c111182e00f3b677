/* Compressed mesh geometry (Sec. 4.6), the plain definition -- test infrastructure only.
 *
 * Positions: q = clamp(rint((p - lo) * scale), 0, 65535) per component, the subtraction and the
 * product in binary32 (rint rounds half to even), scale = (float)(1 / (double)step), 0 for a flat
 * axis; decoding gives fmaf((float)q, step, lo).  The index packing is integer work done in
 * oracle/__init__.py. */
#include <math.h>
#include <stdint.h>

#include "oracle.h"

static float quant_scale(float step) { return step > 0.0f ? (float)(1.0 / (double)step) : 0.0f; }

int orc_quantize_positions(const float* pos, uint32_t V, const float lo[3], const float step[3], uint16_t* out)
{
    if (V && (!pos || !out)) return -1;
    for (uint64_t i = 0; i < 3ull * V; ++i) {
        const int c = (int)(i % 3);
        const float d = pos[i] - lo[c];
        const float t = rintf(d * quant_scale(step[c]));
        out[i] = (uint16_t)(t < 0.0f ? 0.0f : (t > 65535.0f ? 65535.0f : t));
    }
    return 0;
}

int orc_decode_positions(const uint16_t* q, uint32_t V, const float lo[3], const float step[3], float* out)
{
    if (V && (!q || !out)) return -1;
    for (uint64_t i = 0; i < 3ull * V; ++i) {
        const int c = (int)(i % 3);
        out[i] = fmaf((float)q[i], step[c], lo[c]);
    }
    return 0;
}

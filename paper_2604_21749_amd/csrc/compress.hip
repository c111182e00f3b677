// Compression of mesh geometry for gfx950 (Sec. 4.6): index range and position bounding box
// (wave reductions, one atomic per wavefront), bit packing of indices relative to their minimum
// and 16-bit quantization of positions relative to the bounding box.  The decoding side lives in
// device.h (packed_index, mesh_vertex); the host entry points in runtime.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"

namespace curast {

// Order-preserving map of binary32 to uint32 (negative values reversed below the positive ones).
__device__ __forceinline__ uint32_t ordered_bits(float f)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

// out[0..7] = {index min, index max, ordered min x, y, z, ordered max x, y, z}
__global__ void __launch_bounds__(64) range_init_kernel(uint32_t* out)
{
    if (threadIdx.x < 8) out[threadIdx.x] = (threadIdx.x == 0 || (threadIdx.x >= 2 && threadIdx.x < 5)) ? 0xFFFFFFFFu : 0u;
}

__global__ void __launch_bounds__(256) index_range_kernel(const uint32_t* __restrict__ idx, uint64_t n, uint32_t* out)
{
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = gl(idx)[i];
        lo = min(lo, v);
        hi = max(hi, v);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(out + 0, lo);
        atomicMax(out + 1, hi);
    }
}

__global__ void __launch_bounds__(256) bbox_kernel(const float* __restrict__ pos, uint32_t V, uint32_t* out)
{
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint32_t b = ordered_bits(gl(pos)[3 * v + c]);
            lo[c] = min(lo[c], b);
            hi[c] = max(hi[c], b);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = wave_min(lo[c]);
        hi[c] = wave_max(hi[c]);
    }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            atomicMin(out + 2 + c, lo[c]);
            atomicMax(out + 5 + c, hi[c]);
        }
}

// One lane per 32-bit output word: ORs in every value whose bits overlap the word (words past
// the last value, the padding, are 0).
__global__ void __launch_bounds__(256) pack_kernel(const uint32_t* __restrict__ idx, uint64_t n, uint32_t bits,
                                                   uint32_t base, uint32_t* __restrict__ out, uint64_t words)
{
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= words) return;
    const uint64_t b0 = 32 * w;                  // first bit of the word
    const uint64_t first = b0 / bits, last = (b0 + 31) / bits;
    uint32_t word = 0;
    for (uint64_t i = first; i <= last && i < n; ++i) {
        const uint64_t v = (uint64_t)(gl(idx)[i] - base);
        const int64_t shift = (int64_t)(i * bits) - (int64_t)b0;   // position of the value in the word
        word |= (uint32_t)(shift >= 0 ? (v << shift) : (v >> -shift));
    }
    gl(out)[w] = word;
}

// One lane per position component: q = clamp(rint((p - lo) * scale), 0, 65535) in binary32;
// element n, the padding, is 0.
__global__ void __launch_bounds__(256) quantize_kernel(const float* __restrict__ pos, uint64_t n, float lx, float ly,
                                                       float lz, float sx, float sy, float sz,
                                                       uint16_t* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        gl(out)[i] = 0;
        return;
    }
    const uint32_t c = (uint32_t)(i % 3);
    const float lo = c == 0 ? lx : c == 1 ? ly : lz;
    const float sc = c == 0 ? sx : c == 1 ? sy : sz;
    const float t = __builtin_rintf((gl(pos)[i] - lo) * sc);
    gl(out)[i] = (uint16_t)(t < 0.0f ? 0.0f : t > 65535.0f ? 65535.0f : t);
}

static uint32_t blocks_of(uint64_t n, uint32_t cap)
{
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, cap));
}

hipError_t launch_compress_ranges(const uint32_t* idx, uint64_t n_idx, const float* pos, uint32_t V, uint32_t* out,
                                  uint32_t cus, hipStream_t s)
{
    range_init_kernel<<<1, 64, 0, s>>>(out);
    if (n_idx) index_range_kernel<<<blocks_of(n_idx, cus * 8), 256, 0, s>>>(idx, n_idx, out);
    if (V) bbox_kernel<<<blocks_of(V, cus * 8), 256, 0, s>>>(pos, V, out);
    return hipGetLastError();
}

hipError_t launch_compress(const uint32_t* idx, uint64_t n_idx, uint32_t bits, uint32_t base, uint32_t* packed,
                           uint64_t words, const float* pos, uint32_t V, const float lo[3], const float scale[3],
                           uint16_t* qpos, hipStream_t s)
{
    if (words) pack_kernel<<<blocks_of(words, 0xFFFFFFFFu), 256, 0, s>>>(idx, n_idx, bits, base, packed, words);
    const uint64_t n = 3ull * V;
    quantize_kernel<<<blocks_of(n + 1, 0xFFFFFFFFu), 256, 0, s>>>(pos, n, lo[0], lo[1], lo[2], scale[0], scale[1],
                                                                  scale[2], qpos);
    return hipGetLastError();
}

}  // namespace curast

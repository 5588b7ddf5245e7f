// Streaming loader for band-interleaved-by-pixel cubes (gfx950).
//
// A wave reads a group of 8 consecutive pixels; every lane owns 4 band
// "slots" for all stages of a kernel, so per-band running sums stay in
// registers. Two lane layouts:
//   VEC = 4: lane l owns bands 4l .. 4l+3 (one 16-byte float4 / 8-byte ushort4
//            load per pixel; needs ld % 4 == 0 and an aligned base);
//   VEC = 1: lane l owns bands l, l+64, l+128, l+192 (one element per load;
//            any ld). Either way one wave-wide load reads a contiguous run of
//            the pixel's row, so global reads are coalesced.
#pragma once

#include "common.hpp"

namespace pca {

template <int VEC>
__device__ inline int slot_band(int lane, int s)
{
    return VEC == 4 ? 4 * lane + s : lane + 64 * s;
}

template <typename T, int VEC>
__device__ inline void load_group(const T *__restrict__ Y, int64_t ld, int64_t p0, int64_t pend,
                                  int m, int lane, float (&v)[8][4])
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t p = p0 + i;
        const bool okp = p < pend;
        if constexpr (VEC == 4) {
            const int b = 4 * lane;
            float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
            if (okp && b + 3 < m) {
                const T *src = Y + p * ld + b;
                if constexpr (sizeof(T) == 4) {
                    const f32x4 x = *reinterpret_cast<const f32x4 *>(src);
                    x0 = x[0]; x1 = x[1]; x2 = x[2]; x3 = x[3];
                } else {
                    const uint2 raw = *reinterpret_cast<const uint2 *>(src);
                    x0 = (float)(raw.x & 0xffffu); x1 = (float)(raw.x >> 16);
                    x2 = (float)(raw.y & 0xffffu); x3 = (float)(raw.y >> 16);
                }
            } else if (okp && b < m) {
                // Last, partial quad of the row: element loads stay inside it.
                const T *src = Y + p * ld + b;
                x0 = load_elem(src);
                if (b + 1 < m) x1 = load_elem(src + 1);
                if (b + 2 < m) x2 = load_elem(src + 2);
            }
            v[i][0] = x0; v[i][1] = x1; v[i][2] = x2; v[i][3] = x3;
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int b = lane + 64 * s;
                v[i][s] = (okp && b < m) ? load_elem(Y + p * ld + b) : 0.f;
            }
        }
    }
}

// Can the VEC = 4 layout be used for this cube?
inline bool vec4_ok(const void *Y, int dt, int64_t ld)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(Y);
    const uintptr_t align = dt == PCA_IN_F32 ? 16 : 8;
    return (ld % 4 == 0) && (a % align == 0);
}

}  // namespace pca

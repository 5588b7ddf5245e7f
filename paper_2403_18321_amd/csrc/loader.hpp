// Streaming loader for band-interleaved-by-pixel cubes (gfx950).
//
// A wave reads a group of 8 consecutive pixels; every lane owns 4 band
// "slots" for all stages of a kernel, so per-band running sums stay in
// registers. Two lane layouts:
//   VEC = 4: lane l owns bands 4l .. 4l+3 (one 16-byte float4 / 8-byte ushort4
//            load per pixel; needs bands % 4 == 0, ld % 4 == 0 and an aligned
//            base);
//   VEC = 1: lane l owns bands l, l+64, l+128, l+192 (one element per load;
//            any shape).
// Either way one wave-wide load reads a contiguous run of the pixel's row, so
// global reads are coalesced.
//
// Loading is split from use so that a prefetched group stays in flight across
// barriers and other work: load() issues the loads with no consumer (a lane
// or pixel out of range reads element 0 of the cube instead, branch-free), and
// get() converts a raw word when the data is used. Callers mask out-of-range
// bands and pixels themselves (see valid()).
#pragma once

#include <type_traits>

#include "common.hpp"

namespace pca {

template <int VEC>
__device__ inline int slot_band(int lane, int s)
{
    return VEC == 4 ? 4 * lane + s : lane + 64 * s;
}

template <typename T, int VEC>
struct Group {
    using W = typename std::conditional<VEC == 4,
                                        typename std::conditional<sizeof(T) == 4, f32x4, uint2>::type,
                                        T>::type;
    W x[VEC == 4 ? 8 : 32];

    __device__ inline void load(const T *__restrict__ Y, int64_t ld, int64_t p0, int64_t pend, int m, int lane)
    {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if constexpr (VEC == 4) {
                const int b = 4 * lane;
                const bool ok = b < m && (p0 + i) < pend;
                x[i] = *reinterpret_cast<const W *>(Y + (ok ? (p0 + i) * ld + b : 0));
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int b = lane + 64 * s;
                    const bool ok = b < m && (p0 + i) < pend;
                    x[4 * i + s] = Y[ok ? (p0 + i) * ld + b : 0];
                }
            }
        }
    }

    // Value of pixel i (0..7), slot s (0..3), unmasked.
    __device__ inline float get(int i, int s) const
    {
        if constexpr (VEC == 4) {
            if constexpr (sizeof(T) == 4) {
                return x[i][s];
            } else {
                const uint32_t w = (s < 2) ? x[i].x : x[i].y;
                return (float)((s & 1) ? (w >> 16) : (w & 0xffffu));
            }
        } else {
            return (float)x[4 * i + s];
        }
    }
};

// Can the VEC = 4 layout be used for this cube?
inline bool vec4_ok(const void *Y, int dt, int m, int64_t ld)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(Y);
    const uintptr_t align = dt == PCA_IN_F32 ? 16 : 8;
    return (m % 4 == 0) && (ld % 4 == 0) && (a % align == 0);
}

}  // namespace pca

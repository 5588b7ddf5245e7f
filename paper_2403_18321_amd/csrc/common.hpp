// Device-side helpers shared by the gfx950 kernels of libpca.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pca {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

constexpr int kWave = 64;
__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Element loaders: float32 or uint16 cubes, both returned as float (uint16
// values are exact in float32).
__device__ inline float load_elem(const float *p) { return *p; }
__device__ inline float load_elem(const uint16_t *p) { return (float)(*p); }

// Wave-wide sum of a double (butterfly over the 64 lanes).
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline int wave_sum_int(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace pca

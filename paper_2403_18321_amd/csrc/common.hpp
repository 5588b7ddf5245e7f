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

// Round-robin tournament used for the parallel Jacobi steps (n even). Player 0
// stays at position 0; the other n-1 players turn by one position per step.
// Position j of step s holds player 1 + ((j - 1 + s) mod (n - 1)) (j >= 1).
// Pair k of step s is (position k, position n-1-k). Returned with a < b.
__device__ inline void rr_pair(int n, int step, int k, int &a, int &b)
{
    const int m = n - 1;
    auto player = [&](int pos) -> int {
        if (pos == 0) return 0;
        int v = pos - 1 + step;
        v %= m;
        return 1 + v;
    };
    int x = player(k), y = player(n - 1 - k);
    a = x < y ? x : y;
    b = x < y ? y : x;
}

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

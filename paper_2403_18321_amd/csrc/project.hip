// Projection of every pixel onto the first k eigenvectors (Algorithm 1, lines
// 5-6): Q'[p, i] = sum_b (Y[p, b] - mu_b) V[b, i], i < k.
//
// A workgroup stages 64 pixels x all bands in LDS (coalesced reads, the mean
// subtracted on the way in: the centred cube is never written to HBM), then
// each wave multiplies its 16 pixels by V[:, 16g .. 16g+15] with
// v_mfma_f32_16x16x4_f32, K = bands. The eigenvector block lives in
// registers for the whole workgroup. The cube is read once per group of 16
// components (once for k <= 16).
#include "common.hpp"
#include "kernels.hpp"
#include "loader.hpp"

namespace pca {

namespace {

constexpr int kThreads = 256;
constexpr int kTP = 64;                  // pixels per workgroup (4 waves x 16)
constexpr int kMaxKSteps = 64;           // 256 bands / 4

// Tile pitch (floats): a multiple of 4 with pitch/4 odd, so the 16 pixels x 4
// bands read by one MFMA operand load hit 64 distinct LDS banks.
__host__ __device__ inline int proj_pitch(int m4) { return ((m4 / 4) & 1) ? m4 : m4 + 4; }

template <typename T, int VEC>
__global__ __launch_bounds__(kThreads) void project_kernel(const T *__restrict__ Y, int64_t n, int m,
                                                           int64_t ld, const float *__restrict__ mean,
                                                           const float *__restrict__ V, int k,
                                                           float *__restrict__ Q)
{
    __shared__ __attribute__((aligned(16))) float tile[kTP * 260];
    __shared__ float mu[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m4 = round_up(m, 4);
    const int pitch = proj_pitch(m4);
    const int ksteps = m4 / 4;
    const int g = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * kTP;

    for (int b = tid; b < 256; b += kThreads) mu[b] = (mean && b < m) ? mean[b] : 0.f;

    // B operand: lane holds V[4s + lane/16][16g + lane%16] for every K step s.
    float bv[kMaxKSteps];
    {
        const int o = 16 * g + (lane & 15);
#pragma unroll
        for (int s = 0; s < kMaxKSteps; ++s) {
            const int b = 4 * s + (lane >> 4);
            bv[s] = (s < ksteps && b < m && o < k) ? V[(int64_t)b * m + o] : 0.f;
        }
    }
    __syncthreads();

    // Stage the centred pixels: wave w loads groups w and w + 4 (8 pixels each).
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int grp = wave + 4 * h;
        float v[8][4];
        load_group<T, VEC>(Y, ld, p0 + 8 * grp, n, m, lane, v);
        if constexpr (VEC == 4) {
            const int b = 4 * lane;
            if (b < m4) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    f32x4 q;
#pragma unroll
                    for (int s = 0; s < 4; ++s) q[s] = (b + s < m) ? v[i][s] - mu[b + s] : 0.f;
                    *reinterpret_cast<f32x4 *>(&tile[(8 * grp + i) * pitch + b]) = q;
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int b = lane + 64 * s;
                if (b < m4) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) tile[(8 * grp + i) * pitch + b] = (b < m) ? v[i][s] - mu[b] : 0.f;
                }
            }
        }
    }
    __syncthreads();

    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float *arow = &tile[(16 * wave + (lane & 15)) * pitch + (lane >> 4)];
#pragma unroll
    for (int s = 0; s < kMaxKSteps; ++s) {
        if (s < ksteps) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[4 * s], bv[s], acc, 0, 0, 0);
    }

    // 16x16 result layout: lane holds rows 4 (lane/16) + r, column lane % 16.
    const int o = 16 * g + (lane & 15);
    if (o < k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t p = p0 + 16 * wave + 4 * (lane >> 4) + r;
            if (p < n) Q[p * k + o] = acc[r];
        }
    }
}

template <typename T>
hipError_t launch_t(const T *Y, int64_t n, int m, int64_t ld, const float *mean, const float *V, int k,
                    float *Q, hipStream_t st, bool v4)
{
    dim3 grid((unsigned)((n + kTP - 1) / kTP), (unsigned)((k + 15) / 16)), block(kThreads);
    if (v4)
        hipLaunchKernelGGL((project_kernel<T, 4>), grid, block, 0, st, Y, n, m, ld, mean, V, k, Q);
    else
        hipLaunchKernelGGL((project_kernel<T, 1>), grid, block, 0, st, Y, n, m, ld, mean, V, k, Q);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project(const void *Y, int dt, int64_t n, int m, int64_t ld, const float *mean,
                          const float *V, int k, float *Q, hipStream_t st)
{
    const bool v4 = vec4_ok(Y, dt, ld);
    if (dt == PCA_IN_F32) return launch_t(static_cast<const float *>(Y), n, m, ld, mean, V, k, Q, st, v4);
    return launch_t(static_cast<const uint16_t *>(Y), n, m, ld, mean, V, k, Q, st, v4);
}

}  // namespace pca

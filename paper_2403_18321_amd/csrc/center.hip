// Band-average removal on its own (Algorithm 1, line 2): the per-band mean of
// the GPU design's Code 4.2.1 and its subtraction, Code 4.2.2. Used when the
// caller wants the centred cube X itself; the covariance path fuses the
// centring and never writes X.
//   center_sums:     one workgroup per chunk of pixels, float64 band sums;
//   center_mean:     chunk sums added in chunk order, mu = sum / N;
//   center_subtract: X = Y - 1 mu^T, each element rounded once from float64.
#include "common.hpp"
#include "kernels.hpp"
#include "loader.hpp"

namespace pca {

namespace {

constexpr int kThreads = 256;

template <typename T, int VEC>
__global__ __launch_bounds__(kThreads) void center_sums_kernel(const T *__restrict__ Y, int64_t n, int m,
                                                               int64_t ld, int64_t chunk, int mpad,
                                                               double *__restrict__ partSum)
{
    __shared__ double red[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c = blockIdx.x;
    const int64_t pbeg = c * chunk;
    const int64_t pend = (pbeg + chunk < n) ? pbeg + chunk : n;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    Group<T, VEC> v;
    for (int64_t g = pbeg + 8 * wave; g < pend; g += 32) {
        v.load(Y, ld, g, pend, m, lane);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool okb = slot_band<VEC>(lane, s) < m;
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) t += (okb && g + i < pend) ? (double)v.get(i, s) : 0.0;
            sums[s] += t;
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) red[wave][slot_band<VEC>(lane, s)] = sums[s];
    __syncthreads();
    for (int b = tid; b < mpad; b += kThreads)
        partSum[c * mpad + b] = ((red[0][b] + red[1][b]) + red[2][b]) + red[3][b];
}

__global__ __launch_bounds__(256) void center_mean_kernel(int64_t n, int m, int64_t nchunks, int mpad,
                                                          const double *__restrict__ partSum,
                                                          float *__restrict__ mean,
                                                          double *__restrict__ mean64)
{
    for (int b = threadIdx.x; b < m; b += blockDim.x) {
        double a = 0.0;
        for (int64_t w = 0; w < nchunks; ++w) a += partSum[w * mpad + b];
        const double mu = a / (double)n;
        mean64[b] = mu;
        if (mean) mean[b] = (float)mu;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void center_subtract_kernel(const T *__restrict__ Y, int64_t n, int m,
                                                              int64_t ld, const double *__restrict__ mean64,
                                                              float *__restrict__ X, int64_t ldx)
{
    __shared__ double mu[256];
    for (int b = threadIdx.x; b < m; b += blockDim.x) mu[b] = mean64[b];
    __syncthreads();
    const int64_t total = n * (int64_t)m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / m;
        const int b = (int)(e - p * m);
        X[p * ldx + b] = (float)((double)load_elem(Y + p * ld + b) - mu[b]);
    }
}

template <typename T>
hipError_t launch_center_t(const T *Y, int64_t n, int m, int64_t ld, float *mean, float *X, int64_t ldx,
                           const CovPlan &p, double *partSum, double *mean64, hipStream_t st, bool v4)
{
    dim3 grid((unsigned)p.nchunks), block(kThreads);
    if (v4)
        hipLaunchKernelGGL((center_sums_kernel<T, 4>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.mpad, partSum);
    else
        hipLaunchKernelGGL((center_sums_kernel<T, 1>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.mpad, partSum);
    hipLaunchKernelGGL(center_mean_kernel, dim3(1), dim3(256), 0, st, n, m, p.nchunks, p.mpad, partSum, mean, mean64);
    if (X) {
        const int64_t total = n * (int64_t)m;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(center_subtract_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, Y, n, m, ld,
                           mean64, X, ldx);
    }
    return hipGetLastError();
}

// Band-sequential cubes (Y[b * ld + p]): per chunk of pixels, each wave sums
// whole band rows of the chunk (lanes along the row, coalesced), float64.
template <typename T>
__global__ __launch_bounds__(kThreads) void center_sums_bsq_kernel(const T *__restrict__ Y, int64_t n, int m,
                                                                   int64_t ld, int64_t chunk, int mpad,
                                                                   double *__restrict__ partSum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c = blockIdx.x;
    const int64_t pbeg = c * chunk;
    const int64_t pend = (pbeg + chunk < n) ? pbeg + chunk : n;
    for (int b = wave; b < mpad; b += kThreads / 64) {
        double t = 0.0;
        if (b < m) {
            const T *row = Y + (int64_t)b * ld;
            for (int64_t p = pbeg + lane; p < pend; p += 64) t += (double)load_elem(row + p);
        }
        t = wave_sum(t);
        if (lane == 0) partSum[c * mpad + b] = t;
    }
}

// X[b * ldx + p] = Y[b * ld + p] - mu_b; grid (pixel blocks, bands).
template <typename T>
__global__ __launch_bounds__(256) void center_subtract_bsq_kernel(const T *__restrict__ Y, int64_t n, int64_t ld,
                                                                  const double *__restrict__ mean64,
                                                                  float *__restrict__ X, int64_t ldx)
{
    const int b = blockIdx.y;
    const double mu = mean64[b];
    const T *row = Y + (int64_t)b * ld;
    float *out = X + (int64_t)b * ldx;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        out[p] = (float)((double)load_elem(row + p) - mu);
}

template <typename T>
hipError_t launch_center_bsq(const T *Y, int64_t n, int m, int64_t ld, float *mean, float *X, int64_t ldx,
                             const CovPlan &p, double *partSum, double *mean64, hipStream_t st)
{
    hipLaunchKernelGGL(center_sums_bsq_kernel<T>, dim3((unsigned)p.nchunks), dim3(kThreads), 0, st, Y, n, m, ld,
                       p.chunk, p.mpad, partSum);
    hipLaunchKernelGGL(center_mean_kernel, dim3(1), dim3(256), 0, st, n, m, p.nchunks, p.mpad, partSum, mean, mean64);
    if (X) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 64) blocks = 64;
        hipLaunchKernelGGL(center_subtract_bsq_kernel<T>, dim3((unsigned)blocks, (unsigned)m), dim3(256), 0, st, Y, n,
                           ld, mean64, X, ldx);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_center(const void *Y, int dt, int64_t n, int m, int64_t ld, float *mean, float *X,
                         int64_t ldx, const CovPlan &plan, double *partSum, double *mean64, hipStream_t st)
{
    if (dt == PCA_IN_F32_BSQ)
        return launch_center_bsq(static_cast<const float *>(Y), n, m, ld, mean, X, ldx, plan, partSum, mean64, st);
    if (dt == PCA_IN_U16_BSQ)
        return launch_center_bsq(static_cast<const uint16_t *>(Y), n, m, ld, mean, X, ldx, plan, partSum, mean64, st);
    const bool v4 = vec4_ok(Y, dt, m, ld);
    if (dt == PCA_IN_F32)
        return launch_center_t(static_cast<const float *>(Y), n, m, ld, mean, X, ldx, plan, partSum, mean64, st, v4);
    return launch_center_t(static_cast<const uint16_t *>(Y), n, m, ld, mean, X, ldx, plan, partSum, mean64, st, v4);
}

}  // namespace pca

// Reverse-mode derivative of the PCA pipeline of Algorithm 1 (centring,
// covariance, eigenpairs, projection) for a scalar loss L, given the loss's
// gradients at the forward outputs: Qbar = dL/dQ (N x k), lbar = dL/dlambda
// (M), Vbar_k = dL/dV[:, :k] (M x k). With X = Y - 1 mu^T and C = X^T X/(N-1):
//
//   projection  Q = X V_k:     Xbar  = Qbar V_k^T,   Vbar_k += X^T Qbar
//   eigenpairs  C = V diag(lambda) V^T (the standard first-order perturbation
//               of a symmetric eigendecomposition with distinct eigenvalues):
//               Cbar = V (diag(lbar) + F o (V^T Vbar)) V^T, symmetrised,
//               F_ij = 1 / (lambda_j - lambda_i) for i != j, 0 otherwise
//               (and 0 where two eigenvalues are equal)
//   covariance  Xbar += X (Cbar + Cbar^T) / (N - 1) = 2 X Cbar / (N - 1)
//   centring    Ybar = Xbar - (1/N) 1 (1^T Xbar)
//
// Vbar has nonzero columns only below k, so F o (V^T Vbar) has k nonzero
// columns and Cbar = sum_{j<k} w_j v_j^T + sum_j lbar_j v_j v_j^T with
// w_j = V (F[:, j] o (V^T vbar_j)).
//
// Kernels, in launch order:
//   bwd_reduce: per pixel chunk and group of 8 components, float64 sums of
//               X^T Qbar, 1^T Qbar and 1^T X (X formed on the fly from Y, mu);
//   bwd_w:      one 1024-thread workgroup per component j: vbar_j (chunk
//               sums in a fixed order plus Vbar_k), u = F[:, j] o (V^T vbar_j),
//               w_j = V u; one more workgroup finishes 1^T Qbar and 1^T X;
//   bwd_g:      G[a][b] = 2/(N-1) sym(Cbar)[a][b] in 16 x 16 tiles;
//   bwd_r:      rows M .. M+k-1 of G = V_k^T, row M+k = -(1^T Xbar) / N;
//   bwd_apply:  dY = [X | Qbar | 1] G, one GEMM over all pixels with
//               v_mfma_f32_32x32x2_f32, 128 pixels per workgroup, the
//               augmented K dimension staged through LDS 32 at a time (the
//               next slab's loads in flight during the current one's
//               products).
// Band-sequential cubes (Y and dY [bands][pixels], the layout of the paper's
// GPU design, Section 4) take the same kernels with the cube indexed the
// other way; bwd_apply then forms dY^T = G^T [X | Qbar | 1]^T (the MFMA
// operands swapped), so that a result register's lanes hold consecutive
// pixels of one band and its stores stay coalesced.
#include "common.hpp"
#include "kernels.hpp"

namespace pca {

namespace {

constexpr int kThreads = 256;
constexpr int kCompGroup = 8;       // components per bwd_reduce workgroup
constexpr int kRedTile = 64;        // pixels per staged tile of Qbar
constexpr int kApplyPix = 128;      // pixels per bwd_apply workgroup (4 waves x 32)
constexpr int kApplyK = 32;         // augmented-K columns per stage
constexpr int kApplyPitch = kApplyK + 1;

// Partial sums of one (chunk, component group): prod[M][8], sq[8], sx[M].
__host__ __device__ inline int64_t part_stride(int m) { return 9 * (int64_t)m + kCompGroup; }

template <bool BSQ>
__global__ __launch_bounds__(kThreads) void bwd_reduce_kernel(const float *__restrict__ Y, int64_t n, int m,
                                                              int64_t ld, const float *__restrict__ mean,
                                                              const float *__restrict__ dQ, int k, int64_t chunk,
                                                              int kg, double *__restrict__ part)
{
    __shared__ float qt[kRedTile][kCompGroup];
    const int t = threadIdx.x;
    const int w = blockIdx.x, g = blockIdx.y;
    const int j0 = kCompGroup * g;
    const int64_t p0 = (int64_t)w * chunk;
    const int64_t p1 = (p0 + chunk < n) ? p0 + chunk : n;
    const bool hasb = t < m;
    const float mu = hasb ? mean[t] : 0.f;
    double acc[kCompGroup];
#pragma unroll
    for (int j = 0; j < kCompGroup; ++j) acc[j] = 0.0;
    double sx = 0.0, sq = 0.0;
    for (int64_t pt = p0; pt < p1; pt += kRedTile) {
        const int np = (int)((p1 - pt) < kRedTile ? (p1 - pt) : kRedTile);
        __syncthreads();
        for (int e = t; e < kRedTile * kCompGroup; e += kThreads) {
            const int pp = e / kCompGroup, jj = e % kCompGroup;
            qt[pp][jj] = (dQ && pp < np && j0 + jj < k) ? dQ[(pt + pp) * k + j0 + jj] : 0.f;
        }
        __syncthreads();
        if (hasb) {
#pragma unroll 8
            for (int pp = 0; pp < np; ++pp) {
                const double x = (double)(Y[BSQ ? (int64_t)t * ld + pt + pp : (pt + pp) * ld + t] - mu);
                sx += x;
#pragma unroll
                for (int j = 0; j < kCompGroup; ++j) acc[j] += x * (double)qt[pp][j];
            }
        }
        if (t < kCompGroup)
            for (int pp = 0; pp < np; ++pp) sq += (double)qt[pp][t];
    }
    double *dst = part + ((int64_t)w * kg + g) * part_stride(m);
    if (hasb) {
#pragma unroll
        for (int j = 0; j < kCompGroup; ++j) dst[t * kCompGroup + j] = acc[j];
        dst[kCompGroup * m + kCompGroup + t] = sx;
    }
    if (t < kCompGroup) dst[kCompGroup * m + t] = sq;
}

constexpr int kWThreads = 1024;     // bwd_w: slices x bands
constexpr int kWMaxSlices = 8;

// Slice sl (of ns) of sum_w p[w * stride] over w < count: w = sl, sl + ns,
// ..., as eight interleaved partial sums added in a fixed order (eight loads
// in flight).
__device__ inline double slice_sum(const double *__restrict__ p, int64_t stride, int count, int sl, int ns)
{
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int w = sl;
    for (; w + 7 * ns < count; w += 8 * ns) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] += p[(int64_t)(w + i * ns) * stride];
    }
    for (int i = 0; w < count; w += ns, ++i) a[i] += p[(int64_t)w * stride];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Workgroups 0 .. k-1: one per component j, 1024 threads. Thread (band t,
// slice sl) reduces its slice of the chunk sums and of V^T vbar (8 slices of
// 128 bands, or 4 of 256); the slices are added in slice order through LDS;
// w_j = V u is formed one row per wave step with a wave-wide sum.
// Workgroup k: the chunk sums 1^T X and 1^T Qbar. Every reduction has a
// fixed order.
__global__ __launch_bounds__(kWThreads) void bwd_w_kernel(int m, int k, int nchunks, int kg,
                                                          const double *__restrict__ part,
                                                          const float *__restrict__ lam,
                                                          const float *__restrict__ V,
                                                          const float *__restrict__ dVk,
                                                          double *__restrict__ wbuf, double *__restrict__ sums)
{
    __shared__ double red[kWMaxSlices][256];
    __shared__ double vb[256];
    __shared__ double u[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ns = m <= 128 ? 8 : 4;
    const int bw = kWThreads / ns;               // 128 or 256 bands per slice
    const int t = tid % bw, sl = tid / bw;
    const int j = blockIdx.x;
    const int64_t ps = part_stride(m);
    const int64_t cstride = (int64_t)kg * ps;
    auto combine = [&](int b) {
        double a = 0.0;
        for (int q = 0; q < ns; ++q) a += red[q][b];
        return a;
    };
    if (j == k) {
        // sums[0 .. m) = 1^T X, sums[m .. m+k) = 1^T Qbar.
        if (t < m) red[sl][t] = slice_sum(part + kCompGroup * m + kCompGroup + t, cstride, nchunks, sl, ns);
        __syncthreads();
        if (tid < m) sums[tid] = combine(tid);
        __syncthreads();
        if (t < k) red[sl][t] = slice_sum(part + (int64_t)(t / kCompGroup) * ps + kCompGroup * m + t % kCompGroup,
                                          cstride, nchunks, sl, ns);
        __syncthreads();
        if (tid < k) sums[m + tid] = combine(tid);
        return;
    }
    const int g = j / kCompGroup, jj = j % kCompGroup;
    // vbar_j = sum over chunks of X^T Qbar[:, j], plus Vbar_k[:, j].
    if (t < m) red[sl][t] = slice_sum(part + (int64_t)g * ps + t * kCompGroup + jj, cstride, nchunks, sl, ns);
    __syncthreads();
    if (tid < m) {
        double a = combine(tid);
        if (dVk) a += (double)dVk[(int64_t)tid * k + j];
        vb[tid] = a;
    }
    __syncthreads();
    // (V^T vbar)_t over rows b = sl, sl + ns, ...
    if (t < m) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        int b = sl, q = 0;
        for (; b < m; b += ns, q = (q + 1) & 3) a[q] += (double)V[(int64_t)b * m + t] * vb[b];
        red[sl][t] = (a[0] + a[1]) + (a[2] + a[3]);
    }
    __syncthreads();
    if (tid < m) {
        const double T = combine(tid);
        const double li = (double)lam[tid], lj = (double)lam[j];
        u[tid] = (tid == j || li == lj) ? 0.0 : T / (lj - li);
    }
    __syncthreads();
    // w_j[a] = sum_i V[a][i] u[i]: wave `wave` takes rows wave, wave + 16, ...
    for (int a = wave; a < m; a += kWThreads / 64) {
        double x = 0.0;
        for (int i = lane; i < m; i += 64) x += (double)V[(int64_t)a * m + i] * u[i];
        x = wave_sum(x);
        if (lane == 0) wbuf[(int64_t)a * k + j] = x;
    }
}

__global__ __launch_bounds__(kThreads) void bwd_g_kernel(int64_t n, int m, int k, const float *__restrict__ V,
                                                         const float *__restrict__ dEig,
                                                         const double *__restrict__ wbuf, float *__restrict__ G)
{
    const int a = blockIdx.y * 16 + threadIdx.x / 16;
    const int b = blockIdx.x * 16 + threadIdx.x % 16;
    if (a >= m || b >= m) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j)
        s += wbuf[(int64_t)a * k + j] * (double)V[(int64_t)b * m + j] +
             (double)V[(int64_t)a * m + j] * wbuf[(int64_t)b * k + j];
    s *= 0.5;
    if (dEig)
        for (int j = 0; j < m; ++j) s += (double)dEig[j] * (double)V[(int64_t)a * m + j] * (double)V[(int64_t)b * m + j];
    G[(int64_t)a * m + b] = (float)(2.0 / (double)(n - 1) * s);
}

__global__ __launch_bounds__(kThreads) void bwd_r_kernel(int64_t n, int m, int k, const float *__restrict__ V,
                                                         const double *__restrict__ sums, float *__restrict__ G)
{
    for (int c = threadIdx.x; c < m; c += kThreads) {
        double r = 0.0;
        for (int j = 0; j < k; ++j) {
            const float v = V[(int64_t)c * m + j];
            G[(int64_t)(m + j) * m + c] = v;
            r += sums[m + j] * (double)v;
        }
        // Eight interleaved partial sums (eight loads in flight), added in a
        // fixed order.
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int b = 0;
        for (; b + 8 <= m; b += 8) {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] += sums[b + i] * (double)G[(int64_t)(b + i) * m + c];
        }
        for (int i = 0; b < m; ++b, ++i) a[i] += sums[b] * (double)G[(int64_t)b * m + c];
        r += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        G[(int64_t)(m + k) * m + c] = (float)(-r / (double)n);
    }
}

// NT: 32-column tiles of dY held per wave (4 for up to 128 bands, else 8;
// fewer accumulators leave room for more waves per SIMD).
template <int NT, bool BSQ>
__global__ __launch_bounds__(kThreads, NT == 4 ? 2 : 1) void bwd_apply_kernel(const float *__restrict__ Y, int64_t n, int m,
                                                             int64_t ld, const float *__restrict__ mean,
                                                             const float *__restrict__ dQ, int k,
                                                             const float *__restrict__ G, float *__restrict__ dY,
                                                             int64_t ldd)
{
    __shared__ float At[kApplyPix * kApplyPitch];
    __shared__ float Bt[kApplyK * 256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kApplyPix;
    const int K = m + k + 1;
    const int ntiles = (m + 31) / 32;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

    // Slab kc of the augmented operand: thread tid holds column kc + tid % 32
    // of pixel rows tid / 32 + 8 i (raw values; centred when staged), and
    // rows kc .. kc+31 of G at column tid.
    constexpr int kRowsPer = kApplyPix / (kThreads / kApplyK);
    const int kk0 = tid % kApplyK, pr0 = tid / kApplyK;
    float va[kRowsPer], vg[kApplyK];
    auto load = [&](int kc) {
        const int c = kc + kk0;
#pragma unroll
        for (int i = 0; i < kRowsPer; ++i) {
            const int64_t p = base + pr0 + (kThreads / kApplyK) * i;
            float v = 0.f;
            if (p < n) {
                if (c < m) v = Y[BSQ ? (int64_t)c * ld + p : p * ld + c];
                else if (c < m + k) v = dQ ? dQ[p * k + (c - m)] : 0.f;
                else if (c == m + k) v = 1.f;
            }
            va[i] = v;
        }
#pragma unroll
        for (int r = 0; r < kApplyK; ++r) {
            const int cr = kc + r;
            vg[r] = (cr < K && tid < m) ? G[(int64_t)cr * m + tid] : 0.f;
        }
    };
    load(0);
    for (int kc = 0; kc < K; kc += kApplyK) {
        __syncthreads();
        {
            const int c = kc + kk0;
            const float mu = c < m ? mean[c] : 0.f;
#pragma unroll
            for (int i = 0; i < kRowsPer; ++i) At[(pr0 + (kThreads / kApplyK) * i) * kApplyPitch + kk0] = va[i] - mu;
#pragma unroll
            for (int r = 0; r < kApplyK; ++r) Bt[r * 256 + tid] = vg[r];
        }
        __syncthreads();
        if (kc + kApplyK < K) load(kc + kApplyK);
#pragma unroll 4
        for (int s = 0; s < kApplyK / 2; ++s) {
            const int kk = 2 * s + (lane >> 5);
            const float a = At[(32 * wave + (lane & 31)) * kApplyPitch + kk];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t < ntiles) {
                    const float b = Bt[kk * 256 + 32 * t + (lane & 31)];
                    acc[t] = BSQ ? __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc[t], 0, 0, 0)
                                 : __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    }
    // 32x32 result layout: lane l, register r -> row 8 (r/4) + 4 (l/32) + r%4,
    // column l % 32 (rows pixels and columns bands; the other way round for
    // band-sequential cubes).
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t < ntiles) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
                if constexpr (BSQ) {
                    const int band = 32 * t + row;
                    const int64_t p = base + 32 * wave + (lane & 31);
                    if (p < n && band < m) dY[(int64_t)band * ldd + p] = acc[t][r];
                } else {
                    const int col = 32 * t + (lane & 31);
                    const int64_t p = base + 32 * wave + row;
                    if (p < n && col < m) dY[p * ldd + col] = acc[t][r];
                }
            }
        }
    }
}

}  // namespace

BwdPlan bwd_plan(int64_t n, int m, int k)
{
    BwdPlan p;
    p.kg = (k + kCompGroup - 1) / kCompGroup;
    int64_t nch = (n + 63) / 64;
    if (nch > 1024) nch = 1024;
    const int64_t per = (int64_t)p.kg * part_stride(m) * (int64_t)sizeof(double);
    const int64_t cap = ((int64_t)32 << 20) / (per > 0 ? per : 1);
    if (nch > cap) nch = cap;
    if (nch < 1) nch = 1;
    p.chunk = (n + nch - 1) / nch;
    p.nchunks = (int)((n + p.chunk - 1) / p.chunk);
    p.bytes_part = (size_t)p.nchunks * (size_t)per;
    p.bytes_w = (size_t)m * k * sizeof(double);
    p.bytes_sums = (size_t)(m + k) * sizeof(double);
    p.bytes_g = (size_t)(m + k + 1) * m * sizeof(float);
    return p;
}

hipError_t launch_backward(const float *Y, int bsq, int64_t n, int m, int64_t ld, const float *mean, const float *lam,
                           const float *V, int k, const float *dQ, const float *dEig, const float *dVk,
                           float *dY, int64_t ldd, const BwdPlan &p, double *part, double *wbuf, double *sums,
                           float *G, hipStream_t st)
{
    const dim3 gr((unsigned)p.nchunks, (unsigned)p.kg);
    if (bsq)
        hipLaunchKernelGGL(bwd_reduce_kernel<true>, gr, dim3(kThreads), 0, st, Y, n, m, ld, mean, dQ, k, p.chunk, p.kg,
                           part);
    else
        hipLaunchKernelGGL(bwd_reduce_kernel<false>, gr, dim3(kThreads), 0, st, Y, n, m, ld, mean, dQ, k, p.chunk, p.kg,
                           part);
    hipLaunchKernelGGL(bwd_w_kernel, dim3((unsigned)(k + 1)), dim3(kWThreads), 0, st, m, k, p.nchunks, p.kg,
                       (const double *)part, lam, V, dVk, wbuf, sums);
    const unsigned tb = (unsigned)((m + 15) / 16);
    hipLaunchKernelGGL(bwd_g_kernel, dim3(tb, tb), dim3(kThreads), 0, st, n, m, k, V, dEig, (const double *)wbuf, G);
    hipLaunchKernelGGL(bwd_r_kernel, dim3(1), dim3(kThreads), 0, st, n, m, k, V, (const double *)sums, G);
    const dim3 ga((unsigned)((n + kApplyPix - 1) / kApplyPix));
#define PCA_BWD_APPLY(NT, B)                                                                                     \
    hipLaunchKernelGGL((bwd_apply_kernel<NT, B>), ga, dim3(kThreads), 0, st, Y, n, m, ld, mean, dQ, k, (const float *)G, \
                       dY, ldd)
    if (m <= 128) {
        if (bsq) PCA_BWD_APPLY(4, true);
        else PCA_BWD_APPLY(4, false);
    } else {
        if (bsq) PCA_BWD_APPLY(8, true);
        else PCA_BWD_APPLY(8, false);
    }
#undef PCA_BWD_APPLY
    return hipGetLastError();
}

}  // namespace pca

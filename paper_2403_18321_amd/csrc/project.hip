// Projection of every pixel onto the first k eigenvectors (Algorithm 1, lines
// 5-6): Q'[p, i] = sum_b (Y[p, b] - mu_b) V[b, i], i < k.
//
// Persistent workgroups walk over tiles of pixels. A tile is read from HBM
// with coalesced row loads, centred on the way into LDS (the centred cube is
// never written back), and multiplied by the block V[:, 16g .. 16g+15] with
// v_mfma_f32_16x16x4_f32 (K = bands). The eigenvector block stays in LDS for
// the workgroup's lifetime, which leaves the registers to the tiles in
// flight. The cube is read once per group of 16 components (once for k <= 16).
//
// Tiles of 32 pixels, three workgroups per CU, and the loads of the next two
// tiles of a workgroup in flight while it stages and multiplies the current
// one, so that enough of the cube is in flight to keep HBM busy. Waves 0/1
// multiply pixels 0-15/16-31 over the first half of the bands, waves 2/3 over
// the second half; the halves are added through LDS. project_kernel walks the
// tiles of one cube; project_batched_kernel runs the same body over runs of
// tiles of the cubes of a batch.
#include "common.hpp"
#include "kernels.hpp"
#include "loader.hpp"

namespace pca {

namespace {

constexpr int kThreads = 256;
constexpr int kTP = 64;                  // pixels per batched work-item tile unit (kProjTile)
constexpr int kMaxKSteps = 64;           // 256 bands / 4

// Tile pitch (floats): a multiple of 4 with pitch/4 odd, so the 16 pixels x 4
// bands read by one MFMA operand load hit 64 distinct LDS banks.
__host__ __device__ inline int proj_pitch(int m4) { return ((m4 / 4) & 1) ? m4 : m4 + 4; }

constexpr int kTS = 32;          // pixels per tile of project_kernel (4 waves x 8 rows)
constexpr int kWGPerCUS = 3;       // LDS: 3 x 52.7 KB
constexpr int kMaxHalf = 32;     // K steps per half of the bands (256 / 4 / 2)

template <typename T, int VEC>
__device__ __forceinline__ void project_stream_body(const T *__restrict__ Y, int64_t n, int m, int64_t ld,
                                                    const float *__restrict__ mean, const float *__restrict__ V,
                                                    int k, float *__restrict__ Q, int64_t t0, int64_t tstep,
                                                    int64_t ntiles, int g)
{
    __shared__ __attribute__((aligned(16))) float tile[kTS * 260];
    __shared__ float mu[256];
    __shared__ f32x4 red[2][64];
    __shared__ float vsh[kMaxKSteps][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m4 = round_up(m, 4);
    const int pitch = proj_pitch(m4);
    const int ksteps = m4 / 4;
    const int half = (ksteps + 1) / 2;
    const int gq = wave & 1, h = wave >> 1;
    const int s0 = h * half;
    const int ns = min(half, ksteps - s0);

    for (int b = tid; b < 256; b += kThreads) mu[b] = (mean && b < m) ? mean[b] : 0.f;

    // B operand of K step s, lane l: V[4 s + l/16][16g + l%16], kept in LDS
    // (read once per product; registers go to the tiles in flight).
    for (int e = tid; e < ksteps * 64; e += kThreads) {
        const int sk = e >> 6, l = e & 63;
        const int b = 4 * sk + (l >> 4), o = 16 * g + (l & 15);
        vsh[sk][l] = (b < m && o < k) ? V[(int64_t)b * m + o] : 0.f;
    }
    __syncthreads();
    // This lane's four band means (the 16-byte path reads bands 4 lane ..
    // 4 lane + 3 of every row): held in registers, since reading them from
    // LDS at a stride of four words would conflict on the banks.
    f32x4 mu4;
#pragma unroll
    for (int s = 0; s < 4; ++s) mu4[s] = mu[(4 * lane + s) & 255];
    const float *bcol = &vsh[s0][lane];

    const float *arow = &tile[(16 * gq + (lane & 15)) * pitch + 4 * s0 + (lane >> 4)];
    // One tile: stage (centre into LDS), refill the group's registers with the
    // tile two steps ahead, multiply, add the band halves, store.
    auto step = [&](Group<T, VEC> &v, int64_t t) {
        const int64_t pg = t * kTS + 8 * wave;
        if constexpr (VEC == 4) {
            const int b = 4 * lane;
            if (b < m4) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    f32x4 q;
#pragma unroll
                    for (int s = 0; s < 4; ++s) q[s] = (b + s < m && pg + i < n) ? v.get(i, s) - mu4[s] : 0.f;
                    *reinterpret_cast<f32x4 *>(&tile[(8 * wave + i) * pitch + b]) = q;
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int b = lane + 64 * s;
                if (b < m4) {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        tile[(8 * wave + i) * pitch + b] = (b < m && pg + i < n) ? v.get(i, s) - mu[b] : 0.f;
                }
            }
        }
        __syncthreads();
        const int64_t tn = t + 2 * tstep;
        if (tn < ntiles) v.load(Y, ld, tn * kTS + 8 * wave, n, m, lane);

        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < kMaxHalf; ++s) {
            if (s < ns) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[4 * s], bcol[64 * s], acc, 0, 0, 0);
        }
        if (h == 1) red[gq][lane] = acc;
        __syncthreads();
        if (h == 0) {
            acc += red[gq][lane];
            // 16x16 result layout: lane holds rows 4 (lane/16) + r, column lane % 16.
            const int o = 16 * g + (lane & 15);
            if (o < k) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t p = t * kTS + 16 * gq + 4 * (lane >> 4) + r;
                    if (p < n) Q[p * k + o] = acc[r];
                }
            }
        }
    };

    Group<T, VEC> va, vb;
    int64_t t = t0;
    if (t < ntiles) va.load(Y, ld, t * kTS + 8 * wave, n, m, lane);
    if (t + tstep < ntiles) vb.load(Y, ld, (t + tstep) * kTS + 8 * wave, n, m, lane);
    while (t < ntiles) {
        step(va, t);
        t += tstep;
        if (t >= ntiles) break;
        step(vb, t);
        t += tstep;
    }
}

template <typename T, int VEC>
__global__ __launch_bounds__(kThreads, kWGPerCUS) void project_kernel(const T *__restrict__ Y, int64_t n, int m,
                                                           int64_t ld, const float *__restrict__ mean,
                                                           const float *__restrict__ V, int k,
                                                           float *__restrict__ Q)
{
    project_stream_body<T, VEC>(Y, n, m, ld, mean, V, k, Q, (int64_t)blockIdx.x, (int64_t)gridDim.x,
                                (n + kTS - 1) / kTS, (int)blockIdx.y);
}

// Batched: one work item = a run of tiles of one cube; blockIdx.y = the
// 16-component group (workgroups beyond a cube's k return at once).
template <typename T>
__global__ __launch_bounds__(kThreads, kWGPerCUS) void project_batched_kernel(const char *ws, int nc)
{
    const BatchCube *t = reinterpret_cast<const BatchCube *>(ws + sizeof(BatchHeader));
    const int64_t item = blockIdx.x;
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (t[mid].w_proj <= item) lo = mid;
        else hi = mid - 1;
    }
    const BatchCube &cb = t[lo];
    const int g = blockIdx.y;
    if (16 * g >= cb.k) return;
    // A work item is proj_tiles 64-pixel tiles, i.e. twice as many 32-pixel ones.
    const int64_t ntiles = (cb.n + kTS - 1) / kTS;
    const int64_t per = (int64_t)cb.proj_tiles * (kTP / kTS);
    const int64_t t0 = (item - cb.w_proj) * per;
    const int64_t t1 = (t0 + per < ntiles) ? t0 + per : ntiles;
    project_stream_body<T, 1>(static_cast<const T *>(cb.Y), cb.n, cb.m, cb.ld, cb.mean, cb.V, cb.k, cb.Q, t0, 1, t1,
                              g);
}

int num_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

template <typename T>
hipError_t launch_t(const T *Y, int64_t n, int m, int64_t ld, const float *mean, const float *V, int k,
                    float *Q, hipStream_t st, bool v4)
{
    const int64_t ntiles = (n + kTS - 1) / kTS;
    int64_t gx = (int64_t)num_cus() * kWGPerCUS;
    if (gx > ntiles) gx = ntiles;
    dim3 grid((unsigned)gx, (unsigned)((k + 15) / 16)), block(kThreads);
    if (v4)
        hipLaunchKernelGGL((project_kernel<T, 4>), grid, block, 0, st, Y, n, m, ld, mean, V, k, Q);
    else
        hipLaunchKernelGGL((project_kernel<T, 1>), grid, block, 0, st, Y, n, m, ld, mean, V, k, Q);
    return hipGetLastError();
}

// Band-sequential cubes (Y[b * ld + p]): one thread per pixel, consecutive
// threads on consecutive pixels so that every band row is read coalesced;
// the block V[:, 16 g .. 16 g + 15] and the mean sit in LDS, where all lanes
// read the same entry at a time (a broadcast). Float32 FMA chains per pixel,
// bands in order.
// Pixels p0, p0 + step, ... below p1, component group g.
template <typename T>
__device__ __forceinline__ void project_bsq_body(const T *__restrict__ Y, int m, int64_t ld,
                                                 const float *__restrict__ mean, const float *__restrict__ V, int k,
                                                 float *__restrict__ Q, int g, int64_t p0, int64_t p1, int64_t step)
{
    __shared__ __attribute__((aligned(16))) float vs[256][16];
    __shared__ float mu[256];
    for (int e = threadIdx.x; e < 256 * 16; e += kThreads) {
        const int b = e >> 4, o = 16 * g + (e & 15);
        vs[b][e & 15] = (b < m && o < k) ? V[(int64_t)b * m + o] : 0.f;
    }
    for (int b = threadIdx.x; b < 256; b += kThreads) mu[b] = (mean && b < m) ? mean[b] : 0.f;
    __syncthreads();
    const int ncol = (k - 16 * g) < 16 ? (k - 16 * g) : 16;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += step) {
        float acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.f;
        const T *col = Y + p;
#pragma unroll 4
        for (int b = 0; b < m; ++b) {
            const float x = load_elem(col + (int64_t)b * ld) - mu[b];
            const f32x4 *vr = reinterpret_cast<const f32x4 *>(vs[b]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 w = vr[q];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[4 * q + r] = fmaf(x, w[r], acc[4 * q + r]);
            }
        }
        float *out = Q + p * k + 16 * g;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < ncol) out[j] = acc[j];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void project_bsq_kernel(const T *__restrict__ Y, int64_t n, int m, int64_t ld,
                                                               const float *__restrict__ mean,
                                                               const float *__restrict__ V, int k,
                                                               float *__restrict__ Q)
{
    project_bsq_body<T>(Y, m, ld, mean, V, k, Q, (int)blockIdx.y, (int64_t)blockIdx.x * kThreads, n,
                        (int64_t)gridDim.x * kThreads);
}

// Batched band-sequential cubes: a work item is the same run of pixels as
// project_batched_kernel's (proj_tiles 64-pixel tiles), one thread a pixel.
template <typename T>
__global__ __launch_bounds__(kThreads) void project_batched_bsq_kernel(const char *ws, int nc)
{
    const BatchCube *t = reinterpret_cast<const BatchCube *>(ws + sizeof(BatchHeader));
    const int64_t item = blockIdx.x;
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (t[mid].w_proj <= item) lo = mid;
        else hi = mid - 1;
    }
    const BatchCube &cb = t[lo];
    const int g = blockIdx.y;
    if (16 * g >= cb.k) return;
    const int64_t per = (int64_t)cb.proj_tiles * kTP;
    const int64_t p0 = (item - cb.w_proj) * per;
    const int64_t p1 = (p0 + per < cb.n) ? p0 + per : cb.n;
    project_bsq_body<T>(static_cast<const T *>(cb.Y), cb.m, cb.ld, cb.mean, cb.V, cb.k, cb.Q, g, p0, p1, kThreads);
}

template <typename T>
hipError_t launch_project_bsq(const T *Y, int64_t n, int m, int64_t ld, const float *mean, const float *V, int k,
                              float *Q, hipStream_t st)
{
    int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(project_bsq_kernel<T>, dim3((unsigned)blocks, (unsigned)((k + 15) / 16)), dim3(kThreads), 0,
                       st, Y, n, m, ld, mean, V, k, Q);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project(const void *Y, int dt, int64_t n, int m, int64_t ld, const float *mean,
                          const float *V, int k, float *Q, hipStream_t st)
{
    if (dt == PCA_IN_F32_BSQ) return launch_project_bsq(static_cast<const float *>(Y), n, m, ld, mean, V, k, Q, st);
    if (dt == PCA_IN_U16_BSQ) return launch_project_bsq(static_cast<const uint16_t *>(Y), n, m, ld, mean, V, k, Q, st);
    const bool v4 = vec4_ok(Y, dt, m, ld);
    if (dt == PCA_IN_F32) return launch_t(static_cast<const float *>(Y), n, m, ld, mean, V, k, Q, st, v4);
    return launch_t(static_cast<const uint16_t *>(Y), n, m, ld, mean, V, k, Q, st, v4);
}

hipError_t launch_project_batched(int dt, const char *ws, const int64_t total[6], int n_cubes, int max_k,
                                  hipStream_t st)
{
    const dim3 grid((unsigned)total[5], (unsigned)((max_k + 15) / 16)), block(kThreads);
    if (dt == PCA_IN_F32_BSQ)
        hipLaunchKernelGGL(project_batched_bsq_kernel<float>, grid, block, 0, st, ws, n_cubes);
    else if (dt == PCA_IN_U16_BSQ)
        hipLaunchKernelGGL(project_batched_bsq_kernel<uint16_t>, grid, block, 0, st, ws, n_cubes);
    else if (dt == PCA_IN_F32)
        hipLaunchKernelGGL(project_batched_kernel<float>, grid, block, 0, st, ws, n_cubes);
    else
        hipLaunchKernelGGL(project_batched_kernel<uint16_t>, grid, block, 0, st, ws, n_cubes);
    return hipGetLastError();
}

}  // namespace pca

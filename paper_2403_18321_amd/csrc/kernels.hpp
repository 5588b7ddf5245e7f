// Host-side launchers of the gfx950 kernels (internal to libpca).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pca.h"

namespace pca {

constexpr int kMaxBands = 256;

// ---- covariance ----------------------------------------------------------
constexpr int kCovTile = 32;          // pixels per on-chip stage
constexpr int kCovMaxChunk = 16384;   // pixels per workgroup, upper bound
constexpr int kCovTargetChunks = 256; // one chunk per CU when N allows

struct CovPlan {
    int64_t chunk;     // pixels per workgroup
    int64_t nchunks;   // workgroups / partial results
    int mpad;          // bands rounded up to 32
    int nb;            // 32-wide band blocks
    int nblk;          // upper-triangle blocks nb (nb + 1) / 2
    size_t bytes_S;    // partial second moments, float32
    size_t bytes_sum;  // partial sums, float64
    size_t bytes_shift;  // per-chunk shifts, float32
    int groups;          // chunk groups of the first finalize pass
    size_t bytes_part2;  // float64 partial results of those groups + means
    size_t bytes_srow;   // shift row: float32 [256], the same row in the cube's type [256], then the
                         // float16 split's band scales sc [256] and 1 / sc [256]
};
CovPlan cov_plan(int64_t n, int m);

// Plan for a given chunk length (rounded to whole 32-pixel stages, at most
// kCovMaxChunk); the single-cube plan picks the chunk from N.
__host__ __device__ inline CovPlan cov_plan_chunk(int64_t n, int m, int64_t chunk)
{
    CovPlan p;
    int64_t c = (chunk + kCovTile - 1) / kCovTile * kCovTile;
    if (c < kCovTile) c = kCovTile;
    if (c > kCovMaxChunk) c = kCovMaxChunk;
    p.chunk = c;
    p.nchunks = (n + p.chunk - 1) / p.chunk;
    p.mpad = (m + 31) / 32 * 32;
    p.nb = p.mpad / 32;
    p.nblk = p.nb * (p.nb + 1) / 2;
    p.bytes_S = (size_t)p.nchunks * p.nblk * 1024 * sizeof(float);
    p.bytes_sum = (size_t)p.nchunks * p.mpad * sizeof(double);
    p.bytes_shift = (size_t)p.nchunks * p.mpad * sizeof(float);
    p.groups = (int)(p.nchunks < 8 ? p.nchunks : 8);
    p.bytes_part2 = ((size_t)p.groups * p.nblk * 1024 + 1 + 256) * sizeof(double);
    p.bytes_srow = 4 * 256 * sizeof(float);
    return p;
}

// The batched form's plan for one cube: at most two chunk groups in the
// finalisation (a batch has work items enough without more, and each item
// carries a fixed cost of table search and band means).
constexpr int kBatchFinGroups = 2;
__host__ __device__ inline CovPlan batch_cov_plan(int64_t n, int m, int64_t chunk)
{
    CovPlan p = cov_plan_chunk(n, m, chunk);
    p.groups = (int)(p.nchunks < kBatchFinGroups ? p.nchunks : kBatchFinGroups);
    p.bytes_part2 = ((size_t)p.groups * p.nblk * 1024 + 1 + 256) * sizeof(double);
    return p;
}

// Pass 0: the shift row (written to srow, read by pass 1).
hipError_t launch_cov_shift(const void *Y, int dt, int64_t n, int m, int64_t ld, const CovPlan &plan, float *srow,
                            hipStream_t st);
hipError_t launch_cov_partial(const void *Y, int dt, int64_t n, int m, int64_t ld, int centered,
                              int mode, const CovPlan &plan, float *partS, double *partSum,
                              float *partShift, const float *srow, hipStream_t st);
hipError_t launch_cov_finalize(int64_t n, int m, int centered, const CovPlan &plan, const float *partS,
                               const double *partSum, const float *partShift, double *part2, float *C,
                               float *mean, hipStream_t st);

// ---- centring --------------------------------------------------------------
hipError_t launch_center(const void *Y, int dt, int64_t n, int m, int64_t ld, float *mean,
                         float *X, int64_t ldx, const CovPlan &plan, double *partSum,
                         double *mean64, hipStream_t st);

// ---- Jacobi ----------------------------------------------------------------
struct JacPlan {
    int me;              // bands rounded up to even
    int npairs;          // me / 2
    int64_t log_steps;   // capacity of the rotation log in steps
    size_t bytes_log;    // float2 per (step, pair)
    size_t bytes_lam;    // unsorted eigenvalues, float64
    size_t bytes_vu;     // unsorted eigenvectors, float32 me x me
    size_t bytes_info;   // internal pca_info
    size_t bytes_block;  // block-cyclic form: matrix tiles, U's, partial sums, step flags
};

// Block-cyclic Jacobi on many CUs (jacobi_block.hip): blocks of 16 indices
// (an even number of them), one workgroup per (row block pair, column block
// pair), P x P workgroups.
constexpr int kBjBlock = 16;
__host__ __device__ inline int bj_blocks(int m)
{
    int nb = (m + kBjBlock - 1) / kBjBlock;
    nb += nb & 1;
    return nb < 2 ? 2 : nb;
}
__host__ __device__ inline size_t bj_workspace_bytes(int m)
{
    const int nb = bj_blocks(m), P = nb / 2;
    const size_t Mp = (size_t)nb * kBjBlock;
    // H (float64, two steps), U (float64, two steps), V (float32), partial
    // sums (two steps, 32 bytes per workgroup), step flags.
    return 2 * Mp * Mp * sizeof(double) + 2 * (size_t)P * 1024 * sizeof(double) + Mp * Mp * sizeof(float) +
           2 * (size_t)P * P * 32 + 256 * sizeof(unsigned int);
}
// Band counts from which pca_jacobi_eigh takes the block-cyclic form by default.
constexpr int kBjMinBands = 96;
// Workgroups of the block-cyclic form (all on one XCD) and column pairs each.
constexpr int kBjMaxGroups = 32;
constexpr int kBjMaxColPairs = 2;

// The rotation log is read in batches of kLogBatch steps while it is written
// (overlapped replay); its capacity covers the batch that holds the step
// after the last one.
constexpr int kLogBatch = 16;
__host__ __device__ inline JacPlan jac_plan(int m, int max_sweeps)
{
    JacPlan p;
    p.me = m + (m & 1);
    p.npairs = p.me / 2;
    p.log_steps = ((int64_t)(max_sweeps > 0 ? max_sweeps : 0) * (p.me - 1) / kLogBatch + 1) * kLogBatch;
    p.bytes_log = (size_t)p.log_steps * p.npairs * 2 * sizeof(float);
    p.bytes_lam = (size_t)p.me * sizeof(double);
    p.bytes_vu = (size_t)p.me * p.me * sizeof(float);
    p.bytes_info = sizeof(pca_info);
    p.bytes_block = bj_workspace_bytes(m);
    return p;
}

// Eigenvector-replay rows per workgroup of the separate replay launch.
__host__ __device__ inline int replay_rows(int me)
{
    const int r = 512 / (me / 2);
    return r > 8 ? 8 : r;
}

// Rows of E per follower workgroup (1024 threads) of the overlapped replay:
// about two replay tasks per thread, at most 32 rows.
constexpr int kFollowMaxRows = 32;
__host__ __device__ inline int follow_rows(int me)
{
    const int r = 2 * 1024 / (me / 2);
    return r < 1 ? 1 : (r > kFollowMaxRows ? kFollowMaxRows : r);
}

// ---- batched form ----------------------------------------------------------
constexpr size_t kBatchAlign = 256;
__host__ __device__ inline size_t batch_al(size_t x) { return (x + kBatchAlign - 1) / kBatchAlign * kBatchAlign; }
constexpr int kBatchDefaultChunk = 4096;   // pixels per covariance work item
constexpr int kBatchDefaultTiles = 16;     // 64-pixel tiles per projection work item
constexpr int kProjTile = 64;

// Per-cube entry of the device task table (written by the set-up kernel from
// the caller's descriptors, in decreasing order of work).
struct BatchCube {
    const void *Y;
    int64_t n, ld;
    int m, k;
    float *mean, *eigvals, *V, *Q;
    pca_info *info;
    CovPlan cov;
    float *partS;
    double *partSum;
    float *partShift;
    float *srow;
    double *part2;
    float *C;
    float2 *rlog;
    double *lam_u;
    float *Vu;
    pca_info *info_ws;
    int rows;              // eigenvector rows per follower workgroup of the Jacobi launch
    int proj_tiles;        // 64-pixel tiles per projection work item
    // First global work item of this cube in each batched launch.
    int64_t w_cov, w_fin1, w_fin2, w_rep, w_sort, w_proj;
};

struct BatchHeader {
    int n_cubes;
    int pad;
    int64_t total[6];      // work items of each batched launch
    unsigned int counter[4];
};

// Work items of each launch for one cube.
__host__ __device__ inline void batch_counts(const CovPlan &cp, int64_t n, int m, int tiles, int64_t w[6])
{
    const int me = m + (m & 1);
    w[0] = cp.nchunks;
    w[1] = (int64_t)cp.nblk * cp.groups;
    w[2] = cp.nblk;
    w[3] = (me + follow_rows(me) - 1) / follow_rows(me);
    w[4] = (m + 3) / 4;
    w[5] = ((n + kProjTile - 1) / kProjTile + tiles - 1) / tiles;
}

// Workspace bytes of one cube (after the table).
__host__ __device__ inline size_t batch_cube_bytes(const CovPlan &cp, const JacPlan &jp, int m)
{
    return batch_al(cp.bytes_S) + batch_al(cp.bytes_sum) + batch_al(cp.bytes_shift) + batch_al(cp.bytes_srow) +
           batch_al(cp.bytes_part2) +
           batch_al((size_t)m * m * sizeof(float)) + batch_al(jp.bytes_log) + batch_al(jp.bytes_lam) +
           batch_al(jp.bytes_vu) + batch_al(jp.bytes_info);
}

__host__ __device__ inline size_t batch_table_bytes(int n_cubes)
{
    return batch_al(sizeof(BatchHeader) + (size_t)n_cubes * sizeof(BatchCube));
}

hipError_t launch_batch_setup(const pca_cube *cubes_dev, int n_cubes, int mode, int max_sweeps, int cov_chunk,
                              int proj_tiles, char *ws, hipStream_t st);
hipError_t launch_cov_batched(int dt, int mode, const char *ws, const int64_t total[6], int n_cubes, hipStream_t st);
hipError_t launch_jacobi_batched(const char *ws, const int64_t total[6], int n_cubes, double tol, int max_sweeps,
                                 int fp64_angles, hipStream_t st);
hipError_t launch_project_batched(int dt, const char *ws, const int64_t total[6], int n_cubes, int max_k,
                                  hipStream_t st);

// ---- backward ----------------------------------------------------------------
struct BwdPlan {
    int kg;              // groups of 8 components
    int64_t chunk;       // pixels per reduction workgroup
    int nchunks;
    size_t bytes_part;   // float64 partial sums per (chunk, group)
    size_t bytes_w;      // w_j vectors, float64 M x k
    size_t bytes_sums;   // 1^T X and 1^T Qbar, float64
    size_t bytes_g;      // augmented GEMM operand, float32 (M + k + 1) x M
};
BwdPlan bwd_plan(int64_t n, int m, int k);

hipError_t launch_backward(const float *Y, int bsq, int64_t n, int m, int64_t ld, const float *mean, const float *lam,
                           const float *V, int k, const float *dQ, const float *dEig, const float *dVk,
                           float *dY, int64_t ldd, const BwdPlan &p, double *part, double *wbuf, double *sums,
                           float *G, hipStream_t st);

// overlap = 1: the eigenvector replay runs in the Jacobi launch itself, on
// workgroups that follow the rotation log as it is written (the log must
// start zeroed; every call leaves it zeroed).
hipError_t launch_jacobi(const float *C, int m, double tol, int max_sweeps, int fp64_angles, int overlap,
                         const JacPlan &plan, double *lam_u, float2 *log, float *Vu,
                         pca_info *info_ws, float *eigvals, float *V, pca_info *info_out,
                         hipStream_t st);

hipError_t launch_jacobi_block(const float *C, int m, double tol, int max_sweeps, int fp64_angles, char *ws,
                               double *lam_u, float *VuT, int nvu, pca_info *info_ws, hipStream_t st);
hipError_t launch_sort_sign(int m, int n, const double *lam_u, const float *Vu, const pca_info *info_ws,
                            float *eigvals, float *V, pca_info *info_out, hipStream_t st);
// Divides the bounded waits of the Jacobi kernels by 2^shift (tests of the
// failure handling; synchronous copies to the current device).
hipError_t set_wait_shift_one_cu(int shift);
hipError_t set_wait_shift_block(int shift);

// ---- projection ------------------------------------------------------------
hipError_t launch_project(const void *Y, int dt, int64_t n, int m, int64_t ld, const float *mean,
                          const float *V, int k, float *Q, hipStream_t st);

}  // namespace pca

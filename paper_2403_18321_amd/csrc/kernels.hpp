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
};
CovPlan cov_plan(int64_t n, int m);

hipError_t launch_cov_partial(const void *Y, int dt, int64_t n, int m, int64_t ld, int centered,
                              int mode, const CovPlan &plan, float *partS, double *partSum,
                              float *partShift, hipStream_t st);
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
};
JacPlan jac_plan(int m, int max_sweeps);

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

hipError_t launch_backward(const float *Y, int64_t n, int m, int64_t ld, const float *mean, const float *lam,
                           const float *V, int k, const float *dQ, const float *dEig, const float *dVk,
                           float *dY, int64_t ldd, const BwdPlan &p, double *part, double *wbuf, double *sums,
                           float *G, hipStream_t st);

hipError_t launch_jacobi(const float *C, int m, double tol, int max_sweeps, int fp64_angles,
                         const JacPlan &plan, double *lam_u, float2 *log, float *Vu,
                         pca_info *info_ws, float *eigvals, float *V, pca_info *info_out,
                         hipStream_t st);

// ---- projection ------------------------------------------------------------
hipError_t launch_project(const void *Y, int dt, int64_t n, int m, int64_t ld, const float *mean,
                          const float *V, int k, float *Q, hipStream_t st);

}  // namespace pca

// C ABI of libpca: argument validation, workspace layout and kernel launches.
// Declarations and the contract of every entry point are in include/pca.h.
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "kernels.hpp"
#include "pca.h"

// Device memory of pca_jacobi_eigh_noalloc: one copy per GPU, held until the
// process ends. Host code takes its address only through scratch_ptr().
static __device__ __align__(256) unsigned char scratch[PCA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kWsAlign = 256;
inline size_t al(size_t x) { return (x + kWsAlign - 1) / kWsAlign * kWsAlign; }

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline bool valid_dt(int dt) { return dt == PCA_IN_F32 || dt == PCA_IN_U16; }   // BIP
inline bool is_bsq(int dt) { return dt == PCA_IN_F32_BSQ || dt == PCA_IN_U16_BSQ; }

// A cube of either layout: ld is the stride between pixels (BIP, >= m) or
// between bands (BSQ, >= n).
inline pca_status check_cube(const void *Y, int dt, int64_t n, int32_t m, int64_t ld)
{
    if (!Y || !(valid_dt(dt) || is_bsq(dt))) return PCA_ERR_ARG;
    if (n < 2 || m < 2 || m > pca::kMaxBands || ld < (is_bsq(dt) ? n : (int64_t)m)) return PCA_ERR_ARG;
    if (!aligned(Y, (dt == PCA_IN_F32 || dt == PCA_IN_F32_BSQ) ? 4 : 2)) return PCA_ERR_ARG;
    return PCA_OK;
}

inline pca_status hip_status(hipError_t e) { return e == hipSuccess ? PCA_OK : PCA_ERR_HIP; }

size_t center_ws(const pca::CovPlan &p, int m) { return al(p.bytes_sum) + al((size_t)m * sizeof(double)); }
size_t cov_ws(const pca::CovPlan &p)
{
    return al(p.bytes_S) + al(p.bytes_sum) + al(p.bytes_shift) + al(p.bytes_part2) + al(p.bytes_srow);
}
size_t jac_ws(const pca::JacPlan &p)
{
    return al(p.bytes_log) + al(p.bytes_lam) + al(p.bytes_vu) + al(p.bytes_info) + al(p.bytes_block);
}
size_t bwd_ws(const pca::BwdPlan &p) { return al(p.bytes_part) + al(p.bytes_w) + al(p.bytes_sums) + al(p.bytes_g); }

// Host-side checks and sizes of a batch; fills the six launch totals. dt
// kAnyU16 checks each cube as uint16 of whichever layout its stride allows.
constexpr int kAnyU16 = -1;
pca_status batch_plan(const pca_cube *cubes, int32_t n_cubes, int32_t max_sweeps, const pca_batch_tuning *tuning,
                      int dt, size_t *bytes, int64_t total[6], int *max_k, int *cov_chunk, int *proj_tiles)
{
    if (!cubes || n_cubes < 1 || n_cubes > 4096 || max_sweeps < 0 || max_sweeps > 100000) return PCA_ERR_ARG;
    int chunk = pca::kBatchDefaultChunk, tiles = pca::kBatchDefaultTiles;
    if (tuning) {
        if (tuning->cov_chunk < 0 || tuning->cov_chunk > pca::kCovMaxChunk || tuning->cov_chunk % pca::kCovTile)
            return PCA_ERR_ARG;
        if (tuning->proj_tiles < 0 || tuning->proj_tiles > 4096) return PCA_ERR_ARG;
        if (tuning->cov_chunk) chunk = tuning->cov_chunk;
        if (tuning->proj_tiles) tiles = tuning->proj_tiles;
    }
    size_t b = pca::batch_table_bytes(n_cubes);
    for (int q = 0; q < 6; ++q) total[q] = 0;
    int mk = 1;
    for (int32_t i = 0; i < n_cubes; ++i) {
        const pca_cube &c = cubes[i];
        const int cdt = dt != kAnyU16 ? dt : (c.ld_y >= c.n_bands ? PCA_IN_U16 : PCA_IN_U16_BSQ);
        pca_status s = check_cube(c.Y, cdt, c.n_pixels, c.n_bands, c.ld_y);
        if (s != PCA_OK) return s;
        if (c.k < 1 || c.k > c.n_bands || !c.mean || !c.eigvals || !c.V || !c.Q) return PCA_ERR_ARG;
        if (!aligned(c.mean, 4) || !aligned(c.eigvals, 4) || !aligned(c.V, 4) || !aligned(c.Q, 4)) return PCA_ERR_ARG;
        if (c.info && !aligned(c.info, 8)) return PCA_ERR_ARG;
        const pca::CovPlan cp = pca::batch_cov_plan(c.n_pixels, c.n_bands, chunk);
        const pca::JacPlan jp = pca::jac_plan(c.n_bands, max_sweeps);
        b += pca::batch_cube_bytes(cp, jp, c.n_bands);
        int64_t cnt[6];
        pca::batch_counts(cp, c.n_pixels, c.n_bands, tiles, cnt);
        for (int q = 0; q < 6; ++q) total[q] += cnt[q];
        if (c.k > mk) mk = c.k;
    }
    for (int q = 0; q < 6; ++q)
        if (total[q] > 0x7fffffffLL) return PCA_ERR_UNSUPPORTED;
    *bytes = b;
    if (max_k) *max_k = mk;
    if (cov_chunk) *cov_chunk = chunk;
    if (proj_tiles) *proj_tiles = tiles;
    return PCA_OK;
}

// The address of this device's copy of `scratch` (hipGetSymbolAddress once
// per device, with that device current), or nullptr if it cannot be had.
constexpr int kMaxDevices = 64;
void *scratch_ptr()
{
    static std::mutex mu;
    static void *ptr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

}  // namespace

extern "C" {

const char *pca_status_string(pca_status s)
{
    switch (s) {
    case PCA_OK: return "PCA_OK";
    case PCA_ERR_ARG: return "PCA_ERR_ARG: invalid argument";
    case PCA_ERR_UNSUPPORTED: return "PCA_ERR_UNSUPPORTED: unsupported request";
    case PCA_ERR_WORKSPACE: return "PCA_ERR_WORKSPACE: workspace too small";
    case PCA_ERR_HIP: return "PCA_ERR_HIP: HIP runtime error";
    }
    return "unknown pca_status";
}

pca_status pca_workspace_size(int op, int64_t n_pixels, int32_t n_bands, int32_t k, int32_t mode,
                              int32_t max_sweeps, size_t *bytes)
{
    if (!bytes || n_bands < 2 || n_bands > pca::kMaxBands) return PCA_ERR_ARG;
    switch (op) {
    case PCA_OP_CENTER:
        if (n_pixels < 2) return PCA_ERR_ARG;
        *bytes = center_ws(pca::cov_plan(n_pixels, n_bands), n_bands);
        return PCA_OK;
    case PCA_OP_COVARIANCE:
        if (n_pixels < 2 || mode < PCA_COV_F32 || mode > PCA_COV_FP16X3) return PCA_ERR_ARG;
        *bytes = cov_ws(pca::cov_plan(n_pixels, n_bands));
        return PCA_OK;
    case PCA_OP_JACOBI:
        if (max_sweeps < 0) return PCA_ERR_ARG;
        *bytes = jac_ws(pca::jac_plan(n_bands, max_sweeps));
        return PCA_OK;
    case PCA_OP_PROJECT:
        *bytes = 0;
        return PCA_OK;
    case PCA_OP_BACKWARD:
        if (n_pixels < 2 || k < 1 || k > n_bands) return PCA_ERR_ARG;
        *bytes = bwd_ws(pca::bwd_plan(n_pixels, n_bands, k));
        return PCA_OK;
    default:
        return PCA_ERR_UNSUPPORTED;
    }
}

pca_status pca_center(const void *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y, float *mean,
                      float *X, int64_t ld_x, void *ws, size_t ws_bytes, void *stream)
{
    pca_status s = check_cube(Y, dt, n_pixels, n_bands, ld_y);
    if (s != PCA_OK) return s;
    if (!mean || !ws || !aligned(ws, kWsAlign) || !aligned(mean, 4)) return PCA_ERR_ARG;
    if (X && (ld_x < (is_bsq(dt) ? n_pixels : (int64_t)n_bands) || !aligned(X, 4))) return PCA_ERR_ARG;
    const pca::CovPlan plan = pca::cov_plan(n_pixels, n_bands);
    if (ws_bytes < center_ws(plan, n_bands)) return PCA_ERR_WORKSPACE;
    char *w = static_cast<char *>(ws);
    double *partSum = reinterpret_cast<double *>(w);
    double *mean64 = reinterpret_cast<double *>(w + al(plan.bytes_sum));
    return hip_status(pca::launch_center(Y, dt, n_pixels, n_bands, ld_y, mean, X, ld_x, plan, partSum, mean64,
                                         static_cast<hipStream_t>(stream)));
}

pca_status pca_covariance(const void *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y,
                          int32_t input_is_centered, float *mean, int mode, float *C, void *ws,
                          size_t ws_bytes, void *stream)
{
    pca_status s = check_cube(Y, dt, n_pixels, n_bands, ld_y);
    if (s != PCA_OK) return s;
    if (!C || !ws || !aligned(ws, kWsAlign) || !aligned(C, 4) || (mean && !aligned(mean, 4))) return PCA_ERR_ARG;
    if (mode < PCA_COV_F32 || mode > PCA_COV_FP16X3) return PCA_ERR_ARG;
    if (input_is_centered != 0 && input_is_centered != 1) return PCA_ERR_ARG;
    const pca::CovPlan plan = pca::cov_plan(n_pixels, n_bands);
    if (ws_bytes < cov_ws(plan)) return PCA_ERR_WORKSPACE;
    char *w = static_cast<char *>(ws);
    float *partS = reinterpret_cast<float *>(w);
    double *partSum = reinterpret_cast<double *>(w + al(plan.bytes_S));
    float *partShift = reinterpret_cast<float *>(w + al(plan.bytes_S) + al(plan.bytes_sum));
    double *part2 = reinterpret_cast<double *>(w + al(plan.bytes_S) + al(plan.bytes_sum) + al(plan.bytes_shift));
    float *srow = reinterpret_cast<float *>(w + al(plan.bytes_S) + al(plan.bytes_sum) + al(plan.bytes_shift) +
                                            al(plan.bytes_part2));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (pca::launch_cov_shift(Y, dt, n_pixels, n_bands, ld_y, plan, srow, st) != hipSuccess) return PCA_ERR_HIP;
    hipError_t e = pca::launch_cov_partial(Y, dt, n_pixels, n_bands, ld_y, input_is_centered, mode, plan, partS,
                                           partSum, partShift, srow, st);
    if (e != hipSuccess) return PCA_ERR_HIP;
    return hip_status(pca::launch_cov_finalize(n_pixels, n_bands, input_is_centered, plan, partS, partSum,
                                               partShift, part2, C, mean, st));
}

pca_status pca_jacobi_eigh(const float *C, int32_t n_bands, double tol, int32_t max_sweeps, int32_t flags,
                           float *eigvals, float *V, pca_info *info, void *ws, size_t ws_bytes, void *stream)
{
    if (!C || !eigvals || !V || !ws) return PCA_ERR_ARG;
    if (n_bands < 2 || n_bands > pca::kMaxBands) return PCA_ERR_ARG;
    if (!(tol >= 0.0) || !isfinite(tol) || max_sweeps < 0 || max_sweeps > 100000) return PCA_ERR_ARG;
    if (flags & ~(PCA_JACOBI_FP64_ANGLES | PCA_JACOBI_OVERLAP_REPLAY | PCA_JACOBI_ONE_CU | PCA_JACOBI_BLOCK))
        return PCA_ERR_ARG;
    if ((flags & PCA_JACOBI_ONE_CU) && (flags & PCA_JACOBI_BLOCK)) return PCA_ERR_ARG;
    if (!aligned(ws, kWsAlign) || !aligned(C, 4) || !aligned(eigvals, 4) || !aligned(V, 4)) return PCA_ERR_ARG;
    if (info && !aligned(info, 8)) return PCA_ERR_ARG;
    const pca::JacPlan plan = pca::jac_plan(n_bands, max_sweeps);
    if (ws_bytes < jac_ws(plan)) return PCA_ERR_WORKSPACE;
    char *w = static_cast<char *>(ws);
    float2 *rlog = reinterpret_cast<float2 *>(w);
    w += al(plan.bytes_log);
    double *lam_u = reinterpret_cast<double *>(w);
    w += al(plan.bytes_lam);
    float *Vu = reinterpret_cast<float *>(w);
    w += al(plan.bytes_vu);
    pca_info *info_ws = reinterpret_cast<pca_info *>(w);
    w += al(plan.bytes_info);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int fp64 = (flags & PCA_JACOBI_FP64_ANGLES) ? 1 : 0;
    const bool block = (flags & PCA_JACOBI_BLOCK) || (!(flags & PCA_JACOBI_ONE_CU) && n_bands >= pca::kBjMinBands);
    if (block) {
        if (pca::launch_jacobi_block(C, n_bands, tol, max_sweeps, fp64, w, lam_u, Vu, plan.me, info_ws, st) !=
            hipSuccess)
            return PCA_ERR_HIP;
        return hip_status(pca::launch_sort_sign(n_bands, plan.me, lam_u, Vu, info_ws, eigvals, V, info, st));
    }
    return hip_status(pca::launch_jacobi(C, n_bands, tol, max_sweeps, fp64, (flags & PCA_JACOBI_OVERLAP_REPLAY) ? 1 : 0,
                                         plan, lam_u, rlog, Vu, info_ws, eigvals, V, info, st));
}

pca_status pca_jacobi_eigh_noalloc(const float *C, int32_t n_bands, double tol, int32_t max_sweeps, int32_t flags,
                                   float *eigvals, float *V, pca_info *info, void *stream)
{
    if (n_bands < 2 || n_bands > pca::kMaxBands || max_sweeps < 0 || max_sweeps > 100000) return PCA_ERR_ARG;
    if (jac_ws(pca::jac_plan(n_bands, max_sweeps)) > PCA_NOALLOC_SCRATCH_BYTES) return PCA_ERR_WORKSPACE;
    void *ws = scratch_ptr();
    if (!ws) return PCA_ERR_HIP;
    return pca_jacobi_eigh(C, n_bands, tol, max_sweeps, flags, eigvals, V, info, ws, PCA_NOALLOC_SCRATCH_BYTES, stream);
}

pca_status pca_project(const void *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y, const float *mean,
                       const float *V, int32_t k, float *Q, void *stream)
{
    pca_status s = check_cube(Y, dt, n_pixels, n_bands, ld_y);
    if (s != PCA_OK) return s;
    if (!V || !Q || k < 1 || k > n_bands) return PCA_ERR_ARG;
    if (!aligned(V, 4) || !aligned(Q, 4) || (mean && !aligned(mean, 4))) return PCA_ERR_ARG;
    return hip_status(pca::launch_project(Y, dt, n_pixels, n_bands, ld_y, mean, V, k, Q,
                                          static_cast<hipStream_t>(stream)));
}

pca_status pca_backward(const float *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y, const float *mean,
                        const float *eigvals, const float *V, int32_t k, const float *dQ, const float *dEig,
                        const float *dVk, float *dY, int64_t ld_dy, void *ws, size_t ws_bytes, void *stream)
{
    if (dt != PCA_IN_F32 && dt != PCA_IN_F32_BSQ) return PCA_ERR_ARG;
    pca_status s = check_cube(Y, dt, n_pixels, n_bands, ld_y);
    if (s != PCA_OK) return s;
    const bool bsq = dt == PCA_IN_F32_BSQ;
    if (!mean || !eigvals || !V || !dY || !ws || k < 1 || k > n_bands || ld_dy < (bsq ? n_pixels : (int64_t)n_bands))
        return PCA_ERR_ARG;
    if (!aligned(mean, 4) || !aligned(eigvals, 4) || !aligned(V, 4) || !aligned(dY, 4) || !aligned(ws, kWsAlign))
        return PCA_ERR_ARG;
    if ((dQ && !aligned(dQ, 4)) || (dEig && !aligned(dEig, 4)) || (dVk && !aligned(dVk, 4))) return PCA_ERR_ARG;
    const pca::BwdPlan plan = pca::bwd_plan(n_pixels, n_bands, k);
    if (ws_bytes < bwd_ws(plan)) return PCA_ERR_WORKSPACE;
    char *w = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(w);
    w += al(plan.bytes_part);
    double *wbuf = reinterpret_cast<double *>(w);
    w += al(plan.bytes_w);
    double *sums = reinterpret_cast<double *>(w);
    w += al(plan.bytes_sums);
    float *G = reinterpret_cast<float *>(w);
    return hip_status(pca::launch_backward(Y, bsq ? 1 : 0, n_pixels, n_bands, ld_y, mean, eigvals, V, k, dQ, dEig, dVk,
                                           dY, ld_dy,
                                           plan, part, wbuf, sums, G, static_cast<hipStream_t>(stream)));
}

pca_status pca_batched_workspace_size(const pca_cube *cubes, int32_t n_cubes, int mode, int32_t max_sweeps,
                                      const pca_batch_tuning *tuning, size_t *bytes)
{
    if (!bytes || mode < PCA_COV_F32 || mode > PCA_COV_FP16X3) return PCA_ERR_ARG;
    int64_t total[6];
    // Neither the element type nor the layout changes the sizes: check the
    // cubes here as uint16 of either layout, pca_batched checks them again.
    return batch_plan(cubes, n_cubes, max_sweeps, tuning, kAnyU16, bytes, total, nullptr, nullptr, nullptr);
}

pca_status pca_batched(const pca_cube *cubes, const pca_cube *cubes_dev, int32_t n_cubes, int dt, int mode,
                       double tol, int32_t max_sweeps, int32_t fp64_angles, const pca_batch_tuning *tuning,
                       void *ws, size_t ws_bytes, void *stream)
{
    if (!cubes_dev || !aligned(cubes_dev, 8) || !ws || !aligned(ws, kWsAlign) || !(valid_dt(dt) || is_bsq(dt)))
        return PCA_ERR_ARG;
    if (mode < PCA_COV_F32 || mode > PCA_COV_FP16X3) return PCA_ERR_ARG;
    if (!(tol >= 0.0) || !isfinite(tol) || (fp64_angles != 0 && fp64_angles != 1)) return PCA_ERR_ARG;
    size_t need = 0;
    int64_t total[6];
    int max_k = 1, chunk = 0, tiles = 0;
    pca_status s = batch_plan(cubes, n_cubes, max_sweeps, tuning, dt, &need, total, &max_k, &chunk, &tiles);
    if (s != PCA_OK) return s;
    if (ws_bytes < need) return PCA_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    if (pca::launch_batch_setup(cubes_dev, n_cubes, mode, max_sweeps, chunk, tiles, w, st) != hipSuccess)
        return PCA_ERR_HIP;
    if (pca::launch_cov_batched(dt, mode, w, total, n_cubes, st) != hipSuccess) return PCA_ERR_HIP;
    if (pca::launch_jacobi_batched(w, total, n_cubes, tol, max_sweeps, fp64_angles, st) != hipSuccess)
        return PCA_ERR_HIP;
    return hip_status(pca::launch_project_batched(dt, w, total, n_cubes, max_k, st));
}

pca_status pca_set_wait_shift(int32_t shift)
{
    if (shift < 0 || shift > 40) return PCA_ERR_ARG;
    if (pca::set_wait_shift_one_cu(shift) != hipSuccess) return PCA_ERR_HIP;
    return hip_status(pca::set_wait_shift_block(shift));
}

}  // extern "C"

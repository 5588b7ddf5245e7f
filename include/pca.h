/*
 * pca.h - C ABI of the MI355X (gfx950) Jacobi-PCA library, libpca.so.
 *
 * The library computes the principal component analysis of a hyperspectral
 * cube as laid out in Algorithm 1 of Martel et al., "Implementation of the
 * Principal Component Analysis onto High-Performance Computer Facilities for
 * Hyperspectral Dimensionality Reduction" (Section 2): band-mean removal,
 * the bands x bands covariance over all pixels, a cyclic Jacobi
 * eigendecomposition of that covariance, and the projection of every pixel
 * onto the leading eigenvectors.
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer owned by the caller (the
 *     library never allocates, frees or copies to the host). Matrices are
 *     row-major. The cube is band-interleaved-by-pixel: pixel p, band b is
 *     element p * ld_y + b.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every call only enqueues kernels on it and returns without waiting.
 *   - Argument checks are synchronous and touch no device memory; a failed
 *     check returns PCA_ERR_ARG / PCA_ERR_UNSUPPORTED / PCA_ERR_WORKSPACE and
 *     enqueues nothing. A launch failure returns PCA_ERR_HIP.
 *   - Numerical outcomes (non-convergence, non-finite data) are reported in
 *     the device-resident pca_info written by pca_jacobi_eigh.
 *   - Results are deterministic: every reduction runs in a fixed order, no
 *     floating-point atomics are used.
 *   - Calls on one stream run in order; calls sharing a workspace must not
 *     overlap on different streams.
 *   - Limits: 2 <= n_bands <= 256, n_pixels >= 2, pointers 16-byte aligned,
 *     workspace 256-byte aligned.
 */
#ifndef PCA_H
#define PCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCA_OK = 0,
    PCA_ERR_ARG = 1,          /* NULL pointer, size out of range, misalignment */
    PCA_ERR_UNSUPPORTED = 2,  /* valid request that the library does not handle */
    PCA_ERR_WORKSPACE = 3,    /* workspace smaller than pca_workspace_size */
    PCA_ERR_HIP = 4           /* a HIP launch or attribute call failed */
} pca_status;

/* Element type and layout of the cube. Band-interleaved by pixel (BIP):
 * Y[p * ld_y + b], ld_y >= n_bands, a pixel's bands contiguous, as push-broom
 * sensors deliver it. Band-sequential (BSQ): Y[b * ld_y + p], ld_y >=
 * n_pixels, a band's pixels contiguous: the layout of the paper's GPU
 * design (Section 4). Every call takes BSQ cubes (pca_backward in float32). */
typedef enum {
    PCA_IN_F32 = 0,           /* float32, BIP */
    PCA_IN_U16 = 1,           /* uint16 (e.g. raw radiance counts), read as exact integers, BIP */
    PCA_IN_F32_BSQ = 2,       /* float32, BSQ */
    PCA_IN_U16_BSQ = 3        /* uint16, BSQ */
} pca_in_dtype;

/* Arithmetic of the covariance products (the sums are always combined in
 * float64 across pixel chunks). */
typedef enum {
    PCA_COV_F32 = 0,          /* float32 products, float32 MFMA accumulation */
    PCA_COV_BF16X3 = 1,       /* split x = hi + lo into two bfloat16 terms;
                                 hi*hi + hi*lo + lo*hi with bfloat16 MFMA and
                                 float32 accumulation (lo*lo dropped) */
    PCA_COV_BF16X4 = 2,       /* as BF16X3 plus lo*lo: the exact product of
                                 the 16-significant-bit split */
    PCA_COV_FP16X3 = 3        /* split x sc = hi + lo into two float16 terms
                                 (sc: a per-band power of two that the
                                 covariance call derives from a pixel sample:
                                 1/2 for uint16 cubes, the largest sampled
                                 |x| brought to at most 16 for float32 cubes);
                                 hi*hi + hi*lo + lo*hi with float16 MFMA and
                                 float32 accumulation, results scaled back by
                                 1/(sc_i sc_j). About 22 significant bits per
                                 value; a float32 value more than 2^12 times
                                 the largest sampled deviation of its band
                                 overflows float16 and makes the covariance
                                 non-finite */
} pca_cov_mode;

/* Operation selector for pca_workspace_size. */
typedef enum {
    PCA_OP_CENTER = 0,
    PCA_OP_COVARIANCE = 1,
    PCA_OP_JACOBI = 2,
    PCA_OP_PROJECT = 3,
    PCA_OP_BACKWARD = 4
} pca_op;

/* Flags of pca_jacobi_eigh. */
typedef enum {
    /* Rotation angles and the updated diagonal in float64 (else float32). */
    PCA_JACOBI_FP64_ANGLES = 1,
    /* Form the eigenvectors (the product of the rotations, equation (10))
     * while the sweeps run, on other CUs of the same launch, instead of
     * after them: the same results bit for bit, without the replay's time
     * after the sweeps; it holds one more CU per ~2048/n_bands rows of the
     * eigenvector matrix for the length of the sweeps, so it pays when one
     * cube has the GPU to itself. */
    PCA_JACOBI_OVERLAP_REPLAY = 2,
    /* Run the one-workgroup form (the whole matrix on one CU) whatever the
     * band count. */
    PCA_JACOBI_ONE_CU = 4,
    /* Run the block-cyclic form on many CUs whatever the band count. */
    PCA_JACOBI_BLOCK = 8
} pca_jacobi_flag;

/* Written on the device by pca_jacobi_eigh (copy it back to read it). */
typedef struct {
    int32_t sweeps;      /* sweeps carried out */
    int32_t converged;   /* 1 when a stop rule was met before max_sweeps */
    int32_t nonfinite;   /* 1 when C held a NaN or an infinity (outputs are then NaN) */
    int32_t floor_hit;   /* 1 when the last sweep applied no rotation (float32 floor) */
    double off_rel;      /* final sqrt(sum_{i!=j} a_ij^2) / ||C||_F */
    int64_t rotations;   /* rotations applied */
    int32_t steps;       /* parallel rotation steps carried out */
    int32_t n_bands;
} pca_info;

/* One cube of a batch (pca_batched). Every pointer is a device pointer. */
typedef struct {
    const void *Y;       /* the cube, element type and layout given to pca_batched:
                            [n_pixels][ld_y] (BIP) or [n_bands][ld_y] (BSQ) */
    int64_t n_pixels;    /* >= 2 */
    int64_t ld_y;        /* >= n_bands (BIP), >= n_pixels (BSQ) */
    int32_t n_bands;     /* 2 .. 256 */
    int32_t k;           /* kept components, 1 .. n_bands */
    float *mean;         /* [n_bands] out */
    float *eigvals;      /* [n_bands] out, descending */
    float *V;            /* [n_bands][n_bands] out, column i = eigenvector i */
    float *Q;            /* [n_pixels][k] out */
    pca_info *info;      /* out, may be NULL */
} pca_cube;

/* Tile shapes of the batched launches (0 = default). */
typedef struct {
    int32_t cov_chunk;   /* pixels per covariance work item (multiple of 32, <= 16384) */
    int32_t proj_tiles;  /* 64-pixel tiles per projection work item (>= 1) */
} pca_batch_tuning;

/* Human-readable name of a status code (static storage). */
const char *pca_status_string(pca_status s);

/*
 * Bytes of workspace that `op` needs for the given sizes (mode: a
 * pca_cov_mode for PCA_OP_COVARIANCE; max_sweeps: for PCA_OP_JACOBI; k: for
 * PCA_OP_BACKWARD).
 */
pca_status pca_workspace_size(int op, int64_t n_pixels, int32_t n_bands, int32_t k,
                              int32_t mode, int32_t max_sweeps, size_t *bytes);

/*
 * Band-average removal (Algorithm 1, line 2; the per-band average of the
 * GPU design's Code 4.2.1 and its subtraction, Code 4.2.2).
 *   Y     cube of type and layout dt ([n_pixels][ld_y] BIP, [n_bands][ld_y] BSQ).
 *   mean  [n_bands] float32 out: mu_b = (1/N) sum_p Y[p, b], summed in float64.
 *   X     float32 out in the layout of Y ([n_pixels][ld_x] BIP, [n_bands][ld_x]
 *         BSQ): Y - 1 mu^T, or NULL to write only mean.
 *   ws    workspace of pca_workspace_size(PCA_OP_CENTER, ...) bytes.
 */
pca_status pca_center(const void *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y,
                      float *mean, float *X, int64_t ld_x, void *ws, size_t ws_bytes,
                      void *stream);

/*
 * Covariance C = X^T X / (N - 1) of the centred cube (Algorithm 1, line 3,
 * normalised by PIXELS - 1 as in Code 4.3), with the centring fused: the cube
 * is read once. Pixels are processed in chunks; each chunk accumulates
 * sum (y - s)(y - s)^T and sum (y - s) about its first pixel s on chip, and
 * the chunk results are combined in float64 in chunk order into the centred
 * second moment (exact algebra, no cancellation against a global mean).
 *   Y                  cube of type and layout dt ([n_pixels][ld_y] BIP,
 *                      [n_bands][ld_y] BSQ).
 *   input_is_centered  1: Y already is X (C = Y^T Y / (N-1), mean not written);
 *                      0: centre on the fly.
 *   mean               [n_bands] float32 out (may be NULL).
 *   mode               a pca_cov_mode.
 *   C                  [n_bands][n_bands] float32 out, exactly symmetric.
 *   ws                 workspace of pca_workspace_size(PCA_OP_COVARIANCE, ...).
 */
pca_status pca_covariance(const void *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y,
                          int32_t input_is_centered, float *mean, int mode, float *C,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * All eigenpairs of the symmetric C by the cyclic Jacobi method (Section 2,
 * equations (2)-(10)), in one of two forms, both applying disjoint rotations
 * together (the parallel-rotation property stated at the end of Section 2):
 *   - one workgroup holds the matrix in LDS and applies n_bands/2 rotations
 *     per parallel step in round-robin order, n_bands - 1 steps per sweep
 *     (PCA_JACOBI_ONE_CU; the default below 96 bands);
 *   - block-cyclic: the indices are grouped in blocks of 16, a round-robin
 *     over the blocks pairs them, and one workgroup per pair of block pairs
 *     rotates its pair's index pairs and applies the product of those
 *     rotations to its tiles of A and of the eigenvector matrix (equations
 *     (8) and (10) with the rotations of a step grouped); the workgroups
 *     exchange tiles through memory once per block step (PCA_JACOBI_BLOCK;
 *     the default from 96 bands). Every index pair is still rotated once per
 *     sweep; only the order differs. It spreads one call over up to 32 CUs
 *     and needs them all resident at once, so it pays when the call has the
 *     GPU to itself; a workgroup that waits about half a second for the
 *     others gives up and the call reports non-finite output.
 * Rotation angles use equations (2)-(5) with (7) in the cancellation-free
 * form; the flag PCA_JACOBI_FP64_ANGLES evaluates them (and the diagonal) in
 * float64. A rotation is skipped when |a_pq| <= 2^-24 sqrt(|a_pp a_qq|) or
 * |a_pq| <= 2^-24 ||C||_F / n_bands. Stops before a sweep when
 * off(A)/||C||_F <= tol, after a sweep that applied no rotation, or after
 * max_sweeps sweeps.
 * Eigenvalues are sorted in descending order (stable), eigenvector columns
 * permuted to match (Code 4.4.3), and each eigenvector's sign fixed so that
 * its largest-magnitude entry is positive (lowest index on ties).
 *   C        [n_bands][n_bands] float32, symmetric (the upper triangle is read).
 *   eigvals  [n_bands] float32 out, descending.
 *   V        [n_bands][n_bands] float32 out; column j is eigenvector j.
 *   info     device pca_info out (may be NULL).
 *   flags    OR of pca_jacobi_flag values (other bits, or both form flags:
 *            PCA_ERR_ARG). PCA_JACOBI_OVERLAP_REPLAY applies to the
 *            one-workgroup form only.
 *   ws       workspace of pca_workspace_size(PCA_OP_JACOBI, ..., max_sweeps).
 *            Its contents before the call do not matter (every call clears
 *            what it reads before reading it); calls that share a workspace
 *            must not overlap in time.
 */
pca_status pca_jacobi_eigh(const float *C, int32_t n_bands, double tol, int32_t max_sweeps,
                           int32_t flags, float *eigvals, float *V, pca_info *info,
                           void *ws, size_t ws_bytes, void *stream);

/* Bytes of device memory that pca_jacobi_eigh_noalloc holds on each GPU it
 * runs on (until the process ends). */
#define PCA_NOALLOC_SCRATCH_BYTES (12u << 20)

/*
 * pca_jacobi_eigh for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same calls and results, with the workspace taken from a fixed
 * PCA_NOALLOC_SCRATCH_BYTES array in the library's device memory instead of
 * an argument. It allocates and frees nothing. Requests whose workspace
 * (pca_workspace_size(PCA_OP_JACOBI, ...)) exceeds that size return
 * PCA_ERR_WORKSPACE (at 256 bands, max_sweeps up to about 40 fit). The array
 * is shared by every call on one GPU: calls that overlap in time on one GPU
 * (other streams, other host threads) race and must not be issued; calls on
 * one stream run in order and are safe. Arguments and results as for
 * pca_jacobi_eigh; PCA_ERR_HIP if the array's address cannot be obtained.
 */
pca_status pca_jacobi_eigh_noalloc(const float *C, int32_t n_bands, double tol, int32_t max_sweeps, int32_t flags,
                                   float *eigvals, float *V, pca_info *info, void *stream);

/*
 * Projection onto the first k eigenvectors (Algorithm 1, lines 5-6):
 *   Q[p, i] = sum_b (Y[p, b] - mean[b]) V[b, i],  i < k.
 *   Y     cube of type and layout dt ([n_pixels][ld_y] BIP, [n_bands][ld_y] BSQ).
 *   mean  [n_bands] float32, or NULL when Y is already centred.
 *   V     [n_bands][n_bands] float32, column i = eigenvector i.
 *   Q     [n_pixels][k] float32 out. 1 <= k <= n_bands.
 */
pca_status pca_project(const void *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y,
                       const float *mean, const float *V, int32_t k, float *Q, void *stream);

/*
 * Reverse-mode derivative of the whole pipeline (band-mean removal,
 * covariance, eigenpairs, projection; Algorithm 1, lines 2-6) for a scalar
 * loss L. Given the loss's gradients at the forward outputs, writes dL/dY:
 *   Xbar  = dQ V_k^T + 2 X Cbar / (N - 1),      X = Y - 1 mean^T,
 *   Cbar  = sym(V (diag(dEig) + F o (V^T Vbar)) V^T),
 *           Vbar = [X^T dQ + dVk | 0],  F_ij = 1/(lambda_j - lambda_i), i != j
 *           (0 on the diagonal and where two eigenvalues are equal),
 *   dY    = Xbar - (1/N) 1 (1^T Xbar).
 * The eigenpair term is the first-order perturbation of a symmetric
 * eigendecomposition; it assumes the eigenvalues that meet a nonzero F entry
 * (those among the first k and their partners) are distinct. The sign fix and
 * the sort of the forward pass are piecewise constant and add no term.
 *   Y        the forward input: float32, dt PCA_IN_F32 ([n_pixels][ld_y],
 *            BIP) or PCA_IN_F32_BSQ ([n_bands][ld_y], BSQ, ld_y >= n_pixels).
 *   mean     [n_bands] float32 band means written by the forward pass.
 *   eigvals  [n_bands] float32, V [n_bands][n_bands] float32 (column i =
 *            eigenvector i): the forward's eigenpairs.
 *   k        kept components, 1 <= k <= n_bands.
 *   dQ       [n_pixels][k] dL/dQ, or NULL (zero).
 *   dEig     [n_bands] dL/d eigvals, or NULL (zero).
 *   dVk      [n_bands][k] dL/dV[:, :k], or NULL (zero).
 *   dY       float32 out in the layout of Y: [n_pixels][ld_dy], ld_dy >=
 *            n_bands (BIP), or [n_bands][ld_dy], ld_dy >= n_pixels (BSQ).
 *   ws       workspace of pca_workspace_size(PCA_OP_BACKWARD, n_pixels, n_bands, k, ...).
 * Float64 is used for every reduction over pixels and for the small
 * bands x bands algebra; the final pixel pass is a float32 MFMA product.
 */
pca_status pca_backward(const float *Y, int dt, int64_t n_pixels, int32_t n_bands, int64_t ld_y, const float *mean,
                        const float *eigvals, const float *V, int32_t k, const float *dQ, const float *dEig,
                        const float *dVk, float *dY, int64_t ld_dy, void *ws, size_t ws_bytes, void *stream);

/*
 * Workspace bytes of pca_batched for these cubes (host array), covariance
 * mode, max_sweeps and tuning (NULL = defaults).
 */
pca_status pca_batched_workspace_size(const pca_cube *cubes, int32_t n_cubes, int mode, int32_t max_sweeps,
                                      const pca_batch_tuning *tuning, size_t *bytes);

/*
 * The whole pipeline (Algorithm 1) for many cubes of different pixel and
 * band counts, each as pca_covariance + pca_jacobi_eigh + pca_project would
 * compute it alone, in nine launches for the whole batch: a set-up kernel
 * that builds the task table in the workspace, the shift pass (a pixel
 * sample per cube), one persistent covariance
 * launch whose workgroups take (cube, pixel chunk) items from a queue,
 * largest band counts first, the float64 chunk combination, a launch that
 * zeroes the rotation logs, one Jacobi launch with a workgroup per cube (each
 * cube's rotations on its own CU) followed by workgroups that form the
 * eigenvectors from those logs while the sweeps run, the sort and sign fix,
 * and one projection launch.
 *   cubes      host array of n_cubes descriptors (validation and sizing).
 *   cubes_dev  the same array in device memory (read by the set-up kernel;
 *              keeping it resident makes the sequence capturable in a graph).
 *   n_cubes    1 .. 4096.
 *   dt         pca_in_dtype of every cube (one element type and layout per
 *              call); mode a pca_cov_mode.
 *   tol, max_sweeps, fp64_angles  as for pca_jacobi_eigh.
 *   tuning     tile shapes (NULL = defaults), e.g. from an autotuner.
 *   ws         workspace of pca_batched_workspace_size(...) bytes.
 */
pca_status pca_batched(const pca_cube *cubes, const pca_cube *cubes_dev, int32_t n_cubes, int dt, int mode,
                       double tol, int32_t max_sweeps, int32_t fp64_angles, const pca_batch_tuning *tuning,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * For tests of the failure handling only (callers that want a wait to run
 * out without a fault): divides the time or poll bound of every wait inside
 * the Jacobi kernels (the block-cyclic form's step barrier and its U
 * followers' waits, the eigenvector followers of the overlapped replay and
 * of the batched form) by 2^shift, 0 <= shift <= 40, on the current device;
 * 0 restores the defaults. A wait that runs out ends its kernel normally and
 * the call reports a non-finite result (or NaN eigenvector rows from a
 * follower). Synchronous; not to be called while library work is in flight.
 */
pca_status pca_set_wait_shift(int32_t shift);

#ifdef __cplusplus
}
#endif

#endif /* PCA_H */

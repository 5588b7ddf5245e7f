// Block-cyclic Jacobi eigendecomposition on many CUs (Section 2: equations
// (2)-(10), the stop rule, and the property that rotations of disjoint index
// pairs can be applied at the same time).
//
// Ordering. The n_bands indices (padded with zero "phantom" indices to nb
// blocks of 16, nb even) are split into nb blocks. An outer step pairs the
// blocks by a round-robin tournament over the nb blocks (nb/2 block pairs
// per step, nb - 1 steps per sweep); for each block pair (I, J) the 32 x 32
// sub-matrix A[I u J, I u J] is treated by a sequence of inner steps of 16
// disjoint scalar rotations each:
//   - cross steps c = 0..15: index I_k with J_{(k + c) mod 16}, so that over
//     one outer step every pair (i in I, j in J) is rotated once;
//   - in the first outer step of every sweep, 15 intra steps before the
//     cross steps: a round-robin within I and within J.
// Over one sweep every index pair is rotated exactly once, as in the
// row-by-row cyclic order of Section 2 (only the order differs; the paper
// leaves the order open and its two designs use two other orders).
//
// Two-sided block update. The inner rotations of a block pair multiply to a
// 32 x 32 orthogonal U_p; the outer step applies J = diag(U_p) (one U per
// block pair, after the permutation to labels) as A <- J^T A J and V <- V J
// (equations (8) and (10), with the rotations of a step grouped). The matrix
// is kept in global memory in float64, as
//   H_t = J_t^T A_t (the left product of step t, written in 32 x 32 tiles),
//   A_{t+1}[rows, pair q] = H_t[rows, pair q] U_{t,q} (the right product,
//   formed by whoever needs it at step t + 1).
// Workgroup (x, g) of the P x Q grid owns, at step t, the rows of block pair
// x of step t and the columns of the block pairs j = g, g + Q, ... of step
// t - 1:
//   1. D = A_t[pair x, pair x] from two tiles of H_{t-1} and two U's;
//   2. the inner rotations on D (a float32 copy in LDS, one barrier per inner
//      step) give U_{t,x}, accumulated in float64; every workgroup of row x
//      forms the same U_{t,x};
//   3. for each of its column pairs j: R = A_t[pair x, pair j] =
//      H_{t-1}[..] U_{t-1,j}, H_t[pair x, pair j] = U_{t,x}^T R (float64
//      MFMA products of 32 x 32 tiles) and V_t[pair x rows, pair j cols] =
//      V_{t-1}[..] U_{t-1,j} (float32 MFMA);
//   4. R also gives this tile's part of off(A_t)^2, ||A_t||_F^2 and the
//      diagonal of A_t;
//   5. a grid barrier (per-workgroup step flags).
// The stop rule (off(A)/||C||_F <= tol, a sweep without any rotation, or
// max_sweeps) is evaluated at the start of every sweep from the partial sums
// of all workgroups, added in workgroup order, so every workgroup reaches the
// same decision. At the stop, A_t's diagonal is the eigenvalues and V_t the
// eigenvectors (unsorted; sort_sign_kernel follows).
//
// Inner rotations. The thread that produces the next pivot computes its
// rotation, and the diagonal after every step is carried in the rotation
// records, so one barrier per inner step suffices. They run in float32 (the
// tangent in float64 with PCA_JACOBI_FP64_ANGLES); U accumulates them in
// float64 with (cos, sin) normalised in float64. The inner sub-matrix only
// serves to find U: A itself is carried by the float64 tile products with U
// orthogonal to float64 rounding, so the precision of the inner steps sets
// how fast the iteration converges, not the accuracy of the result (a
// rotation that leaves a small residue at its pivot is itself orthogonal;
// the residue is rotated again later).
//
// Placement and synchronisation. Launch 8 G workgroups of which every 8th
// (one residue class, rotated from call to call) takes part, so that, with
// the workgroups of a launch dealt to the chip's 8 XCDs in turn, all G
// participants share one XCD and its L2: step data then goes through that L2
// (plain stores and a wait for their completion; device-scope loads, which
// pass the CU caches) instead of through device-wide release/acquire fences,
// which write back and invalidate whole L2s. The participants first exchange
// their XCD ids over device-scope memory; if they are not all on one XCD the
// call uses device-scope release/acquire fences for every step instead.
// Every wait is bounded in time: a workgroup that waits about half a second
// for the others gives up, and the call reports nonfinite output (NaN), so
// the launch always ends. Step flags are cleared by bj_clear_kernel before
// every launch, so a call does not depend on what the workspace held.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace pca {

namespace {

typedef __attribute__((ext_vector_type(4))) double f64x4;

constexpr int kB = kBjBlock;   // indices per block
constexpr int kThreads = 512;  // threads per workgroup (8 waves)
constexpr int kLd = 36;        // LDS pitch of a float32 32 x 32 tile
constexpr int kLdd = 34;       // LDS pitch of a float64 32 x 32 tile
constexpr int kTile = 32 * kLd;
constexpr int kTiled = 32 * kLdd;
constexpr int kNS = 31;        // inner steps of the first outer step of a sweep
constexpr int kC0 = 15;        // index of the first cross step
constexpr int kUpper = 120;    // 2x2 blocks (k < l) of 16 pairs
constexpr int kCg = kBjMaxColPairs;   // column pairs per workgroup, at most
constexpr long long kWaitTicks = 50000000;   // 0.5 s of the 100 MHz real-time counter
constexpr unsigned kRsrcWord3 = 0x00020000u;  // raw buffer resource, gfx9 family

struct BjPart {
    double off;          // sum of squares of this workgroup's off-diagonal entries of A_t
    double tot;          // sum of squares of all of its entries of A_t
    long long rot;       // rotations applied before step t (row's g = 0 workgroup only)
    long long pad;
};
static_assert(sizeof(BjPart) == 32, "partial-sum record size is part of the workspace layout");

struct Smem {
    double T1[kTiled], T2[kTiled], U1[kTiled], U2[kTiled];
    double Tj[kCg][kTiled], Uj[kCg][kTiled], R[kCg][kTiled];
    double Ui[kTiled];
    float Ujf[kCg][kTile], Vb[kCg][kTile];
    float D[kTile];
    unsigned char sp[kC0 + 1][16], sq[kC0 + 1][16], pid[kC0 + 1][32];   // intra steps and cross step 0
    unsigned char prodA[kC0][kUpper], prodB[kC0][kUpper];                // productions of the intra steps
    float2 rcf[2][16];      // (cos, sin) of each pair's rotation
    float2 rdg[2][16];      // the pair's diagonal (a_pp, a_qq) after the step
    float rpv[2][16];       // pivot entry after the step
    int rap[2][16];         // 1 when the rotation was applied
    double red[2][8];
    int st_bad, st_cnt, st_fail;
};

// Rotation of the pivot block [[app, apq], [apq, aqq]] of the float32
// sub-matrix (equations (2)-(5) with (7), the cancellation-free form of the
// tangent), written into record slot (par, k): cos, sin, the diagonal after
// the step a_pp - t a_pq, a_qq + t a_pq, the pivot after the step (0). fp64
// evaluates the tangent in float64. Skipped (cos 1, sin 0) at the float32
// rounding floor of the block.
__device__ inline void make_rec(Smem &L, int par, int k, float app, float aqq, float apq, float floor_abs, int fp64)
{
    const float ad = fabsf(apq);
    float c = 1.f, s = 0.f, dp = app, dq = aqq, pv = apq;
    int applied = 0;
    if (ad > floor_abs && ad * ad > 3.5527137e-15f * fabsf(app * aqq)) {   // |a_pq| > 2^-24 sqrt(|a_pp a_qq|)
        float tf;
        if (fp64) {
            const double d = (double)aqq - (double)app, a = (double)apq;
            const double r = sqrt(fma(d, d, 4.0 * a * a));
            tf = (float)((d >= 0.0 ? 2.0 * a : -2.0 * a) / (fabs(d) + r));
        } else {
            const float df = aqq - app;
            const float rf = __builtin_amdgcn_sqrtf(fmaf(df, df, 4.f * apq * apq));
            tf = (df >= 0.f ? 2.f * apq : -2.f * apq) * __builtin_amdgcn_rcpf(fabsf(df) + rf);
        }
        c = __builtin_amdgcn_rsqf(fmaf(tf, tf, 1.f));
        s = tf * c;
        dp = fmaf(-tf, apq, app);
        dq = fmaf(tf, apq, aqq);
        pv = 0.f;
        applied = 1;
    }
    L.rcf[par][k] = make_float2(c, s);
    L.rdg[par][k] = make_float2(dp, dq);
    L.rpv[par][k] = pv;
    L.rap[par][k] = applied;
}

// (cos, sin) of a record, normalised in float64 (one Newton step of
// 1/sqrt(c^2 + s^2) from 1), so that the rotations that make up U are
// orthogonal to float64 rounding.
__device__ inline double2 rot64(float2 cs)
{
    const double c = (double)cs.x, s = (double)cs.y;
    const double g = fma(-0.5, fma(c, c, s * s), 1.5);
    return make_double2(c * g, s * g);
}

// Position i of the round-robin (circle) over n players at round u: player 0
// stays, players 1..n-1 turn by one per round. Pair k of the round is
// (pos(k), pos(n-1-k)).
__device__ inline int rr_pos(int n, int u, int i) { return i == 0 ? 0 : 1 + (i - 1 + u) % (n - 1); }
// The inverse: which pair and which side (0 first, 1 second) player a is on.
__device__ inline void rr_where(int n, int u, int a, int &k, int &side)
{
    const int i = a == 0 ? 0 : 1 + ((a - 1 - u) % (n - 1) + (n - 1)) % (n - 1);
    if (i < n / 2) { k = i; side = 0; }
    else { k = n - 1 - i; side = 1; }
}

__device__ inline int sym(int i, int j) { return i < j ? i * kLd + j : j * kLd + i; }

// 16 x 16 tile of op(A) B with K = 32 from LDS: A element (i, k) at
// A[i * lda + k] (or A[k * lda + i] when transposed), B element (k, j) at
// B[k * ldb + j]. Lane l holds rows 4 (l / 16) + r, column l % 16 of the
// result (v_mfma_*_16x16x4: operand lanes l = row/column l % 16, k l / 16).
// The operands are read from LDS first, then multiplied, so that the reads
// overlap instead of each product waiting for its own.
__device__ inline f32x4 tile16(const float *A, int lda, bool trA, const float *B, int ldb)
{
    const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
    float a[8], b[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int k = 4 * s + kk;
        a[s] = trA ? A[k * lda + i] : A[i * lda + k];
        b[s] = B[k * ldb + i];
    }
    // Two accumulation chains of four products each, added at the end.
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 8; s += 2) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 1], b[s + 1], acc1, 0, 0, 0);
    }
    return acc0 + acc1;
}
__device__ inline f64x4 tile16d(const double *A, int lda, bool trA, const double *B, int ldb)
{
    const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
    double a[8], b[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int k = 4 * s + kk;
        a[s] = trA ? A[k * lda + i] : A[i * lda + k];
        b[s] = B[k * ldb + i];
    }
    f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; s += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s + 1], b[s + 1], acc1, 0, 0, 0);
    }
    return acc0 + acc1;
}

// Global label of local row/column r (0..31) of the block pair (b0, b1).
__device__ inline int lab(int b0, int b1, int r) { return r < kB ? b0 * kB + r : b1 * kB + (r - kB); }

typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ inline Rsrc rsrc(const void *p, size_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, (int)kRsrcWord3);
}
// 16-byte load of step data: device-scope (sc1: past the CU's own cache, from
// the XCD's L2 that the writers' stores reached) in the one-XCD mode, a plain
// load after a device-scope acquire otherwise.
template <bool kLocal>
__device__ inline uint4 ld16(Rsrc r, int off)
{
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kLocal ? 16 : 0));
}

// Loads of one step's operand tiles are issued all at once into registers
// (one round trip), then written to LDS.
// 32 x 32 float64 tile of a label-space matrix (pitch ld elements): one
// 16-byte piece per thread.
template <bool kLocal>
__device__ inline uint4 issue_tiled(Rsrc src, int ld, int r0, int r1, int c0, int c1)
{
    const int e = threadIdx.x, r = e >> 4, c = (e & 15) * 2;
    return ld16<kLocal>(src, 8 * (lab(r0, r1, r) * ld + lab(c0, c1, c)));
}
__device__ inline void commit_tiled(double *dst, uint4 v)
{
    const int e = threadIdx.x, r = e >> 4, c = (e & 15) * 2;
    const double2 d = __builtin_bit_cast(double2, v);
    dst[r * kLdd + c] = d.x;
    dst[r * kLdd + c + 1] = d.y;
}
// U matrix number q (32 x 32 float64, contiguous).
template <bool kLocal>
__device__ inline uint4 issue_u(Rsrc src, int q)
{
    const int e = threadIdx.x, r = e >> 4, c = (e & 15) * 2;
    return ld16<kLocal>(src, 8 * (q * 1024 + r * 32 + c));
}
__device__ inline void commit_u(double *dst, float *dstf, uint4 v)
{
    const int e = threadIdx.x, r = e >> 4, c = (e & 15) * 2;
    const double2 d = __builtin_bit_cast(double2, v);
    dst[r * kLdd + c] = d.x;
    dst[r * kLdd + c + 1] = d.y;
    if (dstf) {
        dstf[r * kLd + c] = (float)d.x;
        dstf[r * kLd + c + 1] = (float)d.y;
    }
}
// 32 x 32 float32 tile of a label-space matrix: one 16-byte piece for each
// of the first 256 threads.
template <bool kLocal>
__device__ inline uint4 issue_tile(Rsrc src, int ld, int r0, int r1, int c0, int c1)
{
    const int e = threadIdx.x & 255, r = e >> 3, c = (e & 7) * 4;
    return ld16<kLocal>(src, 4 * (lab(r0, r1, r) * ld + lab(c0, c1, c)));
}
__device__ inline void commit_tile(float *dst, uint4 v)
{
    if (threadIdx.x >= 256) return;
    const int r = threadIdx.x >> 3, c = (threadIdx.x & 7) * 4;
    *reinterpret_cast<float4 *>(&dst[r * kLd + c]) = __builtin_bit_cast(float4, v);
}

__device__ inline long long now_ticks() { return (long long)__builtin_amdgcn_s_memrealtime(); }

__device__ inline unsigned xcc_id()
{
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x;
}

// A step flag read with a device-scope load (past the CU's own cache); the
// load completes inside the asm block.
__device__ inline unsigned poll_local(const unsigned *p)
{
    unsigned v;
    asm volatile("global_load_dword %0, %1, off sc1\n\ts_waitcnt vmcnt(0)" : "=v"(v) : "v"(p) : "memory");
    return v;
}

// Grid barrier: every workgroup raises its flag to `target` (with the bad
// bit), then waits until all G flags reach it. Returns after every
// workgroup's stores of this step can be read.
template <bool kLocal>
__device__ void grid_sync(Smem &L, unsigned *flags, int w, int G, unsigned target)
{
    const int tid = threadIdx.x, lane = tid & 63;
    if (kLocal) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores are in the L2
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (tid == 0) {
        const unsigned v = (target << 1) | (unsigned)(L.st_bad != 0);
        if (kLocal) *reinterpret_cast<volatile unsigned *>(&flags[w]) = v;
        else __hip_atomic_store(&flags[w], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid < 64) {
        const long long t0 = now_ticks();
        int anybad = 0, fail = 0;
        while (true) {
            unsigned v = target << 1;
            if (lane < G)
                v = kLocal ? poll_local(&flags[lane])
                           : __hip_atomic_load(&flags[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__all((v >> 1) >= target)) { anybad = __any((v & 1u) != 0u); break; }
            if (now_ticks() - t0 > kWaitTicks) { fail = 1; break; }
        }
        if (lane == 0) {
            if (anybad) L.st_bad = 1;
            if (fail) L.st_fail = 1;
        }
    }
    __syncthreads();
    if (!kLocal) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__global__ __launch_bounds__(64) void bj_clear_kernel(unsigned int *flags, int n)
{
    for (int i = threadIdx.x; i < n; i += 64) flags[i] = 0u;
}

#ifdef BJ_PROFILE
__device__ long long bj_prof[16];
#define PROF(i)                                                                   \
    do {                                                                          \
        const long long tn_ = now_ticks();                                        \
        prof_[i] += tn_ - tprev_;                                                 \
        tprev_ = tn_;                                                             \
    } while (0)
#else
#define PROF(i) do { } while (0)
#endif

struct BjArgs {
    const float *C;
    int m, nb, Q, max_sweeps, fp64;
    double tol;
    double *H;          // [2][Mp][Mp]
    double *U;          // [2][P][32][32]
    float *V;           // [Mp][Mp]
    BjPart *part;       // [2][G]
    unsigned *flags;    // [G] step flags, then [G] XCD ids
    double *lam_u;
    float *VuT;
    int nvu;
    pca_info *info;
};

// The iteration of one participating workgroup w (see the file comment).
template <bool kLocal>
__device__ void bj_run(Smem &L, const BjArgs &A, int w, unsigned target0)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = A.nb, m = A.m, Q = A.Q, P = nb / 2, G = P * Q, S = nb - 1;
    const int Mp = nb * kB;
    const int x = w / Q, g = w - (w / Q) * Q;
    const int ncg = (P - g + Q - 1) / Q;   // column pairs g, g + Q, ... below P
    const Rsrc rH = rsrc(A.H, (size_t)2 * Mp * Mp * sizeof(double));
    const Rsrc rU = rsrc(A.U, (size_t)2 * P * 1024 * sizeof(double));
    const Rsrc rV = rsrc(A.V, (size_t)Mp * Mp * sizeof(float));
    const Rsrc rP = rsrc(A.part, (size_t)2 * G * sizeof(BjPart));
    const int fp64 = A.fp64;
#ifdef BJ_PROFILE
    long long tprev_ = now_ticks();
    long long prof_[16] = {0};
#endif

    // Roles in the inner steps: threads 0..119 rotate the 2x2 blocks (bk, bl),
    // bk < bl, and compute the next pivots' rotations; threads 128..143 write
    // the pivots back; threads 256..511 rotate the columns of U.
    int bk = 0, bl = 1;
    if (tid < kUpper) {
        int e = tid, k = 0;
        while (e >= kB - 1 - k) { e -= kB - 1 - k; ++k; }
        bk = k;
        bl = k + 1 + e;
    }
    const int ptid = tid < kUpper ? tid : 0;
    const bool uthr = tid >= 256;
    const int uk = tid & 15, ur = (tid >> 4) & 15;   // U task: pair uk, rows ur and ur + 16
    // Tile products: wave w takes output tile (ti, tj) of column pair wjj.
    const int wjj = wave >> 2, ti = (wave >> 1) & 1, tj = wave & 1;
    const int orow = 4 * (lane >> 4), ocol = lane & 15;
    f32x4 vacc = {0.f, 0.f, 0.f, 0.f};
    long long mycnt = 0, cnt_prev = 0;
    double fro2 = 0.0, off2 = 0.0, lim2 = 0.0;
    float floor_abs = 0.f;
    int sweeps = 0, converged = 0, floor_hit = 0, bad = 0, failed = 0;
    int t = 0;
    int I = 0, J = 0;
    int Kc[kCg] = {0}, Lc[kCg] = {0};

    for (;; ++t) {
        const int u = t % S;
        const int up = t == 0 ? S - 1 : (t - 1) % S;
        I = rr_pos(nb, u, x);
        J = rr_pos(nb, u, nb - 1 - x);
#pragma unroll
        for (int jj = 0; jj < kCg; ++jj) {
            const int j = g + (jj < ncg ? jj : 0) * Q;
            Kc[jj] = rr_pos(nb, up, j);
            Lc[jj] = rr_pos(nb, up, nb - 1 - j);
        }
        int q1, o1, q2, o2;
        rr_where(nb, up, I, q1, o1);
        rr_where(nb, up, J, q2, o2);

        // ---- operands of step t: D = A_t[pair x, pair x] -------------------------
        if (t == 0) {
            // A_0 = C (padded with zeros), U_{-1} = I, V_0 = I.
            int nonfin = 0;
            for (int e = tid; e < 1024; e += kThreads) {
                const int r = e >> 5, c = e & 31;
                const int gr = lab(I, J, r), gd = lab(I, J, c);
                const float vd = (gr < m && gd < m) ? A.C[(int64_t)gr * m + gd] : 0.f;
                if (!isfinite(vd)) nonfin = 1;
                L.D[r * kLd + c] = vd;
                for (int jj = 0; jj < ncg; ++jj) {
                    const int gc = lab(Kc[jj], Lc[jj], c);
                    const float vr = (gr < m && gc < m) ? A.C[(int64_t)gr * m + gc] : 0.f;
                    if (!isfinite(vr)) nonfin = 1;
                    L.R[jj][r * kLdd + c] = (double)vr;
                }
            }
            if (nonfin) atomicOr(&L.st_bad, 1);
            {
                const int gc = lab(Kc[wjj], Lc[wjj], 16 * tj + ocol);
#pragma unroll
                for (int r = 0; r < 4; ++r) vacc[r] = lab(I, J, 16 * ti + orow + r) == gc ? 1.f : 0.f;
            }
        } else {
            const int hb = ((t - 1) & 1) * nb;              // block-row offset of H_{t-1}
            const int uoff = ((t - 1) & 1) * P;             // U index offset of step t-1
            uint4 vTj[kCg], vUj[kCg], vVb[kCg];
            const uint4 vT1 = issue_tiled<kLocal>(rH, Mp, hb + I, hb + J, rr_pos(nb, up, q1),
                                                  rr_pos(nb, up, nb - 1 - q1));
            const uint4 vT2 = issue_tiled<kLocal>(rH, Mp, hb + I, hb + J, rr_pos(nb, up, q2),
                                                  rr_pos(nb, up, nb - 1 - q2));
            const uint4 vU1 = issue_u<kLocal>(rU, uoff + q1);
            const uint4 vU2 = issue_u<kLocal>(rU, uoff + q2);
#pragma unroll
            for (int jj = 0; jj < kCg; ++jj) {
                // (a second copy of column pair 0 when there is no second)
                vTj[jj] = issue_tiled<kLocal>(rH, Mp, hb + I, hb + J, Kc[jj], Lc[jj]);
                vUj[jj] = issue_u<kLocal>(rU, uoff + g + (jj < ncg ? jj : 0) * Q);
                vVb[jj] = issue_tile<kLocal>(rV, Mp, I, J, Kc[jj], Lc[jj]);
            }
            commit_tiled(L.T1, vT1);
            commit_tiled(L.T2, vT2);
            commit_u(L.U1, nullptr, vU1);
            commit_u(L.U2, nullptr, vU2);
#pragma unroll
            for (int jj = 0; jj < kCg; ++jj) {
                commit_tiled(L.Tj[jj], vTj[jj]);
                commit_u(L.Uj[jj], L.Ujf[jj], vUj[jj]);
                commit_tile(L.Vb[jj], vVb[jj]);
            }
            __syncthreads();
            PROF(0);
            // Columns of block I from (T1, U1), of block J from (T2, U2): waves 0..3.
            if (wave < 4) {
                const double *Ta = tj == 0 ? L.T1 : L.T2;
                const double *Ua = (tj == 0 ? L.U1 : L.U2) + 16 * (tj == 0 ? o1 : o2);
                const f64x4 dacc = tile16d(Ta + 16 * ti * kLdd, kLdd, false, Ua, kLdd);
#pragma unroll
                for (int r = 0; r < 4; ++r) L.D[(16 * ti + orow + r) * kLd + 16 * tj + ocol] = (float)dacc[r];
            }
        }

        // ---- inner rotations on D -> Ui ---------------------------------------------
        const int s0 = (u == 0) ? 0 : kC0;
        for (int e = tid; e < 1024; e += kThreads) {
            const int r = e >> 5, c = e & 31;
            L.Ui[r * kLdd + c] = r == c ? 1.0 : 0.0;
        }
        if (tid == 0) L.st_cnt = 0;
        __syncthreads();
        if (tid < 16) {
            const int p = L.sp[s0][tid], q = L.sq[s0][tid];
            make_rec(L, s0 & 1, tid, L.D[p * kLd + p], L.D[q * kLd + q], L.D[sym(p, q)], floor_abs, fp64);
        }
        __syncthreads();
        PROF(1);
        int my_applied = 0;
        for (int s = s0; s < kNS; ++s) {
            const int ps = s & 1;
            const bool intra = s < kC0;
            const int c = s - kC0;   // cross step index
            if (tid < kUpper) {
                int pk, qk, pl, ql;
                if (intra) {
                    pk = L.sp[s][bk]; qk = L.sq[s][bk]; pl = L.sp[s][bl]; ql = L.sq[s][bl];
                } else {
                    pk = bk; qk = kB + ((bk + c) & 15); pl = bl; ql = kB + ((bl + c) & 15);
                }
                // Rows p_k, q_k by pair bk's rotation, columns p_l, q_l by
                // pair bl's, in place. Every LDS read of the step first.
                const float2 rk = L.rcf[ps][bk], rl = L.rcf[ps][bl];
                const float2 dk = L.rdg[ps][bk], dl = L.rdg[ps][bl];
                const int i00 = sym(pk, pl), i01 = sym(pk, ql), i10 = sym(qk, pl), i11 = sym(qk, ql);
                const float x00 = L.D[i00], x01 = L.D[i01], x10 = L.D[i10], x11 = L.D[i11];
                unsigned pa = 0xffu, pb = 0xffu;
                if (intra) {
                    pa = L.prodA[s][ptid];
                    pb = L.prodB[s][ptid];
                } else if (c < kB - 1) {
                    // Cross steps: block (k, k+1) produces pair k (entry
                    // (p_k, q_l)), block (0, 15) pair 15 (entry (q_k, p_l)).
                    if (bl == bk + 1) pa = 1u | ((unsigned)bk << 2);
                    else if (bk == 0 && bl == kB - 1) pa = 2u | ((unsigned)(kB - 1) << 2);
                }
                const float y00 = rk.x * x00 - rk.y * x10, y10 = rk.y * x00 + rk.x * x10;
                const float y01 = rk.x * x01 - rk.y * x11, y11 = rk.y * x01 + rk.x * x11;
                const float z00 = rl.x * y00 - rl.y * y01, z01 = rl.y * y00 + rl.x * y01;
                const float z10 = rl.x * y10 - rl.y * y11, z11 = rl.y * y10 + rl.x * y11;
                // A next-step pivot among the four entries: its rotation, from
                // the entry and the two diagonal entries after this step.
                for (int h = 0; h < 2; ++h) {
                    const unsigned pr = h == 0 ? pa : pb;
                    if (pr != 0xffu) {
                        const int e = pr & 3, kn = pr >> 2;
                        const float z = e == 0 ? z00 : (e == 1 ? z01 : (e == 2 ? z10 : z11));
                        const int a = e < 2 ? pk : qk, b = (e & 1) ? ql : pl;
                        const float da = e < 2 ? dk.x : dk.y, db = (e & 1) ? dl.y : dl.x;
                        const bool lo = a < b;
                        make_rec(L, ps ^ 1, kn, lo ? da : db, lo ? db : da, z, floor_abs, fp64);
                    }
                }
                L.D[i00] = z00;
                L.D[i01] = z01;
                L.D[i10] = z10;
                L.D[i11] = z11;
            } else if (tid >= 128 && tid < 144) {
                const int k = tid - 128;
                const int p = intra ? L.sp[s][k] : k, q = intra ? L.sq[s][k] : kB + ((k + c) & 15);
                L.D[sym(p, q)] = L.rpv[ps][k];
                my_applied += L.rap[ps][k];
            } else if (uthr) {
                // Ui <- Ui P_s: columns p, q of pair uk in rows ur and ur + 16.
                const int up_ = intra ? L.sp[s][uk] : uk, uq_ = intra ? L.sq[s][uk] : kB + ((uk + c) & 15);
                const float2 ucs = L.rcf[ps][uk];
                const double ua0 = L.Ui[ur * kLdd + up_], ub0 = L.Ui[ur * kLdd + uq_];
                const double ua1 = L.Ui[(ur + 16) * kLdd + up_], ub1 = L.Ui[(ur + 16) * kLdd + uq_];
                const double2 cs = rot64(ucs);
                L.Ui[ur * kLdd + up_] = cs.x * ua0 - cs.y * ub0;
                L.Ui[ur * kLdd + uq_] = cs.y * ua0 + cs.x * ub0;
                L.Ui[(ur + 16) * kLdd + up_] = cs.x * ua1 - cs.y * ub1;
                L.Ui[(ur + 16) * kLdd + uq_] = cs.y * ua1 + cs.x * ub1;
            }
            __syncthreads();
        }
        if (my_applied) atomicAdd(&L.st_cnt, my_applied);
        PROF(2);

        // ---- R = A_t[pair x, pair j], H_t = Ui^T R, V_t, partial sums ------------------
        if (t > 0 && wjj < ncg) {
            const f64x4 racc = tile16d(L.Tj[wjj] + 16 * ti * kLdd, kLdd, false, L.Uj[wjj] + 16 * tj, kLdd);
#pragma unroll
            for (int r = 0; r < 4; ++r) L.R[wjj][(16 * ti + orow + r) * kLdd + 16 * tj + ocol] = racc[r];
            vacc = tile16(L.Vb[wjj] + 16 * ti * kLd, kLd, false, L.Ujf[wjj] + 16 * tj, kLd);
        }
        if (wjj < ncg) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                A.V[(int64_t)lab(I, J, 16 * ti + orow + r) * Mp + lab(Kc[wjj], Lc[wjj], 16 * tj + ocol)] = vacc[r];
        }
        __syncthreads();
        {
            if (wjj < ncg) {
                const f64x4 hacc = tile16d(L.Ui + 16 * ti, kLdd, true, L.R[wjj] + 16 * tj, kLdd);
                double *Hd = A.H + (int64_t)(t & 1) * Mp * Mp;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Hd[(int64_t)lab(I, J, 16 * ti + orow + r) * Mp + lab(Kc[wjj], Lc[wjj], 16 * tj + ocol)] = hacc[r];
            }
            double so = 0.0, st = 0.0;
            for (int jj = 0; jj < ncg; ++jj) {
                for (int e = tid; e < 1024; e += kThreads) {
                    const int r = e >> 5, c = e & 31;
                    const double v = L.R[jj][r * kLdd + c];
                    st += v * v;
                    if (lab(I, J, r) != lab(Kc[jj], Lc[jj], c)) so += v * v;
                }
            }
            so = wave_sum(so);
            st = wave_sum(st);
            if (lane == 0) { L.red[0][wave] = so; L.red[1][wave] = st; }
        }
        if (g == 0) {
            const int r = tid >> 4, c = (tid & 15) * 2;
            double *Ud = A.U + ((int64_t)(t & 1) * P + x) * 1024;
            *reinterpret_cast<double2 *>(&Ud[r * 32 + c]) = make_double2(L.Ui[r * kLdd + c], L.Ui[r * kLdd + c + 1]);
        }
        __syncthreads();
        if (tid == 0) {
            BjPart pp;
            pp.off = ((L.red[0][0] + L.red[0][1]) + (L.red[0][2] + L.red[0][3])) +
                     ((L.red[0][4] + L.red[0][5]) + (L.red[0][6] + L.red[0][7]));
            pp.tot = ((L.red[1][0] + L.red[1][1]) + (L.red[1][2] + L.red[1][3])) +
                     ((L.red[1][4] + L.red[1][5]) + (L.red[1][6] + L.red[1][7]));
            pp.rot = g == 0 ? mycnt : 0;
            pp.pad = 0;
            A.part[(t & 1) * G + w] = pp;
        }
        if (g == 0) mycnt += L.st_cnt;
        PROF(3);

        grid_sync<kLocal>(L, A.flags, w, G, target0 + (unsigned)t);
        PROF(4);
        bad = L.st_bad;
        failed = L.st_fail;
        if (failed || bad) break;

        // ---- stop rule at the start of a sweep -------------------------------------------
        if (u == 0) {
            double so = 0.0, st = 0.0;
            long long cnt = 0;
            for (int v = 0; v < G; ++v) {
                const uint4 a = ld16<kLocal>(rP, (int)sizeof(BjPart) * ((t & 1) * G + v));
                const uint4 b = ld16<kLocal>(rP, (int)sizeof(BjPart) * ((t & 1) * G + v) + 16);
                so += __builtin_bit_cast(double, ((unsigned long long)a.y << 32) | a.x);
                st += __builtin_bit_cast(double, ((unsigned long long)a.w << 32) | a.z);
                cnt += (long long)(((unsigned long long)b.y << 32) | b.x);
            }
            off2 = so;
            if (t == 0) {
                fro2 = st;
                lim2 = A.tol * A.tol * fro2;
                floor_abs = (float)(5.9604644775390625e-08 * sqrt(fro2) / (double)m);
            }
            sweeps = t / S;
            if (off2 <= lim2) { converged = 1; break; }
            if (t > 0 && cnt == cnt_prev) { converged = 1; floor_hit = 1; break; }
            if (sweeps >= A.max_sweeps) break;
            cnt_prev = cnt;
        }
    }
#ifdef BJ_PROFILE
    if (w == 0 && tid == 0)
        for (int i = 0; i < 16; ++i) bj_prof[i] = prof_[i];
#endif

    // ---- outputs: diagonal of A_t, V_t (transposed), info -------------------------------
    if (!(failed || bad)) {
        for (int jj = 0; jj < ncg; ++jj) {
            for (int e = tid; e < 1024; e += kThreads) {
                const int r = e >> 5, c = e & 31;
                const int gr = lab(I, J, r), gc = lab(Kc[jj], Lc[jj], c);
                if (gr == gc && gr < m) A.lam_u[gr] = L.R[jj][r * kLdd + c];
            }
        }
        if (wjj < ncg) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = lab(I, J, 16 * ti + orow + r), gc = lab(Kc[wjj], Lc[wjj], 16 * tj + ocol);
                if (gr < m && gc < m) A.VuT[(int64_t)gc * A.nvu + gr] = vacc[r];
            }
        }
    }
    if (w == 0 && tid == 0) {
        long long rots = 0;
        if (!(failed || bad))
            for (int v = 0; v < G; ++v) {
                const uint4 b = ld16<kLocal>(rP, (int)sizeof(BjPart) * ((t & 1) * G + v) + 16);
                rots += (long long)(((unsigned long long)b.y << 32) | b.x);
            }
        // A failed call (a wait gave up, or C was not finite) is reported as
        // nonfinite; the sort kernel then writes NaN outputs.
        A.info->sweeps = failed ? -1 : sweeps;
        A.info->converged = (failed || bad) ? 0 : converged;
        A.info->nonfinite = (failed || bad) ? 1 : 0;
        A.info->floor_hit = floor_hit;
        A.info->off_rel = (failed || bad) ? (double)NAN : (fro2 > 0.0 ? sqrt(off2 / fro2) : 0.0);
        A.info->rotations = rots;
        A.info->steps = t;
        A.info->n_bands = m;
    }
}

__global__ __launch_bounds__(kThreads) void bj_kernel(BjArgs A, int res)
{
    __shared__ Smem L;
    if ((int)(blockIdx.x & 7) != res) return;
    const int w = (int)(blockIdx.x >> 3);
    const int tid = threadIdx.x;
    const int P = A.nb / 2, G = P * A.Q;

    // Inner schedule tables: steps 0..14 round-robin within each block, 15
    // the first cross step.
    for (int e = tid; e < (kC0 + 1) * 16; e += kThreads) {
        const int s = e >> 4, k = e & 15;
        int p, q;
        if (s < kC0) {
            const int kk = k & 7, off = (k >> 3) * kB;
            p = rr_pos(kB, s, kk) + off;
            q = rr_pos(kB, s, kB - 1 - kk) + off;
        } else {
            p = k;
            q = kB + k;
        }
        if (p > q) { const int tt = p; p = q; q = tt; }
        L.sp[s][k] = (unsigned char)p;
        L.sq[s][k] = (unsigned char)q;
        L.pid[s][p] = (unsigned char)k;
        L.pid[s][q] = (unsigned char)k;
    }
    if (tid == 0) { L.st_bad = 0; L.st_fail = 0; L.st_cnt = 0; }
    __syncthreads();
    if (tid < kUpper) {
        int e = tid, bk = 0;
        while (e >= kB - 1 - bk) { e -= kB - 1 - bk; ++bk; }
        const int bl = bk + 1 + e;
        for (int s = 0; s < kC0; ++s) {
            unsigned char a = 0xff, b = 0xff;
            const int pk = L.sp[s][bk], qk = L.sq[s][bk], pl = L.sp[s][bl], ql = L.sq[s][bl];
            const int ii[4] = {pk, pk, qk, qk}, jj[4] = {pl, ql, pl, ql};
            for (int h = 0; h < 4; ++h) {
                const int kn = L.pid[s + 1][ii[h]];
                if (kn == L.pid[s + 1][jj[h]]) {
                    const unsigned char v = (unsigned char)(h | (kn << 2));
                    if (a == 0xff) a = v;
                    else b = v;
                }
            }
            L.prodA[s][tid] = a;
            L.prodB[s][tid] = b;
        }
    }

    // XCD check: every participant publishes its XCD id, one device-scope
    // barrier, then the same decision everywhere.
    unsigned *xccs = A.flags + G;
    if (tid == 0) __hip_atomic_store(&xccs[w], xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    grid_sync<false>(L, A.flags, w, G, 1u);
    if (L.st_fail) {
        // A workgroup never arrived: report the failure (the sort kernel then
        // writes NaN outputs).
        if (w == 0 && tid == 0) {
            A.info->sweeps = -1;
            A.info->converged = 0;
            A.info->nonfinite = 1;
            A.info->floor_hit = 0;
            A.info->off_rel = (double)NAN;
            A.info->rotations = 0;
            A.info->steps = 0;
            A.info->n_bands = A.m;
        }
        return;
    }
    __shared__ int st_local;
    if (tid == 0) {
        const unsigned x0 = __hip_atomic_load(&xccs[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int same = 1;
        for (int v = 1; v < G; ++v)
            same &= __hip_atomic_load(&xccs[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == x0;
        st_local = same;
    }
    __syncthreads();
    if (st_local) bj_run<true>(L, A, w, 2u);
    else bj_run<false>(L, A, w, 2u);
}

}  // namespace

int bj_col_groups(int m)
{
    const int P = bj_blocks(m) / 2;
    int Q = P;
    while (Q > 1 && (P * Q > kBjMaxGroups || (P + Q - 1) / Q > kBjMaxColPairs)) --Q;
    return Q;
}

hipError_t launch_jacobi_block(const float *C, int m, double tol, int max_sweeps, int fp64_angles, char *ws,
                               double *lam_u, float *VuT, int nvu, pca_info *info_ws, hipStream_t st)
{
    static unsigned call_count = 0;
    const int nb = bj_blocks(m), P = nb / 2, Q = bj_col_groups(m), G = P * Q;
    const size_t Mp = (size_t)nb * kB;
    BjArgs a;
    a.C = C;
    a.m = m;
    a.nb = nb;
    a.Q = Q;
    a.max_sweeps = max_sweeps;
    a.fp64 = fp64_angles;
    a.tol = tol;
    a.H = reinterpret_cast<double *>(ws);
    a.U = a.H + 2 * Mp * Mp;
    a.V = reinterpret_cast<float *>(a.U + 2 * (size_t)P * 1024);
    a.part = reinterpret_cast<BjPart *>(a.V + Mp * Mp);
    a.flags = reinterpret_cast<unsigned *>(a.part + 2 * (size_t)G);
    a.lam_u = lam_u;
    a.VuT = VuT;
    a.nvu = nvu;
    a.info = info_ws;
    const int res = (int)(__atomic_fetch_add(&call_count, 1u, __ATOMIC_RELAXED) & 7u);
    hipLaunchKernelGGL(bj_clear_kernel, dim3(1), dim3(64), 0, st, a.flags, 2 * G);
    hipLaunchKernelGGL(bj_kernel, dim3((unsigned)(8 * G)), dim3(kThreads), 0, st, a, res);
    return hipGetLastError();
}

}  // namespace pca

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
//     cross steps, in four levels h = 8, 4, 2, 1: at level h each block is
//     cut into groups of 2h indices, and the first h of a group meet the
//     last h in h steps (member o with member (o + c) mod h), so that every
//     pair inside I and inside J is rotated once.
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
// t - 1. Its eight waves split a step as follows:
//   A. waves 0-3 load the operands of D into LDS; waves 4-7 start the loads
//      of the R and V operands;
//   B. waves 0-3: D = A_t[pair x, pair x] from two tiles of H_{t-1} and two
//      U's (float64 MFMA); waves 4-7 put the R and V operands in LDS;
//   C. wave 0: the inner rotations on D, held in registers (below), which
//      publish every step's rotations in LDS; waves 1-2: U_{t,x} from those
//      rotations in float64, one step behind; waves 3, 5-7 (wave 4 shares
//      wave 0's SIMD and stays idle): R = A_t[pair x,
//      pair j] = H_{t-1}[..] U_{t-1,j} (float64 MFMA), V_t[pair x rows, pair
//      j cols] = V_{t-1}[..] U_{t-1,j} (float32 MFMA), and the tiles' shares
//      of off(A_t)^2, ||A_t||_F^2;
//   D. all: H_t[pair x, pair j] = U_{t,x}^T R (float64 MFMA), stored with
//      U_{t,x} and the partial sums; then a grid barrier.
// Every workgroup of row x forms the same U_{t,x}. The stop rule (off(A)/
// ||C||_F <= tol, a sweep without any rotation, or max_sweeps) is evaluated
// at the start of every sweep from the partial sums of all workgroups, added
// in workgroup order, so every workgroup reaches the same decision. At the
// stop, A_t's diagonal is the eigenvalues and V_t the eigenvectors (unsorted;
// sort_sign_kernel follows).
//
// Inner rotations in registers. Wave 0 holds D in a relabelled order: the
// 16 rotation pairs of a phase (a level of the intra steps, or the cross
// steps) are (position k, position 16 + sigma_c(k)), k = 0..15, where sigma_c
// turns k by c inside its group of h positions. Lane 16 kg + l holds, for
// k = 4 kg + r (slots r = 0..3), the 2 x 2 block of rows (k, 16 + sigma_c(k))
// and columns (l, 16 + sigma_c(l)), so a step is four two-sided 2 x 2
// rotations per lane with no exchange; afterwards the second-member rows
// and columns move one group position on (in-lane slot renaming and lane
// permutes) to form the next step's blocks. The next step's pivot of pair k
// lies in the block (k, next(k)) of this step, so the lane holding it forms
// that rotation right after its own update (the diagonal after the step
// comes in closed form with the rotation records), and one LDS round trip
// per step publishes the 16 rotations to every lane and to waves 1-2. The
// rotations run in float32 (the tangent in float64 with
// PCA_JACOBI_FP64_ANGLES); U accumulates them in float64 with (cos, sin)
// normalised in float64. The inner sub-matrix only serves to find U: A itself
// is carried by the float64 tile products with U orthogonal to float64
// rounding, so the precision of the inner steps sets how fast the iteration
// converges, not the accuracy of the result (a rotation that leaves a small
// residue at its pivot is itself orthogonal; the residue is rotated again
// later).
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
// for the others gives up (and waves 1-2 give up on wave 0 likewise), and the
// call reports nonfinite output (NaN), so the launch always ends. Step flags
// are cleared by bj_clear_kernel before every launch, so a call does not
// depend on what the workspace held.
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
constexpr int kCg = kBjMaxColPairs;   // column pairs per workgroup, at most
constexpr long long kWaitTicks = 50000000;   // 0.5 s of the 100 MHz real-time counter
// Every bounded wait of this file is divided by 2^g_wait_shift (0 unless a
// test of the failure handling shortens them: pca_set_wait_shift).
__device__ int g_wait_shift = 0;
__device__ inline int wait_shift() { const int s = g_wait_shift; return s < 0 ? 0 : (s > 40 ? 40 : s); }
constexpr unsigned kRsrcWord3 = 0x00020000u;  // raw buffer resource, gfx9 family

struct BjPart {
    double off;          // sum of squares of this workgroup's off-diagonal entries of A_t
    double tot;          // sum of squares of all of its entries of A_t
    long long rot;       // rotations applied before step t (row's g = 0 workgroup only)
    long long pad;
};
static_assert(sizeof(BjPart) == 32, "partial-sum record size is part of the workspace layout");

struct Smem {
    double T1[kTiled], T2[kTiled], U1[kTiled], U2[kTiled];   // operands of D
    double Tj[kCg][kTiled], Uj[kCg][kTiled];                 // operands of R
    double R[kCg][kTiled];                                   // A_t[pair x, column pair]
    double Ui[kTiled];                                       // U_{t,x}
    float Ujf[kCg][kTile], Vb[kCg][kTile], Vo[kCg][kTile];   // V_{t-1} tiles, U_{t-1,j}, V_t tiles
    float D[kTile];                                          // A_t[pair x, pair x] (float32)
    float4 rec[kNS][16];   // rotation records of the inner steps: (cos, sin, a_pp, a_qq after)
    double red[2][2 * kCg * 4];   // per-tile off and total sums of squares of R
    int pub;               // inner steps whose records are published (wave 0 to waves 1-2)
    int st_bad, st_cnt, st_fail;
    int pub_spins;         // bound of waves 1-2's wait for a record, in polls
    long long wait_ticks;  // bound of a grid barrier wait, in real-time counter ticks
#ifdef BJ_PROFILE
    long long prof_w[8];
#endif
};

// Rotation of the pivot block [[app, apq], [apq, aqq]] (equations (2)-(5)
// with (7), the cancellation-free form of the tangent) as a record (cos,
// sin, a_pp - t a_pq, a_qq + t a_pq): row p becomes cos p - sin q, row q
// sin p + cos q, and the pivot vanishes. FP64 evaluates the tangent in
// float64. Skipped (cos 1, sin 0, diagonal unchanged) at the float32
// rounding floor of the block. No branches: every lane of the wave computes
// it and the caller keeps the records it needs.
template <bool FP64>
__device__ inline float4 make_rec(float app, float aqq, float apq, float floor_abs, int &applied)
{
    const float ad = fabsf(apq);
    const bool on = ad > floor_abs && ad * ad > 3.5527137e-15f * fabsf(app * aqq);   // |a_pq| > 2^-24 sqrt(|a_pp a_qq|)
    float tf;
    if constexpr (FP64) {
        // sqrt and the quotient from the hardware float64 estimates (about
        // single precision) refined by one Newton step each: relative error
        // near 2^-44, far below the float32 rounding of the result, with a
        // much shorter dependency chain than the correctly rounded forms.
        // A zero x (no pivot) gives inf / NaN here, which `on` discards.
        const double d = (double)aqq - (double)app, a = (double)apq;
        const double x = fma(d, d, 4.0 * a * a);
        double y = __builtin_amdgcn_rsq(x);
        y = y * fma(-0.5 * x * y, y, 1.5);
        const double den = fabs(d) + x * y;
        double q = __builtin_amdgcn_rcp(den);
        q = q * fma(-den, q, 2.0);
        tf = (float)((d >= 0.0 ? 2.0 * a : -2.0 * a) * q);
    } else {
        const float df = aqq - app;
        const float rf = __builtin_amdgcn_sqrtf(fmaf(df, df, 4.f * apq * apq));
        tf = (df >= 0.f ? 2.f * apq : -2.f * apq) * __builtin_amdgcn_rcpf(fabsf(df) + rf);
    }
    tf = on ? tf : 0.f;
    const float c = __builtin_amdgcn_rsqf(fmaf(tf, tf, 1.f));
    applied = on ? 1 : 0;
    return make_float4(on ? c : 1.f, tf * c, fmaf(-tf, apq, app), fmaf(tf, apq, aqq));
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

// Loads of one step's operand tiles go into registers, then to LDS; each
// helper takes the 16-byte piece e of its tile.
// 32 x 32 float64 tile of a label-space matrix (pitch ld elements): pieces
// 0..511.
template <bool kLocal>
__device__ inline uint4 issue_tiled(Rsrc src, int ld, int r0, int r1, int c0, int c1, int e)
{
    const int r = e >> 4, c = (e & 15) * 2;
    return ld16<kLocal>(src, 8 * (lab(r0, r1, r) * ld + lab(c0, c1, c)));
}
__device__ inline void commit_tiled(double *dst, uint4 v, int e)
{
    const int r = e >> 4, c = (e & 15) * 2;
    const double2 d = __builtin_bit_cast(double2, v);
    dst[r * kLdd + c] = d.x;
    dst[r * kLdd + c + 1] = d.y;
}
// U matrix number q (32 x 32 float64, contiguous): pieces 0..511.
template <bool kLocal>
__device__ inline uint4 issue_u(Rsrc src, int q, int e)
{
    const int r = e >> 4, c = (e & 15) * 2;
    return ld16<kLocal>(src, 8 * (q * 1024 + r * 32 + c));
}
__device__ inline void commit_u(double *dst, float *dstf, uint4 v, int e)
{
    const int r = e >> 4, c = (e & 15) * 2;
    const double2 d = __builtin_bit_cast(double2, v);
    dst[r * kLdd + c] = d.x;
    dst[r * kLdd + c + 1] = d.y;
    if (dstf) {
        dstf[r * kLd + c] = (float)d.x;
        dstf[r * kLd + c + 1] = (float)d.y;
    }
}
// 32 x 32 float32 tile of a label-space matrix: pieces 0..255.
template <bool kLocal>
__device__ inline uint4 issue_tile(Rsrc src, int ld, int r0, int r1, int c0, int c1, int e)
{
    const int r = e >> 3, c = (e & 7) * 4;
    return ld16<kLocal>(src, 4 * (lab(r0, r1, r) * ld + lab(c0, c1, c)));
}
__device__ inline void commit_tile(float *dst, uint4 v, int e)
{
    const int r = e >> 3, c = (e & 7) * 4;
    *reinterpret_cast<float4 *>(&dst[r * kLd + c]) = __builtin_bit_cast(float4, v);
}

// Workgroup barrier for LDS traffic only: this wave's LDS accesses complete,
// then s_barrier; global loads still in flight stay in flight (a
// __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xF | (0x3 << 14) | (0x7 << 4));   // lgkmcnt(0); vmcnt and expcnt not waited for
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
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
        const long long lim = L.wait_ticks;
        const long long t0 = now_ticks();
        int anybad = 0, fail = 0;
        bool done = false;
        while (!done) {
            // Eight polls between reads of the clock, so that the clock's
            // latency does not lengthen every poll.
            for (int i = 0; i < 8; ++i) {
                unsigned v = target << 1;
                if (lane < G)
                    v = kLocal ? poll_local(&flags[lane])
                               : __hip_atomic_load(&flags[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__all((v >> 1) >= target)) { anybad = __any((v & 1u) != 0u); done = true; break; }
            }
            if (!done && now_ticks() - t0 > lim) { fail = 1; break; }
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

// ---- inner rotations (wave 0) and U (waves 1-2) ----------------------------

// Position p (0..31) of phase H -> local index (0..31) of the block pair
// (block I = 0..15, block J = 16..31). The cross phase (H = 16) is the
// identity; intra level H takes, in each block, the first H indices of every
// group of 2H to positions 0..7 (block I) or 8..15 (block J) and their
// partners H further on to positions 16..31.
template <int H>
__device__ inline int ph_local(int p)
{
    if constexpr (H == 16) {
        return p;
    } else {
        const int k = p & 15, kk = k & 7;
        return ((k >> 3) << 4) + (kk / H) * (2 * H) + (kk % H) + (p >> 4) * H;
    }
}
// Position k turned by c inside its group of H positions, and its successor.
template <int H>
__device__ inline int ph_sigma(int c, int k) { return (k & ~(H - 1)) | ((k + c) & (H - 1)); }
template <int H>
__device__ inline int ph_next(int k) { return ph_sigma<H>(1, k); }

// Value v of lane src (any lane of the wave).
__device__ inline float lane_take(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ inline double lane_take(double v, int src)
{
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)b);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(b >> 32));
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (long long)(unsigned)lo);
}

// The value of lane 16 kg + next(l) of the same 16-lane row (next turns l
// inside its group of H): DPP row rotations and quad permutations, which
// move data between lanes without the LDS unit.
template <int CTRL>
__device__ inline float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int H>
__device__ inline float col_next(float v, int l)
{
    if constexpr (H == 16) {
        return dpp<0x12F>(v);                          // row_ror:15: lane i <- lane (i + 1) mod 16
    } else if constexpr (H == 8) {
        const float a = dpp<0x12F>(v), b = dpp<0x127>(v);   // row_ror:7: lane i <- lane (i - 7) mod 16
        return (l & 7) == 7 ? b : a;
    } else if constexpr (H == 4) {
        return dpp<0x39>(v);                           // quad_perm [1, 2, 3, 0]
    } else if constexpr (H == 2) {
        return dpp<0xB1>(v);                           // quad_perm [1, 0, 3, 2]
    } else {
        return v;
    }
}
template <int H>
__device__ inline double col_next(double v, int l)
{
    const unsigned long long b = __double_as_longlong(v);
    const float lo = col_next<H>(__int_as_float((int)(unsigned)b), l);
    const float hi = col_next<H>(__int_as_float((int)(unsigned)(b >> 32)), l);
    return __longlong_as_double(((long long)(unsigned)__float_as_int(hi) << 32) |
                                (long long)(unsigned)__float_as_int(lo));
}

// Wave 0 tells waves 1-2 that the records of inner steps below n are in LDS. The
// records were written earlier by this wave, and LDS carries out one wave's
// accesses in order; the empty asm keeps the compiler from moving them.
__device__ inline void publish(Smem &L, int n)
{
    asm volatile("" ::: "memory");
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(&L.pub, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    asm volatile("" ::: "memory");
}
// Waves 1-2 wait for the records of inner step s (bounded: false if wave 0
// never publishes them).
__device__ inline bool wait_pub(Smem &L, int s)
{
    int spins = 0;
    const int lim = L.pub_spins;
    while (__hip_atomic_load(&L.pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= s) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > lim) return false;
    }
    asm volatile("" ::: "memory");
    return true;
}

// Wave 0: the H inner steps of one phase, from inner step s0 on. D is read
// from LDS (local index space) at the start and written back at the end
// (kWrite). Returns the number of rotations applied by this lane's records.
// A step: the four 2 x 2 updates; the shifted values' lane permutes are
// issued; the pivot's owner forms the next step's rotation while they are in
// flight; the next step's records are read back while the loop turns.
template <int H, bool kWrite, bool FP64>
__device__ __attribute__((noinline)) int inner_phase(Smem &L, int s0, float floor_abs)
{
    const int lane = threadIdx.x & 63, kg = lane >> 4, l = lane & 15;
    float aII[4], aIJ[4], aJI[4], aJJ[4];
    {
        const int c0 = ph_local<H>(l), c1 = ph_local<H>(16 + l);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int r0 = ph_local<H>(4 * kg + r), r1 = ph_local<H>(16 + 4 * kg + r);
            aII[r] = L.D[r0 * kLd + c0];
            aIJ[r] = L.D[r0 * kLd + c1];
            aJI[r] = L.D[r1 * kLd + c0];
            aJJ[r] = L.D[r1 * kLd + c1];
        }
    }
    int napplied = 0;
    {
        const int k = lane & 15;
        const int p = ph_local<H>(k), q = ph_local<H>(16 + k);
        int ap;
        const float4 rc = make_rec<FP64>(L.D[p * kLd + p], L.D[q * kLd + q], L.D[p * kLd + q], floor_abs, ap);
        if (lane < 16) {
            L.rec[s0][lane] = rc;
            napplied += ap;
        }
    }
    publish(L, s0 + 1);
    // The slot whose block holds the next step's pivot of a pair (if any),
    // and the lanes the next step's values come from.
    int rp = -1;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (ph_next<H>(4 * kg + r) == l) rp = r;
    const int kg_row = H == 16 ? ((kg + 1) & 3) : (kg ^ 1);   // H = 8, 16: where slot 3's next row lives
    float4 rk[4], rl;
#pragma unroll
    for (int r = 0; r < 4; ++r) rk[r] = L.rec[s0][4 * kg + r];
    rl = L.rec[s0][l];
    for (int c = 0; c < H; ++c) {
        const int s = s0 + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float ck = rk[r].x, sk = rk[r].y;
            const float yII = ck * aII[r] - sk * aJI[r], yJI = sk * aII[r] + ck * aJI[r];
            const float yIJ = ck * aIJ[r] - sk * aJJ[r], yJJ = sk * aIJ[r] + ck * aJJ[r];
            aII[r] = rl.x * yII - rl.y * yIJ;
            aIJ[r] = rl.y * yII + rl.x * yIJ;
            aJI[r] = rl.x * yJI - rl.y * yJJ;
            aJJ[r] = rl.y * yJI + rl.x * yJJ;
        }
        if (c == H - 1) break;
        // The next step's rotation of pair 4 kg + rp: its pivot is this
        // block's (k, next(k)) entry, its diagonal the closed forms carried
        // by the records of pairs k and l = next(k).
        {
            float z = 0.f, dp = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r == rp) { z = aIJ[r]; dp = rk[r].z; }
            int ap;
            const float4 rc = make_rec<FP64>(dp, rl.w, z, floor_abs, ap);
            if (rp >= 0) {
                L.rec[s + 1][4 * kg + rp] = rc;
                napplied += ap;
            }
        }
        publish(L, s + 2);
        // The next step's records (read while the values below move).
#pragma unroll
        for (int r = 0; r < 4; ++r) rk[r] = L.rec[s + 1][4 * kg + r];
        rl = L.rec[s + 1][l];
        // Second members move one group position on: rows next(k) (in this
        // lane, or slot 3 from another 16-lane row), columns next(l).
        float nJI[4], nJJ[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int kn = ph_next<H>(r) & 3;   // slot of next(4 kg + r) when it stays in this lane
            if (H >= 8 && r == 3) {
                nJI[r] = lane_take(aJI[0], 16 * kg_row + l);
                nJJ[r] = lane_take(aJJ[0], 16 * kg_row + ph_next<H>(l));
            } else {
                nJI[r] = aJI[kn];
                nJJ[r] = col_next<H>(aJJ[kn], l);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            aIJ[r] = col_next<H>(aIJ[r], l);
            aJI[r] = nJI[r];
            aJJ[r] = nJJ[r];
        }
    }
    if constexpr (kWrite) {
        const int c0 = ph_local<H>(l), c1 = ph_local<H>(16 + ph_sigma<H>(H - 1, l));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 4 * kg + r;
            const int r0 = ph_local<H>(k), r1 = ph_local<H>(16 + ph_sigma<H>(H - 1, k));
            L.D[r0 * kLd + c0] = aII[r];
            L.D[r0 * kLd + c1] = aIJ[r];
            L.D[r1 * kLd + c0] = aJI[r];
            L.D[r1 * kLd + c1] = aJJ[r];
        }
    }
    return napplied;
}

// All inner steps of outer step t (the intra levels first at a sweep start).
template <bool FP64>
__device__ int inner_all(Smem &L, bool first, float floor_abs)
{
    int napp = 0;
    if (first) {
        napp += inner_phase<8, true, FP64>(L, 0, floor_abs);
        napp += inner_phase<4, true, FP64>(L, 8, floor_abs);
        napp += inner_phase<2, true, FP64>(L, 12, floor_abs);
        napp += inner_phase<1, true, FP64>(L, 14, floor_abs);
        napp += inner_phase<16, false, FP64>(L, 15, floor_abs);
    } else {
        napp += inner_phase<16, false, FP64>(L, 0, floor_abs);
    }
    return napp;
}

// Waves 1 and 2: U <- U P for the H steps of one phase, one step behind
// wave 0. Wave 1 + h (h = 0, 1) holds rows 16 h .. 16 h + 15: lane 16 rg + l
// the columns at positions l and 16 + sigma_c(l) of rows 16 h + 4 rg ..
// 16 h + 4 rg + 3. U starts as the identity (first) or from LDS, and ends
// in LDS. False if wave 0's records never came.
template <int H>
__device__ __attribute__((noinline)) bool u_phase(Smem &L, int s0, bool first, int h)
{
    const int lane = threadIdx.x & 63, rg = lane >> 4, l = lane & 15;
    double uI[4], uJ[4];
    {
        const int c0 = ph_local<H>(l), c1 = ph_local<H>(16 + l);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rho = 16 * h + 4 * rg + q;
            uI[q] = first ? (rho == c0 ? 1.0 : 0.0) : L.Ui[rho * kLdd + c0];
            uJ[q] = first ? (rho == c1 ? 1.0 : 0.0) : L.Ui[rho * kLdd + c1];
        }
    }
    for (int c = 0; c < H; ++c) {
        if (!wait_pub(L, s0 + c)) return false;
        const float4 rr = L.rec[s0 + c][l];
        const double2 cs = rot64(make_float2(rr.x, rr.y));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double a = uI[q], b = uJ[q];
            uI[q] = cs.x * a - cs.y * b;
            uJ[q] = cs.y * a + cs.x * b;
        }
        if (c < H - 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) uJ[q] = col_next<H>(uJ[q], l);
        }
    }
    const int c0 = ph_local<H>(l), c1 = ph_local<H>(16 + ph_sigma<H>(H - 1, l));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rho = 16 * h + 4 * rg + q;
        L.Ui[rho * kLdd + c0] = uI[q];
        L.Ui[rho * kLdd + c1] = uJ[q];
    }
    return true;
}

// ---- tile tasks of the other waves ------------------------------------------

// Shares of off(A_t)^2 and ||A_t||_F^2 of one 16 x 16 tile of R (this
// lane's four entries), into slot e.
__device__ inline void tile_sums(Smem &L, const double (&v)[4], int I, int J, int K, int Lb, int ti, int tj, int e)
{
    const int lane = threadIdx.x & 63, orow = 4 * (lane >> 4), ocol = lane & 15;
    const int gc = lab(K, Lb, 16 * tj + ocol);
    double so = 0.0, st = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double q = v[r] * v[r];
        st += q;
        if (lab(I, J, 16 * ti + orow + r) != gc) so += q;
    }
    so = wave_sum(so);
    st = wave_sum(st);
    if (lane == 0) {
        L.red[0][e] = so;
        L.red[1][e] = st;
    }
}

// Tile (ti, tj) of R[jj] = Tj[jj] Uj[jj] (t > 0; at t = 0 R[jj] holds C's
// tile already).
__device__ inline void r_tile(Smem &L, int jj, int ti, int tj)
{
    const int lane = threadIdx.x & 63, orow = 4 * (lane >> 4), ocol = lane & 15;
    const f64x4 acc = tile16d(L.Tj[jj] + 16 * ti * kLdd, kLdd, false, L.Uj[jj] + 16 * tj, kLdd);
#pragma unroll
    for (int r = 0; r < 4; ++r) L.R[jj][(16 * ti + orow + r) * kLdd + 16 * tj + ocol] = acc[r];
}
// The sums of tile (ti, tj) of R[jj] (read back by the lanes that wrote it,
// or any lanes once a barrier has passed).
__device__ inline void r_sums(Smem &L, int jj, int ti, int tj, int I, int J, int K, int Lb)
{
    const int lane = threadIdx.x & 63, orow = 4 * (lane >> 4), ocol = lane & 15;
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = L.R[jj][(16 * ti + orow + r) * kLdd + 16 * tj + ocol];
    tile_sums(L, v, I, J, K, Lb, ti, tj, 4 * jj + 2 * ti + tj);
}

// Tile (ti, tj) of V_t[pair x rows, column pair jj] = V_{t-1} U_{t-1,j}
// (the identity's tile at t = 0): to global V and to Vo.
__device__ inline void v_task(Smem &L, float *V, int Mp, int jj, int ti, int tj, bool first, int I, int J, int K,
                              int Lb)
{
    const int lane = threadIdx.x & 63, orow = 4 * (lane >> 4), ocol = lane & 15;
    const int gc = lab(K, Lb, 16 * tj + ocol);
    f32x4 acc;
    if (first) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = lab(I, J, 16 * ti + orow + r) == gc ? 1.f : 0.f;
    } else {
        acc = tile16(L.Vb[jj] + 16 * ti * kLd, kLd, false, L.Ujf[jj] + 16 * tj, kLd);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        V[(int64_t)lab(I, J, 16 * ti + orow + r) * Mp + gc] = acc[r];
        L.Vo[jj][(16 * ti + orow + r) * kLd + 16 * tj + ocol] = acc[r];
    }
}

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
    const int orow = 4 * (lane >> 4), ocol = lane & 15;
    long long mycnt = 0, cnt_prev = 0;
    double fro2 = 0.0, off2 = 0.0, lim2 = 0.0;
    float floor_abs = 0.f;
    int sweeps = 0, converged = 0, floor_hit = 0, bad = 0, failed = 0;
    int t = 0;
    int I = 0, J = 0;
    int Kc[kCg] = {0}, Lc[kCg] = {0};

    for (;; ++t) {
        uint4 vRT[kCg][2], vRU[kCg][2], vRV[kCg];   // R and V operand pieces in flight (waves 4-7)
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

        // ---- A: operands of step t ---------------------------------------------
        if (t == 0) {
            // A_0 = C (padded with zeros): D and the R tiles straight from C.
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
        } else {
            // Waves 0-3 load the operands of D (T1, T2, U1, U2: two pieces of
            // each per thread) and put them in LDS; waves 4-7 start the loads
            // of the R and V operands, which stay in flight across the next
            // barrier and reach LDS while D is formed.
            const int hb = ((t - 1) & 1) * nb;              // block-row offset of H_{t-1}
            const int uoff = ((t - 1) & 1) * P;             // U index offset of step t-1
            const int e0 = tid & 255;
            if (wave < 4) {
                uint4 v[8];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + 256 * h;
                    v[h] = issue_tiled<kLocal>(rH, Mp, hb + I, hb + J, rr_pos(nb, up, q1), rr_pos(nb, up, nb - 1 - q1), e);
                    v[2 + h] = issue_tiled<kLocal>(rH, Mp, hb + I, hb + J, rr_pos(nb, up, q2),
                                                   rr_pos(nb, up, nb - 1 - q2), e);
                    v[4 + h] = issue_u<kLocal>(rU, uoff + q1, e);
                    v[6 + h] = issue_u<kLocal>(rU, uoff + q2, e);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + 256 * h;
                    commit_tiled(L.T1, v[h], e);
                    commit_tiled(L.T2, v[2 + h], e);
                    commit_u(L.U1, nullptr, v[4 + h], e);
                    commit_u(L.U2, nullptr, v[6 + h], e);
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < kCg; ++jj) {
                    // (a second copy of column pair 0 when there is no second)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        vRT[jj][h] = issue_tiled<kLocal>(rH, Mp, hb + I, hb + J, Kc[jj], Lc[jj], e0 + 256 * h);
                        vRU[jj][h] = issue_u<kLocal>(rU, uoff + g + (jj < ncg ? jj : 0) * Q, e0 + 256 * h);
                    }
                    vRV[jj] = issue_tile<kLocal>(rV, Mp, I, J, Kc[jj], Lc[jj], e0);
                }
            }
        }
        if (tid == 0) L.pub = 0;
        if (t == 0) __syncthreads();
        else lds_barrier();
        PROF(0);

        // ---- B: D (waves 0-3); the R and V operands reach LDS (waves 4-7) ------
        if (t > 0) {
            const int ti = (wave >> 1) & 1, tj = wave & 1;
            if (wave < 4) {
                // Columns of block I from (T1, U1), of block J from (T2, U2).
                const double *Ta = tj == 0 ? L.T1 : L.T2;
                const double *Ua = (tj == 0 ? L.U1 : L.U2) + 16 * (tj == 0 ? o1 : o2);
                const f64x4 dacc = tile16d(Ta + 16 * ti * kLdd, kLdd, false, Ua, kLdd);
#pragma unroll
                for (int r = 0; r < 4; ++r) L.D[(16 * ti + orow + r) * kLd + 16 * tj + ocol] = (float)dacc[r];
            } else {
                const int e0 = tid & 255;
#pragma unroll
                for (int jj = 0; jj < kCg; ++jj) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        commit_tiled(L.Tj[jj], vRT[jj][h], e0 + 256 * h);
                        commit_u(L.Uj[jj], L.Ujf[jj], vRU[jj][h], e0 + 256 * h);
                    }
                    commit_tile(L.Vb[jj], vRV[jj], e0);
                }
            }
        }
        __syncthreads();
        PROF(1);

        // ---- C: inner rotations (wave 0), U (waves 1-2), other tiles (waves 3, 5-7)
#ifdef BJ_PROFILE
        const long long tC = now_ticks();
#endif
        if (wave == 0) {
            int napp = fp64 ? inner_all<true>(L, u == 0, floor_abs) : inner_all<false>(L, u == 0, floor_abs);
            napp = wave_sum_int(napp);
            if (lane == 0) L.st_cnt = napp;
#ifdef BJ_PROFILE
            if (lane == 0) prof_[5] += now_ticks() - tC;
#endif
        } else if (wave <= 2) {
            const int h = wave - 1;
            bool ok;
            if (u == 0) {
                ok = u_phase<8>(L, 0, true, h) && u_phase<4>(L, 8, false, h) && u_phase<2>(L, 12, false, h) &&
                     u_phase<1>(L, 14, false, h) && u_phase<16>(L, 15, false, h);
            } else {
                ok = u_phase<16>(L, 0, true, h);
            }
            if (!ok && lane == 0) L.st_fail = 1;
#ifdef BJ_PROFILE
            if (lane == 0) L.prof_w[wave] = now_ticks() - tC;
#endif
        } else if (wave != 4) {
            // Tasks: 0-7 the R tiles of the column pairs (with their sums),
            // 8-15 V tiles, over waves 3, 5, 6, 7: wave 4 shares a SIMD with
            // wave 0, whose inner steps are the critical path, and stays
            // idle here so that they get its issue slots (1.52 -> 1.44 ms at
            // 224 bands; the tasks, about 5 us a step, stay off the path).
            const int slot = wave == 3 ? 0 : wave - 4;
            for (int task = slot; task < 16; task += 4) {
                const int jj = (task >> 2) & 1;
                const int K = jj ? Kc[1] : Kc[0], Lb = jj ? Lc[1] : Lc[0];   // (selects, not an indexed array)
                if (jj >= ncg) continue;
                if (task < 8) {
                    if (t > 0) r_tile(L, jj, (task >> 1) & 1, task & 1);
                    r_sums(L, jj, (task >> 1) & 1, task & 1, I, J, K, Lb);
                } else {
                    v_task(L, A.V, Mp, jj, (task >> 1) & 1, task & 1, t == 0, I, J, K, Lb);
                }
            }
#ifdef BJ_PROFILE
            if (lane == 0) L.prof_w[wave] = now_ticks() - tC;
#endif
        }
        __syncthreads();
#ifdef BJ_PROFILE
        if (tid == 0) {
            prof_[6] += L.prof_w[1] > L.prof_w[2] ? L.prof_w[1] : L.prof_w[2];
            long long mx = 0;
            for (int v = 3; v < 8; ++v) mx = L.prof_w[v] > mx ? L.prof_w[v] : mx;
            prof_[7] += mx;
        }
#endif
        PROF(2);

        // ---- D: H_t = U_{t,x}^T R, U_{t,x}, partial sums -----------------------
        {
            const int wjj = wave >> 2, ti = (wave >> 1) & 1, tj = wave & 1;
            if (wjj < ncg) {
                const f64x4 hacc = tile16d(L.Ui + 16 * ti, kLdd, true, L.R[wjj] + 16 * tj, kLdd);
                double *Hd = A.H + (int64_t)(t & 1) * Mp * Mp;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Hd[(int64_t)lab(I, J, 16 * ti + orow + r) * Mp + lab(Kc[wjj], Lc[wjj], 16 * tj + ocol)] = hacc[r];
            }
        }
        if (g == 0) {
            const int r = tid >> 4, c = (tid & 15) * 2;
            double *Ud = A.U + ((int64_t)(t & 1) * P + x) * 1024;
            *reinterpret_cast<double2 *>(&Ud[r * 32 + c]) = make_double2(L.Ui[r * kLdd + c], L.Ui[r * kLdd + c + 1]);
        }
        if (tid == 0) {
            BjPart pp;
            double so = 0.0, st = 0.0;
            for (int e = 0; e < 4 * ncg; ++e) {
                so += L.red[0][e];
                st += L.red[1][e];
            }
            pp.off = so;
            pp.tot = st;
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

        // ---- stop rule at the start of a sweep -------------------------------------
        // (Checked per sweep, not per outer step: the quadratic convergence of
        // the last sweep takes off(A) well below the tolerance, which the
        // eigenvector accuracy needs on spectra with small gaps.)
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
                if (gr < m && gc < m) A.VuT[(int64_t)gc * A.nvu + gr] = L.Vo[jj][r * kLd + c];
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
    if (tid == 0) {
        L.st_bad = 0;
        L.st_fail = 0;
        L.st_cnt = 0;
        L.pub = 0;
        // The wait bounds, read once per launch (see g_wait_shift).
        const int sh = wait_shift();
        L.wait_ticks = kWaitTicks >> sh;
        L.pub_spins = (1 << 22) >> (sh > 22 ? 22 : sh);
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

hipError_t set_wait_shift_block(int shift)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(g_wait_shift), &shift, sizeof(int));
}

}  // namespace pca

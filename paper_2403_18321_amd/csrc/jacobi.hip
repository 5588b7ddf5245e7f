// Cyclic Jacobi eigendecomposition of the covariance (Section 2: equations
// (2)-(10), the parallel-rotation property and the stop rule).
//
// Ordering. n = bands rounded up to even (an odd band count gets a phantom
// index with a zero row, which is never rotated). A parallel step rotates
// n/2 disjoint pairs; the pairs come from a round-robin tournament ("circle"
// construction: position 0 stays, positions 1..n-1 turn by one each step), so
// n - 1 steps visit every pair once, which is one sweep.
//
// Slot layout. Position k (k < n/2) is slot T_k and position n-1-k is slot
// B_k, so pair k is always (T_k, B_k). The matrix is kept in slot
// coordinates and physically permuted after every step, so that the pairs
// never move: the permutation is the same fixed map every step and each
// thread's source and destination LDS addresses are computed once. After
// n - 1 steps the slots are back in their initial places.
//
// Storage (LDS). The off-diagonal entries form 2x2 blocks (k, l), k < l:
// rows (T_k, B_k) x columns (T_l, B_l), 16 bytes each, read with one b128
// load; block row k is contiguous and starts at a padded offset (3k mod 16
// blocks) so that the lanes of a wave, which hold the same place in
// consecutive rows, read distinct banks; the four components sit in a
// per-row swizzled order so that their b32 stores hit distinct banks too.
// The pivots (T_k, B_k) are not stored: the thread that produces one
// computes its rotation on the spot. The diagonal is float64 in a separate
// double-buffered array, as are the rotations (tan, cos).
//
// jacobi_kernel (one workgroup of 1024 threads, one CU). A step:
//   a. every thread rotates its 2x2 blocks: rows by R_k^T, columns by R_l --
//      the row and column updates of C_k = P^T C P, equation (8), for all
//      pairs of the step at once;
//   b. barrier; the rotated entries are written to their permuted places.
//      Whoever produces a pivot of the next step also computes that pivot's
//      rotation (equations (2)-(5) with (7), as t = sgn(theta) / (|theta| +
//      sqrt(1 + theta^2)), float64 by default), the new diagonal entries
//      a_pp - t a_pq and a_qq + t a_pq, and logs (cos, sin).
// Two barriers per step. Before each sweep the off-diagonal norm is reduced
// in float64; the iteration stops when it is <= tol ||C||_F, after a sweep
// that applied no rotation, or after max_sweeps sweeps.
//
// vreplay_kernel: E = P_1 P_2 ... P_K (equation (10)) from the rotation log.
// Rows of E evolve independently under E <- E P; each workgroup replays the
// whole log on a few rows, in the same slot coordinates.
//
// jacobi_follow_kernel: the same two computations in one launch. Workgroup 0
// runs the Jacobi sweeps; workgroups 1.. replay the rotation log on their
// rows of E while it is being written, so that the replay ends a batch or so
// after the last rotation instead of starting then. The log entries validate
// themselves: the log starts zeroed, a real entry has cos >= 1/sqrt(2) > 0,
// and after the last step the Jacobi workgroup fills the rest of the current
// kLogBatch-step batch with end marks (cos = -1). A follower waits until every
// entry of its next batch is non-zero (each entry is written once per call,
// so its first non-zero value is final), replays the steps before the first
// end mark and stops there. Entries go through agent-scope coherent stores
// and loads, which are visible across the chip's separate L2 caches without
// cache flushes or fences. log_clear_kernel zeroes the whole log before the
// launch, so nothing a previous call left in the workspace is ever read as an
// entry. The Jacobi workgroup never waits for the followers,
// and a follower that sees an entry stay zero for about a second writes NaN
// rows and exits, so every workgroup ends.
//
// sort_sign_kernel: eigenvalues from the diagonal, sorted in descending order
// (stable), eigenvector columns permuted to match (Code 4.4.3), and the sign
// of each column fixed so its largest-magnitude entry is positive.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace pca {

namespace {

constexpr int kJThreads = 1024;
constexpr int kMaxP = 128;
constexpr int kMaxRowBlocks = 9088;   // padded block rows for 128 pairs (see row_start)
constexpr int kBlockPad = 32;         // tail that segment reads may run into
constexpr int kCsPad = 32;
constexpr int kLoadPerThread = 16;    // loads in flight per pass
constexpr double kFloorRel2 = 3.552713678800501e-15;   // (2^-24)^2
constexpr float kLogEnd = -1.f;       // cos of an end mark in the rotation log

// The matrix blocks of the Jacobi workgroup; a follower workgroup of the
// same launch uses the same LDS for its rows of E and its log batch.
__shared__ float4 jac_blk[kMaxRowBlocks + kBlockPad];

__device__ inline void log_store(float2 *p, float2 v)
{
    const unsigned long long bits =
        (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), bits, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float2 log_load(const float2 *p)
{
    const unsigned long long bits = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((unsigned int)bits), __uint_as_float((unsigned int)(bits >> 32)));
}

struct Slots {
    int P, n;
    const int *R;   // first block of each block row (LDS)

    __device__ void init(int n_, const int *R_, const unsigned char *W_) {
        n = n_;
        P = n_ / 2;
        R = R_;
        W = W_;
    }
    // Slot ids: T_k = k, B_k = P + k. Where a slot's entries go after a step:
    // the index at position j moves to position j - 1 (j >= 2), position 1
    // wraps to n - 1, position 0 stays. (Turning the circle this way round
    // took 7 instead of 10 sweeps on the 224-band covariance and never more
    // sweeps on the other workloads; the other direction is the same set of
    // rounds in reverse order.)
    __device__ int next(int x) const {
        if (P == 1) return x;
        if (x < P) {
            if (x == 0) return 0;
            return x == 1 ? P : x - 1;
        }
        const int k = x - P;
        return k <= P - 2 ? P + k + 1 : P - 1;
    }
    // Index of block (k, l), k < l: block row k is stored contiguously from
    // R[k]; rows start at R[k] = 3k (mod 16) so that the lanes of a wave,
    // which take the same place in consecutive rows, hit distinct LDS banks.
    __device__ int bi(int k, int l) const { return R[k] + (l - k - 1); }
    // Component c = 2 [row is a B slot] + [column is a B slot] of a block in
    // block row a is stored at position c ^ W[a] of the block's 16 bytes
    // (T/B rows and/or columns swapped). Lanes of a half-wave take rows
    // k .. k+31 and write a component of a block in row k -/+ 1 whose index
    // repeats mod 8 every 8 rows; the b32 write path resolves 32 banks per 32
    // lanes, so the position must differ between rows 8 apart. W[a] is the
    // running XOR of (j >> 3) & 3 over j = 1 .. a: a row's source swizzle and
    // its neighbour's destination swizzle then differ by (a >> 3) & 3.
    const unsigned char *W;
    __device__ int sw(int a) const { return W[a]; }
    // Where the off-diagonal entry (x, y), x != y, lives: a float index into
    // the block rows, or -1 - k for the pivot (T_k, B_k).
    __device__ int code(int x, int y) const {
        int a = x, b = y, xb = 0, yb = 0;
        if (a >= P) { a -= P; xb = 1; }
        if (b >= P) { b -= P; yb = 1; }
        if (a == b) return -1 - a;
        if (a > b) {
            const int t = a; a = b; b = t;
            const int u = xb; xb = yb; yb = u;
        }
        return 4 * bi(a, b) + ((2 * xb + yb) ^ W[a]);
    }
    // Slot of physical index i at the start of a sweep, and back.
    __device__ int slot_of(int i) const { return i < P ? i : P + (n - 1 - i); }
    __device__ int phys(int x) const { return x < P ? x : n - 1 - (x - P); }
};

// Start of each padded block row (R[0 .. P]).
__host__ __device__ inline int row_start_next(int P, int k, int Rk)
{
    const int e = Rk + (P - 1 - k);
    return e + (((3 * (k + 1) - e) % 16) + 16) % 16;
}

// Generic blocks of row k: l = k + 3 .. P - 2. For them every rotated entry
// lands in a regular component of another block at a fixed offset, so a run
// of them along a row moves by constant strides.
__host__ __device__ inline int generic_len(int P, int k) { return (P >= 5 && k <= P - 5) ? P - k - 4 : 0; }
// Generic segments with segment index s (one per row that is long enough).
__host__ __device__ inline int segments_at(int P, int L, int s)
{
    const int c = P - 4 - L * s;
    return c > 0 ? c : 0;
}

// 1/sqrt(x) and 1/x in float64 from the hardware estimates refined by two
// Newton steps each (the estimates carry roughly single precision, so two
// steps reach double precision).
__device__ inline double rsqrt64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}
__device__ inline double rcp64(double x)
{
    double q = __builtin_amdgcn_rcp(x);
    q = q * fma(-x, q, 2.0);
    q = q * fma(-x, q, 2.0);
    return q;
}

// Rotation of a pivot pair, equations (2)-(5) with (7):
//   theta = (a_qq - a_pp) / (2 a_pq), t = sgn(theta) / (|theta| + sqrt(1 + theta^2))
// evaluated as t = sgn(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp
// (the same number), cos = 1/sqrt(1 + t^2), sin = t cos. Skipped (t = 0,
// cos = 1) when |a_pq| is at the float32 rounding floor. Returns (t, cos).
__device__ inline void rotation(double app, double aqq, float apq, double floor_abs, int fp64, float2 &tc,
                                double &dT, double &dB, float &pv)
{
    const double a = (double)apq;
    const double ad = fabs(a);
    if (apq != 0.f && ad > floor_abs && ad * ad > kFloorRel2 * fabs(app * aqq)) {
        double t;
        if (fp64) {
            const double d = aqq - app;
            const double x = fma(d, d, 4.0 * a * a);
            const double r = x * rsqrt64(x);
            t = (d >= 0.0 ? 2.0 * a : -2.0 * a) * rcp64(fabs(d) + r);
            tc = make_float2((float)t, (float)rsqrt64(fma(t, t, 1.0)));
        } else {
            const float df = (float)aqq - (float)app;
            const float rf = sqrtf(df * df + 4.f * apq * apq);
            const float tf = (df >= 0.f ? 2.f * apq : -2.f * apq) / (fabsf(df) + rf);
            tc = make_float2(tf, 1.f / sqrtf(1.f + tf * tf));
            t = tf;
        }
        dT = app - t * a;
        dB = aqq + t * a;
        pv = 0.f;
    } else {
        tc = make_float2(0.f, 1.f);
        dT = app;
        dB = aqq;
        pv = apq;
    }
}

__device__ inline double block_sum_d(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

__device__ inline int block_sum_i(int v, int *red)
{
    v = wave_sum_int(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

// Work of one thread in a step (fixed for the whole run):
//   a generic segment: blocks (k, l0 .. l0 + len - 1) of one row, len <= L.
//     Source and destination addresses are the segment's base plus a
//     constant per block, so the step code holds five base registers and
//     uses immediate LDS offsets (one b128 read per block). Segments are
//     numbered segment-index-major, so the lanes of a wave take the same
//     segment of consecutive rows;
//   one special block (the diagonals next to the pivots and the last column),
//     with explicit destination codes; a special block that produces a pivot
//     of the next step also computes that pivot's rotation;
//   thread j < P moves pair j's rotated pivot to its next place;
//   thread 1024 - P + j logs pair j's rotation.
// kFollow: the rotation log is read while it is written (coherent stores,
// end marks after the last step).
template <int L, bool kFollow>
__device__ __forceinline__ void jacobi_body(const float *__restrict__ C, int m, int n, double tol, int max_sweeps,
                                   int fp64_angles, double *__restrict__ lam_u, float2 *__restrict__ rlog,
                                   pca_info *__restrict__ info)
{
    float4 *blk = jac_blk;
    __shared__ double dg[2][256];
    __shared__ float2 csb[2][kMaxP + kCsPad];   // (tan, cos) of each pair's rotation
    __shared__ float pvb[2][kMaxP];             // pivot after its rotation (0 unless skipped)
    __shared__ float pva[kMaxP];                // pivot before its rotation
    __shared__ int rowR[kMaxP + 1];
    __shared__ unsigned char rowW[kMaxP];
    __shared__ double redd[16];
    __shared__ int redi[16];
    __shared__ int bad;

    const int tid = threadIdx.x;
    const int P = n / 2;
    if (tid == 0) {
        int r = 0;
        rowR[0] = 0;
        int w = 0;
        for (int k = 0; k < P; ++k) {
            r = row_start_next(P, k, r);
            rowR[k + 1] = r;
            w ^= (k >> 3) & 3;
            rowW[k] = (unsigned char)w;
        }
        bad = 0;
    }
    __syncthreads();
    Slots S;
    S.init(n, rowR, rowW);
    const int nbf = 4 * rowR[P];   // floats of the padded block rows
    float *Af = reinterpret_cast<float *>(blk);

    // Generic segment of this thread.
    int gk = 0, l0 = 0, len = 0;
    {
        int cum = 0, sg = 0;
        while (true) {
            const int c = segments_at(P, L, sg);
            if (c == 0 || tid < cum + c) {
                if (c > 0) {
                    gk = tid - cum;
                    l0 = gk + 3 + L * sg;
                    len = min(L, P - 1 - l0);
                }
                break;
            }
            cum += c;
            ++sg;
        }
    }
    // Register r of a block read from row k holds component r ^ sw(k); the
    // rotation is applied in that order with the tangents of swapped pairs
    // negated (swapping T and B of a pair turns its rotation into the one by
    // the opposite angle), and result r goes to component r ^ sw(k)'s place.
    int gsrc = 0, gd[4] = {0, 0, 0, 0};
    float gsr = 1.f, gsc = 1.f;
    if (len > 0) {
        gsrc = S.bi(gk, l0);
        const int w = S.sw(gk);
        gsr = (w & 2) ? -1.f : 1.f;
        gsc = (w & 1) ? -1.f : 1.f;
        const int xs[2] = {gk, P + gk}, ys[2] = {l0, P + l0};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) gd[(2 * a + b) ^ w] = S.code(S.next(xs[a]), S.next(ys[b]));
    }

    // Special block of this thread: the pivot sources (k, k + 2), (0, 1) and
    // (P-2, P-1) first, then the other (k, k + 1), then (k, P - 1).
    int ssrc = 0, sk = 0, sl = 0, sd[4] = {0, 0, 0, 0};
    int mine0 = -1, mc0 = 0, mine1 = -1, mc1 = 0;
    float ssr = 1.f, ssc = 1.f;
    bool has_sp = false;
    {
        const int nd2 = P >= 2 ? P - 2 : 0;
        int k = -1, l = -1;
        const int i = tid;
        if (P >= 2) {
            if (i < nd2) { k = i; l = i + 2; }
            else if (i == nd2) { k = 0; l = 1; }
            else if (P >= 3 && i == nd2 + 1) { k = P - 2; l = P - 1; }
            else if (P >= 4) {
                int j = i - nd2 - 2;
                if (j < P - 3) { k = 1 + j; l = 2 + j; }
                else if ((j -= P - 3) < P - 3) { k = j; l = P - 1; }
            }
        }
        if (k >= 0) {
            has_sp = true;
            ssrc = S.bi(k, l);
            sk = k;
            sl = l;
            const int w = S.sw(k);
            ssr = (w & 2) ? -1.f : 1.f;
            ssc = (w & 1) ? -1.f : 1.f;
            const int xs[2] = {k, P + k}, ys[2] = {l, P + l};
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const int c = S.code(S.next(xs[a]), S.next(ys[b]));
                    const int r = (2 * a + b) ^ w;
                    sd[r] = c;
                    if (c < 0) {
                        if (mine0 < 0) { mine0 = -1 - c; mc0 = r; }
                        else { mine1 = -1 - c; mc1 = r; }
                    }
                }
        }
    }
    // Where thread j's rotated pivot goes.
    const int pcode = tid < P ? S.code(S.next(tid), S.next(P + tid)) : 0;

    // ---- load C (upper triangle) into the slot layout ---------------------
    for (int e = tid; e < 4 * (kMaxRowBlocks + kBlockPad); e += kJThreads) Af[e] = 0.f;
    for (int i = tid; i < 256; i += kJThreads) { dg[0][i] = 0.0; dg[1][i] = 0.0; }
    for (int i = tid; i < kMaxP; i += kJThreads) { pva[i] = 0.f; pvb[0][i] = 0.f; pvb[1][i] = 0.f; }
    for (int i = tid; i < 2 * (kMaxP + kCsPad); i += kJThreads) (&csb[0][0])[i] = make_float2(0.f, 1.f);
    __syncthreads();
    {
        const int mm = m * m;
        int nonfin = 0;
        for (int base = 0; base < mm; base += kLoadPerThread * kJThreads) {
            float tmp[kLoadPerThread];
#pragma unroll
            for (int q = 0; q < kLoadPerThread; ++q) {
                const int e = base + tid + q * kJThreads;
                tmp[q] = e < mm ? C[e] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < kLoadPerThread; ++q) {
                const int e = base + tid + q * kJThreads;
                if (e < mm) {
                    const int i = e / m, j = e - (e / m) * m;
                    if (j >= i) {
                        if (!isfinite(tmp[q])) nonfin = 1;
                        const int si = S.slot_of(i), sj = S.slot_of(j);
                        if (i == j) {
                            dg[0][si] = (double)tmp[q];
                        } else {
                            const int c = S.code(si, sj);
                            if (c >= 0) Af[c] = tmp[q];
                            else pva[-1 - c] = tmp[q];
                        }
                    }
                }
            }
        }
        if (nonfin) atomicOr(&bad, 1);
    }
    __syncthreads();

    auto offnorm2 = [&]() -> double {
        double part = 0.0;
        for (int e = tid; e < nbf; e += kJThreads) part += (double)Af[e] * (double)Af[e];
        for (int j = tid; j < P; j += kJThreads) part += (double)pva[j] * (double)pva[j];
        return 2.0 * block_sum_d(part, redd);
    };

    double fro2;
    {
        double part = 0.0;
        for (int i = tid; i < n; i += kJThreads) part += dg[0][i] * dg[0][i];
        fro2 = block_sum_d(part, redd) + offnorm2();
    }
    const bool failed = bad != 0;
    const double floor_abs = 5.9604644775390625e-08 * sqrt(fro2) / (double)m;

    // Rotation of pair k for the step whose diagonal is in dg[src]; writes
    // (tan, cos) and the rotated pivot into slot `par`, the rotated diagonal
    // (already permuted) into dg[dsto].
    auto rotate = [&](int k, float apq, int src, int dsto, int par) {
        float2 tc;
        double dT, dB;
        float pv;
        rotation(dg[src][k], dg[src][P + k], apq, floor_abs, fp64_angles, tc, dT, dB, pv);
        csb[par][k] = tc;
        pvb[par][k] = pv;
        dg[dsto][S.next(k)] = dT;
        dg[dsto][S.next(P + k)] = dB;
    };

    // Rotations of step 0.
    if (tid < P && !failed) rotate(tid, pva[tid], 0, 1, 0);
    __syncthreads();

    int sweeps = 0, converged = 0, floor_hit = 0;
    long long rotations = 0;
    const double lim2 = tol * tol * fro2;
    double off2 = 0.0;
    int64_t g = 0;

    // Rows T_k, B_k by R_k^T, then columns T_l, B_l by R_l, in the tangent
    // form c (x - t y), the two cosines applied at the end.
    auto rot2 = [](float4 x, float tk, float ckc, float tl, float clc) -> float4 {
        const float u0 = fmaf(-tk, x.z, x.x), u1 = fmaf(-tk, x.w, x.y);
        const float u2 = fmaf(tk, x.x, x.z), u3 = fmaf(tk, x.y, x.w);
        const float cc = ckc * clc;
        return make_float4(cc * fmaf(-tl, u1, u0), cc * fmaf(tl, u0, u1), cc * fmaf(-tl, u3, u2),
                           cc * fmaf(tl, u2, u3));
    };
    auto pick = [](float4 z, int c) -> float { return c == 0 ? z.x : (c == 1 ? z.y : (c == 2 ? z.z : z.w)); };

    while (!failed) {
        off2 = offnorm2();
        if (off2 <= lim2) { converged = 1; break; }
        if (sweeps >= max_sweeps) break;

        int cnt = 0;
        for (int sIn = 0; sIn < n - 1; ++sIn, ++g) {
            const int par = (int)(g & 1);
            const float2 *cs = csb[par];
            float4 z[L];
            if (len > 0) {
                const float2 ck = cs[gk];
                const float tk = gsr * ck.x;
                const float4 *src = &blk[gsrc];
                const float2 *csl = &cs[l0];
#pragma unroll
                for (int q = 0; q < L; ++q) {
                    const float2 cl = csl[q];
                    z[q] = rot2(src[q], tk, ck.y, gsc * cl.x, cl.y);
                }
            }
            float4 zs = make_float4(0.f, 0.f, 0.f, 0.f);
            if (has_sp) {
                const float2 ck = cs[sk], cl = cs[sl];
                zs = rot2(blk[ssrc], ssr * ck.x, ck.y, ssc * cl.x, cl.y);
            }
            __syncthreads();
            if (len > 0) {
#pragma unroll
                for (int q = 0; q < L; ++q) {
                    if (q < len) {
                        Af[gd[0] + 4 * q] = z[q].x;
                        Af[gd[1] + 4 * q] = z[q].y;
                        Af[gd[2] + 4 * q] = z[q].z;
                        Af[gd[3] + 4 * q] = z[q].w;
                    }
                }
            }
            if (has_sp) {
                if (sd[0] >= 0) Af[sd[0]] = zs.x;
                if (sd[1] >= 0) Af[sd[1]] = zs.y;
                if (sd[2] >= 0) Af[sd[2]] = zs.z;
                if (sd[3] >= 0) Af[sd[3]] = zs.w;
                // The next step's rotation of the pivot this block produced.
                if (mine0 >= 0) {
                    const float pv = pick(zs, mc0);
                    pva[mine0] = pv;
                    rotate(mine0, pv, par ^ 1, par, par ^ 1);
                }
                if (mine1 >= 0) {
                    const float pv = pick(zs, mc1);
                    pva[mine1] = pv;
                    rotate(mine1, pv, par ^ 1, par, par ^ 1);
                }
            }
            // The last P threads (the waves with the least work in a step)
            // log the step's rotations, so that no global store and no wait
            // for one sits in the waves on the step's critical path.
            if (tid >= kJThreads - P) {
                const int j = tid - (kJThreads - P);
                const float2 tc = cs[j];
                cnt += tc.x != 0.f;
                const float2 e = make_float2(tc.y, tc.x * tc.y);
                if (kFollow) log_store(&rlog[g * P + j], e);
                else rlog[g * P + j] = e;
            }
            if (tid < P) {
                const float pv = pvb[par][tid];
                if (pcode >= 0) {
                    Af[pcode] = pv;
                } else {
                    pva[-1 - pcode] = pv;
                    rotate(-1 - pcode, pv, par ^ 1, par, par ^ 1);
                }
            }
            __syncthreads();
        }
        ++sweeps;
        const int applied = block_sum_i(cnt, redi);
        rotations += applied;
        if (applied == 0) { converged = 1; floor_hit = 1; break; }
    }

    if (kFollow) {
        // End marks from step g to the end of its batch.
        const int64_t ends = (g / kLogBatch + 1) * kLogBatch - g;
        for (int64_t t = tid; t < ends * P; t += kJThreads) log_store(&rlog[g * P + t], make_float2(kLogEnd, 0.f));
    }
    if (!converged || floor_hit || failed) off2 = offnorm2();
    const int fin = (int)(g & 1);
    for (int x = tid; x < n; x += kJThreads) lam_u[S.phys(x)] = failed ? (double)NAN : dg[fin][x];
    if (tid == 0) {
        info->sweeps = sweeps;
        info->converged = converged;
        info->nonfinite = failed ? 1 : 0;
        info->floor_hit = floor_hit;
        info->off_rel = failed ? (double)NAN : (fro2 > 0.0 ? sqrt(off2 / fro2) : 0.0);
        info->rotations = rotations;
        info->steps = (int32_t)g;
        info->n_bands = m;
    }
}

template <int L>
__global__ __launch_bounds__(kJThreads) void jacobi_kernel(const float *__restrict__ C, int m, int n, double tol,
                                                           int max_sweeps, int fp64_angles,
                                                           double *__restrict__ lam_u, float2 *__restrict__ rlog,
                                                           pca_info *__restrict__ info)
{
    jacobi_body<L, false>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info);
}

constexpr int kReplayThreads = 512;
constexpr int kReplayMaxRows = 8;
constexpr int kReplayBatch = 16;
constexpr int kReplayPre = (kReplayBatch * kMaxP + kReplayThreads - 1) / kReplayThreads;

// Rows r0 .. r0+R-1 of the eigenvector matrix, in slot coordinates,
// double-buffered: thread (r, k) rotates columns (T_k, B_k) of row r and
// writes them to their permuted places, one barrier per step.
__device__ __forceinline__ void vreplay_body(int n, int rows, const float2 *__restrict__ rlog,
                                    const pca_info *__restrict__ info, float *__restrict__ VuT, int wg)
{
    __shared__ float vb[2][kReplayMaxRows][256];
    __shared__ float2 lcs[2][kReplayBatch][kMaxP];
    Slots S;
    S.init(n, nullptr, nullptr);
    const int P = S.P;
    const int tid = threadIdx.x;
    const int r0 = wg * rows;
    const int nsteps = info->steps;
    const int per = kReplayBatch * P;

    for (int t = tid; t < rows * n; t += kReplayThreads) {
        const int r = t / n, x = t - (t / n) * n;
        vb[0][r][x] = (S.phys(x) == r0 + r) ? 1.f : 0.f;
    }
    for (int t = tid; t < per; t += kReplayThreads) {
        const int gg = t / P, k = t - (t / P) * P;
        lcs[0][gg][k] = gg < nsteps ? rlog[(int64_t)gg * P + k] : make_float2(1.f, 0.f);
    }
    __syncthreads();

    const int tr = tid / P, tk = tid - (tid / P) * P;
    const bool has = tid < rows * P;
    const int nT = S.next(tk), nB = S.next(P + tk);
    const int nbatch = (nsteps + kReplayBatch - 1) / kReplayBatch;
    for (int bt = 0; bt < nbatch; ++bt) {
        float2 pre[kReplayPre];
#pragma unroll
        for (int q = 0; q < kReplayPre; ++q) {
            const int t = tid + q * kReplayThreads;
            pre[q] = make_float2(1.f, 0.f);
            if (t < per) {
                const int64_t gg = (int64_t)(bt + 1) * kReplayBatch + t / P;
                if (gg < nsteps) pre[q] = rlog[gg * P + (t - (t / P) * P)];
            }
        }
        const int cur = bt & 1;
        for (int gg = 0; gg < kReplayBatch; ++gg) {
            const int g = bt * kReplayBatch + gg;
            if (g >= nsteps) break;
            const int vin = g & 1;
            if (has) {
                const float2 cs = lcs[cur][gg][tk];
                const float vT = vb[vin][tr][tk], vB = vb[vin][tr][P + tk];
                vb[vin ^ 1][tr][nT] = cs.x * vT - cs.y * vB;
                vb[vin ^ 1][tr][nB] = cs.y * vT + cs.x * vB;
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < kReplayPre; ++q) {
            const int t = tid + q * kReplayThreads;
            if (t < per) lcs[cur ^ 1][t / P][t - (t / P) * P] = pre[q];
        }
        __syncthreads();
    }
    const int fin = nsteps & 1;
    for (int t = tid; t < rows * n; t += kReplayThreads) {
        const int r = t / n, x = t - (t / n) * n;
        if (r0 + r < n) VuT[(int64_t)S.phys(x) * n + r0 + r] = vb[fin][r][x];
    }
}

__global__ __launch_bounds__(kReplayThreads) void vreplay_kernel(int n, int rows, const float2 *__restrict__ rlog,
                                                                  const pca_info *__restrict__ info,
                                                                  float *__restrict__ VuT)
{
    vreplay_body(n, rows, rlog, info, VuT, (int)blockIdx.x);
}

constexpr int kFollowSpins = 1 << 19;   // polls of about 1 us on one entry before giving up
// The followers' bound is divided by 2^g_wait_shift (0 unless a test of the
// failure handling shortens it: pca_set_wait_shift).
__device__ int g_wait_shift = 0;

// Rows of E replayed beside the Jacobi workgroup (workgroup wg + 1 of the
// launch): rows r0 .. r0+rows-1, in slot coordinates, double-buffered in the
// LDS the Jacobi workgroup uses for its matrix; the log is read kLogBatch
// steps at a time.
__device__ __forceinline__ void follow_body(int n, int rows, const float2 *__restrict__ rlog,
                                            float *__restrict__ VuT, int wg)
{
    float *vb = reinterpret_cast<float *>(jac_blk);                     // [2][kFollowMaxRows][256]
    float2 *lcs = reinterpret_cast<float2 *>(vb + 2 * kFollowMaxRows * 256);   // [kLogBatch][kMaxP]
    __shared__ int st_fail, st_steps;
    Slots S;
    S.init(n, nullptr, nullptr);
    const int P = S.P;
    const int tid = threadIdx.x;
    const int r0 = wg * rows;
    const int tasks = rows * P;

    for (int t = tid; t < rows * n; t += kJThreads) {
        const int r = t / n, x = t - (t / n) * n;
        vb[r * 256 + x] = (S.phys(x) == r0 + r) ? 1.f : 0.f;
    }
    if (tid == 0) st_fail = 0;
    __syncthreads();
    int64_t done_steps = 0;
    int fail = 0;
    const int spin_lim = kFollowSpins >> (g_wait_shift < 0 ? 0 : (g_wait_shift > 19 ? 19 : g_wait_shift));
    while (true) {
        // Wait for every entry of the batch (bounded), then count its steps
        // before the first end mark.
        int bad = 0;
        for (int t = tid; t < kLogBatch * P; t += kJThreads) {
            const float2 *src = &rlog[done_steps * P + t];
            float2 e = log_load(src);
            int spins = 0;
            while (__float_as_uint(e.x) == 0u && __float_as_uint(e.y) == 0u) {
                if (++spins > spin_lim) { bad = 1; break; }
                __builtin_amdgcn_s_sleep(32);
                e = log_load(src);
            }
            lcs[t] = e;
        }
        if (bad) atomicOr(&st_fail, 1);
        if (tid == 0) st_steps = kLogBatch;
        __syncthreads();
        if (tid < kLogBatch && lcs[tid * P].x == kLogEnd) atomicMin(&st_steps, tid);
        __syncthreads();
        fail = st_fail;
        const int nb = st_steps;
        if (fail) break;
        for (int gg = 0; gg < nb; ++gg) {
            const int vin = (int)((done_steps + gg) & 1);
            const float *src = vb + vin * (kFollowMaxRows * 256);
            float *dst = vb + (vin ^ 1) * (kFollowMaxRows * 256);
            for (int t = tid; t < tasks; t += kJThreads) {
                const int r = t / P, k = t - (t / P) * P;
                const float2 cs = lcs[gg * P + k];
                const float vT = src[r * 256 + k], vB = src[r * 256 + P + k];
                dst[r * 256 + S.next(k)] = cs.x * vT - cs.y * vB;
                dst[r * 256 + S.next(P + k)] = cs.y * vT + cs.x * vB;
            }
            __syncthreads();
        }
        done_steps += nb;
        if (nb < kLogBatch) break;
        __syncthreads();   // lcs is rewritten by the next batch
    }
    const float *fin = vb + (int)(done_steps & 1) * (kFollowMaxRows * 256);
    for (int t = tid; t < rows * n; t += kJThreads) {
        const int r = t / n, x = t - (t / n) * n;
        if (r0 + r < n) VuT[(int64_t)S.phys(x) * n + r0 + r] = fail ? (float)NAN : fin[r * 256 + x];
    }
}

template <int L>
__global__ __launch_bounds__(kJThreads) void jacobi_follow_kernel(const float *__restrict__ C, int m, int n,
                                                                  double tol, int max_sweeps, int fp64_angles,
                                                                  double *__restrict__ lam_u,
                                                                  float2 *__restrict__ rlog,
                                                                  pca_info *__restrict__ info, int rows,
                                                                  float *__restrict__ VuT)
{
    if (blockIdx.x == 0)
        jacobi_body<L, true>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info);
    else
        follow_body(n, rows, rlog, VuT, (int)blockIdx.x - 1);
}

// One wave per output column: rank by counting (stable, descending), then the
// sign from the column's largest-magnitude entry (lowest row on ties).
__device__ __forceinline__ void sort_sign_body(int m, int n, const double *__restrict__ lam_u, const float *__restrict__ VuT,
                                      const pca_info *__restrict__ info_ws, float *__restrict__ eigvals,
                                      float *__restrict__ V, pca_info *__restrict__ info_out, int wg)
{
    __shared__ int perm[256];
    __shared__ double lam[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = wg * 4 + wave;
    if (info_ws->nonfinite) {
        if (wg == 0) for (int i = tid; i < m; i += 256) eigvals[i] = NAN;
        if (c < m) for (int r = lane; r < m; r += 64) V[(int64_t)r * m + c] = NAN;
        if (wg == 0 && tid == 0 && info_out) *info_out = *info_ws;
        return;
    }
    if (tid < m) lam[tid] = lam_u[tid];
    __syncthreads();
    if (tid < m) {
        const double x = lam[tid];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double y = lam[j];
            rank += (y > x) || (y == x && j < tid);
        }
        perm[rank] = tid;
        if (wg == 0) eigvals[rank] = (float)x;
    }
    __syncthreads();
    if (c < m) {
        const int j = perm[c];
        float v[4];
        float best = -1.f;
        int bidx = 1 << 30;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = lane + 64 * i;
            v[i] = r < m ? VuT[(int64_t)j * n + r] : 0.f;
            if (r < m && fabsf(v[i]) > best) { best = fabsf(v[i]); bidx = r; }
        }
        float bval = 0.f;
        for (int i = 0; i < 4; ++i) if (lane + 64 * i == bidx) bval = v[i];
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bidx, off, 64);
            const float ov = __shfl_xor(bval, off, 64);
            if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; bval = ov; }
        }
        const float sgn = bval < 0.f ? -1.f : 1.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = lane + 64 * i;
            if (r < m) V[(int64_t)r * m + c] = sgn * v[i];
        }
    }
    if (wg == 0 && tid == 0 && info_out) *info_out = *info_ws;
}

__global__ __launch_bounds__(256) void sort_sign_kernel(int m, int n, const double *__restrict__ lam_u,
                                                        const float *__restrict__ VuT,
                                                        const pca_info *__restrict__ info_ws,
                                                        float *__restrict__ eigvals, float *__restrict__ V,
                                                        pca_info *__restrict__ info_out)
{
    sort_sign_body(m, n, lam_u, VuT, info_ws, eigvals, V, info_out, (int)blockIdx.x);
}

// ---- batched form ------------------------------------------------------------
constexpr int kBatchL = 9;    // segment length that fits every band count (1024 threads)

__device__ inline const BatchCube *jbatch_table(const char *ws)
{
    return reinterpret_cast<const BatchCube *>(ws + sizeof(BatchHeader));
}

template <int64_t BatchCube::*W>
__device__ inline int jbatch_find(const BatchCube *t, int nc, int64_t item)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (t[mid].*W <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Zeroes every cube's whole rotation log before the batched Jacobi launch
// (the followers read the logs while they are written, and a batch's
// workspace layout, so where each log sits, changes with the batch and the
// tile sizes; no state is carried from call to call).
__global__ __launch_bounds__(256) void log_clear_batched_kernel(const char *ws, int nc, int max_sweeps)
{
    const BatchCube *t = jbatch_table(ws);
    for (int c = 0; c < nc; ++c) {
        const BatchCube &cb = t[c];
        const JacPlan jp = jac_plan(cb.m, max_sweeps);
        const int64_t n4 = jp.log_steps * jp.npairs / 2;   // two entries per 16 bytes (log_steps is a multiple of 16)
        float4 *p = reinterpret_cast<float4 *>(cb.rlog);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Workgroups 0 .. nc-1: the Jacobi sweeps of cube blockIdx.x (one CU each);
// the rest: follower workgroups replaying the rotation logs as they are
// written (cube order, so the widest cubes' followers are dispatched first;
// followers that find no free CU start later and replay a finished log).
__global__ __launch_bounds__(kJThreads) void jacobi_batched_kernel(const char *ws, int nc, double tol, int max_sweeps,
                                                                   int fp64_angles)
{
    const BatchCube *t = jbatch_table(ws);
    if ((int)blockIdx.x < nc) {
        const BatchCube &cb = t[blockIdx.x];
        jacobi_body<kBatchL, true>(cb.C, cb.m, cb.m + (cb.m & 1), tol, max_sweeps, fp64_angles, cb.lam_u, cb.rlog,
                                   cb.info_ws);
    } else {
        const int64_t item = (int64_t)blockIdx.x - nc;
        const BatchCube &cb = t[jbatch_find<&BatchCube::w_rep>(t, nc, item)];
        follow_body(cb.m + (cb.m & 1), cb.rows, cb.rlog, cb.Vu, (int)(item - cb.w_rep));
    }
}

__global__ __launch_bounds__(256) void sort_sign_batched_kernel(const char *ws, int nc)
{
    const BatchCube *t = jbatch_table(ws);
    const int64_t item = blockIdx.x;
    const BatchCube &cb = t[jbatch_find<&BatchCube::w_sort>(t, nc, item)];
    sort_sign_body(cb.m, cb.m + (cb.m & 1), cb.lam_u, cb.Vu, cb.info_ws, cb.eigvals, cb.V, cb.info,
                   (int)(item - cb.w_sort));
}


__global__ __launch_bounds__(256) void log_clear_kernel(float4 *p, int64_t n4)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int L>
void launch_jac(const float *C, int m, int n, double tol, int max_sweeps, int fp64_angles, double *lam_u,
                float2 *rlog, pca_info *info_ws, int overlap, float *Vu, hipStream_t st)
{
    if (overlap) {
        // The followers read the log while it is written and take the first
        // non-zero value of an entry as final: clear the whole log first, so
        // the call depends on nothing a previous call left in the workspace.
        const JacPlan jp = jac_plan(m, max_sweeps);
        const int64_t n4 = jp.log_steps * jp.npairs / 2;   // two entries per 16 bytes (log_steps is a multiple of 16)
        const unsigned nclr = (unsigned)((n4 + 255) / 256 < 1024 ? (n4 + 255) / 256 : 1024);
        hipLaunchKernelGGL(log_clear_kernel, dim3(nclr), dim3(256), 0, st, reinterpret_cast<float4 *>(rlog), n4);
        const int rows = follow_rows(n);
        const unsigned nf = (unsigned)((n + rows - 1) / rows);
        hipLaunchKernelGGL(jacobi_follow_kernel<L>, dim3(1 + nf), dim3(kJThreads), 0, st, C, m, n, tol, max_sweeps,
                           fp64_angles, lam_u, rlog, info_ws, rows, Vu);
    } else {
        hipLaunchKernelGGL(jacobi_kernel<L>, dim3(1), dim3(kJThreads), 0, st, C, m, n, tol, max_sweeps, fp64_angles,
                           lam_u, rlog, info_ws);
    }
}

// Generic segments of length at most L for P pairs.
int jac_segments(int P, int L)
{
    int s = 0;
    for (int k = 0; k < P; ++k) s += (generic_len(P, k) + L - 1) / L;
    return s;
}

}  // namespace

hipError_t launch_jacobi(const float *C, int m, double tol, int max_sweeps, int fp64_angles, int overlap,
                         const JacPlan &plan, double *lam_u, float2 *rlog, float *Vu, pca_info *info_ws,
                         float *eigvals, float *V, pca_info *info_out, hipStream_t st)
{
    const int n = plan.me;
    const int P = plan.npairs;
    // Shortest segment length (odd, so that the lanes of a wave hit distinct
    // LDS banks) that gives every segment its own thread; 9 suffices for 128
    // pairs with 1024 threads.
    int L = 1;
    while (L < kBatchL && jac_segments(P, L) > kJThreads) L += 2;
    switch (L) {
    case 1: launch_jac<1>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, overlap, Vu, st); break;
    case 3: launch_jac<3>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, overlap, Vu, st); break;
    case 5: launch_jac<5>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, overlap, Vu, st); break;
    case 7: launch_jac<7>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, overlap, Vu, st); break;
    default: launch_jac<kBatchL>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, overlap, Vu, st); break;
    }
    if (!overlap) {
        const int rows = replay_rows(n);
        const unsigned nwg = (unsigned)((n + rows - 1) / rows);
        hipLaunchKernelGGL(vreplay_kernel, dim3(nwg), dim3(kReplayThreads), 0, st, n, rows, rlog,
                           (const pca_info *)info_ws, Vu);
    }
    hipLaunchKernelGGL(sort_sign_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, m, n,
                       (const double *)lam_u, (const float *)Vu, (const pca_info *)info_ws, eigvals, V, info_out);
    return hipGetLastError();
}

hipError_t launch_sort_sign(int m, int n, const double *lam_u, const float *Vu, const pca_info *info_ws,
                            float *eigvals, float *V, pca_info *info_out, hipStream_t st)
{
    hipLaunchKernelGGL(sort_sign_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, m, n, lam_u, Vu, info_ws,
                       eigvals, V, info_out);
    return hipGetLastError();
}

hipError_t launch_jacobi_batched(const char *ws, const int64_t total[6], int n_cubes, double tol, int max_sweeps,
                                 int fp64_angles, hipStream_t st)
{
    hipLaunchKernelGGL(log_clear_batched_kernel, dim3(1024), dim3(256), 0, st, ws, n_cubes, max_sweeps);
    hipLaunchKernelGGL(jacobi_batched_kernel, dim3((unsigned)(n_cubes + total[3])), dim3(kJThreads), 0, st, ws,
                       n_cubes, tol, max_sweeps, fp64_angles);
    hipLaunchKernelGGL(sort_sign_batched_kernel, dim3((unsigned)total[4]), dim3(256), 0, st, ws, n_cubes);
    return hipGetLastError();
}

hipError_t set_wait_shift_one_cu(int shift)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(g_wait_shift), &shift, sizeof(int));
}

}  // namespace pca

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
// thread's source and destination LDS addresses are computed once. Storage
// (LDS, float32): T-T and B-B off-diagonal entries as packed strict upper
// triangles, T-B entries as a full (n/2) x (n/2 + 1) array (T_k-B_k are the
// pivots); the diagonal is float64 in a separate double-buffered array.
// After n - 1 steps the slots are back in their initial places.
//
// jacobi_kernel (one workgroup, one CU). A step:
//   a. every thread rotates its 2x2 blocks (pairs k < l): rows by R_k^T,
//      columns by R_l -- the row and column updates of C_k = P^T C P,
//      equation (8), for all pairs of the step at once;
//   b. barrier; the rotated entries are written to their permuted places.
//      Whoever writes a pivot of the next step also computes that pivot's
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
// sort_sign_kernel: eigenvalues from the diagonal, sorted in descending order
// (stable), eigenvector columns permuted to match (Code 4.4.3), and the sign
// of each column fixed so its largest-magnitude entry is positive.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace pca {

namespace {

constexpr int kJThreads = 512;
constexpr int kMaxP = 128;
constexpr int kMaxSlotFloats = 128 * 127 + 128 * 129;
constexpr int kLoadPerThread = 64;                       // loads in flight per pass
constexpr double kFloorRel2 = 3.552713678800501e-15;     // (2^-24)^2

struct Slots {
    int P, n, PT, baseBB, baseTB;

    __device__ void init(int n_) {
        n = n_;
        P = n_ / 2;
        PT = P + 1;
        baseBB = P * (P - 1) / 2;
        baseTB = P * (P - 1);
    }
    __device__ int total() const { return baseTB + P * PT; }
    __device__ int tt(int a, int b) const { return a * (2 * P - a - 1) / 2 + (b - a - 1); }   // a < b
    __device__ int bb(int a, int b) const { return baseBB + tt(a, b); }
    __device__ int tb(int t, int b) const { return baseTB + t * PT + b; }
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
    // LDS index of the off-diagonal entry (x, y), x != y.
    __device__ int addr(int x, int y) const {
        const bool xt = x < P, yt = y < P;
        if (xt && yt) return x < y ? tt(x, y) : tt(y, x);
        if (!xt && !yt) {
            const int a = x - P, b = y - P;
            return a < b ? bb(a, b) : bb(b, a);
        }
        return xt ? tb(x, y - P) : tb(y, x - P);
    }
    // Pair whose pivot (T_k, B_k) the entry (x, y) is, or -1.
    __device__ int pivot_of(int x, int y) const {
        if (x < P && y == x + P) return x;
        if (y < P && x == y + P) return y;
        return -1;
    }
    // Slot of physical index i at the start of a sweep, and back.
    __device__ int slot_of(int i) const { return i < P ? i : P + (n - 1 - i); }
    __device__ int phys(int x) const { return x < P ? x : n - 1 - (x - P); }
};

// Rotation of a pivot pair, equations (2)-(5) with (7):
//   theta = (a_qq - a_pp) / (2 a_pq), t = sgn(theta) / (|theta| + sqrt(1 + theta^2))
// evaluated as t = sgn(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp
// (the same number), cos = 1/sqrt(1 + t^2), sin = t cos. Skipped (cos = 1,
// sin = 0) when |a_pq| is at the float32 rounding floor.
__device__ inline void rotation(double app, double aqq, float apq, double floor_abs, int fp64, float2 &cs,
                                double &dT, double &dB, float &pv)
{
    const double a = (double)apq;
    const double ad = fabs(a);
    if (apq != 0.f && ad > floor_abs && ad * ad > kFloorRel2 * fabs(app * aqq)) {
        double t;
        if (fp64) {
            const double d = aqq - app;
            const double r = sqrt(d * d + 4.0 * a * a);
            t = (d >= 0.0 ? 2.0 * a : -2.0 * a) / (fabs(d) + r);
            const double c = rsqrt(1.0 + t * t);
            cs = make_float2((float)c, (float)(t * c));
        } else {
            const float df = (float)aqq - (float)app;
            const float rf = sqrtf(df * df + 4.f * apq * apq);
            const float tf = (df >= 0.f ? 2.f * apq : -2.f * apq) / (fabsf(df) + rf);
            const float c = 1.f / sqrtf(1.f + tf * tf);
            cs = make_float2(c, tf * c);
            t = tf;
        }
        dT = app - t * a;
        dB = aqq + t * a;
        pv = 0.f;
    } else {
        cs = make_float2(1.f, 0.f);
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

template <int MAXB>
__global__ __launch_bounds__(kJThreads) void jacobi_kernel(const float *__restrict__ C, int m, int n, double tol,
                                                           int max_sweeps, int fp64_angles,
                                                           double *__restrict__ lam_u, float2 *__restrict__ rlog,
                                                           pca_info *__restrict__ info)
{
    __shared__ float A[kMaxSlotFloats];
    __shared__ double dg[2][256];
    __shared__ float2 csb[2][kMaxP];
    __shared__ float pvb[2][kMaxP];
    __shared__ double redd[16];
    __shared__ int redi[16];
    __shared__ int bad;

    Slots S;
    S.init(n);
    const int P = S.P;
    const int tid = threadIdx.x;
    const int total = S.total();

    if (tid == 0) bad = 0;
    for (int e = tid; e < total; e += kJThreads) A[e] = 0.f;
    for (int i = tid; i < 256; i += kJThreads) { dg[0][i] = 0.0; dg[1][i] = 0.0; }
    __syncthreads();

    // Load the upper triangle of C into slot coordinates (each pass issues all
    // its global loads before any LDS store).
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
                        if (i == j) dg[0][si] = (double)tmp[q];
                        else A[S.addr(si, sj)] = tmp[q];
                    }
                }
            }
        }
        if (nonfin) atomicOr(&bad, 1);
    }
    __syncthreads();

    double fro2;
    {
        double part = 0.0;
        for (int e = tid; e < total; e += kJThreads) part += 2.0 * (double)A[e] * (double)A[e];
        for (int i = tid; i < n; i += kJThreads) part += dg[0][i] * dg[0][i];
        fro2 = block_sum_d(part, redd);
    }
    const bool nonfinite = bad != 0;
    const double floor_abs = 5.9604644775390625e-08 * sqrt(fro2) / (double)m;

    // This thread's blocks (k, l), k < l, of the pair grid: source and
    // destination LDS indices of the entries (T_k,T_l), (T_k,B_l), (B_k,T_l),
    // (B_k,B_l), and which of them become pivots of the next step.
    const int nblocks = P * (P - 1) / 2;
    int bk[MAXB], bl[MAXB], be[MAXB], sTB[MAXB], sBT[MAXB], dst[MAXB][4];
    // Pairs whose next pivot this thread writes (at most two for any n <= 256
    // with 512 threads; a third would be reported as a failure).
    int piv0 = -1, piv1 = -1, piv_over = 0;
    int myn = 0;
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        int e = tid + q * kJThreads;
        bk[q] = bl[q] = be[q] = sTB[q] = sBT[q] = 0;
        dst[q][0] = dst[q][1] = dst[q][2] = dst[q][3] = 0;
        if (e < nblocks) {
            be[q] = e;
            int k = 0;
            while (e >= P - 1 - k) { e -= P - 1 - k; ++k; }
            const int l = k + 1 + e;
            bk[q] = k;
            bl[q] = l;
            sTB[q] = S.tb(k, l);
            sBT[q] = S.tb(l, k);
            const int xs[2] = {k, P + k}, ys[2] = {l, P + l};
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int nx = S.next(xs[a]), ny = S.next(ys[b]);
                    dst[q][2 * a + b] = S.addr(nx, ny);
                    const int kp = S.pivot_of(nx, ny);
                    if (kp >= 0) {
                        if (piv0 < 0) piv0 = kp;
                        else if (piv1 < 0) piv1 = kp;
                        else piv_over = 1;
                    }
                }
            }
            myn = q + 1;
        }
    }
    // Thread k < P moves pivot k after each step.
    int pdst = 0, pdst_pivot = -1;
    if (tid < P) {
        const int nx = S.next(tid), ny = S.next(P + tid);
        pdst = S.addr(nx, ny);
        pdst_pivot = S.pivot_of(nx, ny);
    }

    if (piv_over) atomicOr(&bad, 2);
    __syncthreads();
    const bool failed = nonfinite || bad != 0;

    // Rotation of pair k for the step whose diagonal is in dg[src]; writes
    // its (cos, sin) and moved pivot into slot `par`, the rotated diagonal
    // (already permuted) into dg[dsto].
    auto rotate = [&](int k, float apq, int src, int dsto, int par) {
        float2 cs;
        double dT, dB;
        float pv;
        rotation(dg[src][k], dg[src][P + k], apq, floor_abs, fp64_angles, cs, dT, dB, pv);
        csb[par][k] = cs;
        pvb[par][k] = pv;
        dg[dsto][S.next(k)] = dT;
        dg[dsto][S.next(P + k)] = dB;
    };

    // Rotations of step 0.
    if (tid < P && !failed) rotate(tid, A[S.tb(tid, tid)], 0, 1, 0);
    __syncthreads();

    int sweeps = 0, converged = 0, floor_hit = 0;
    long long rotations = 0;
    const double lim2 = tol * tol * fro2;
    double off2 = 0.0;
    int64_t g = 0;

    while (!failed) {
        {
            double part = 0.0;
            for (int e = tid; e < total; e += kJThreads) part += (double)A[e] * (double)A[e];
            off2 = 2.0 * block_sum_d(part, redd);
        }
        if (off2 <= lim2) { converged = 1; break; }
        if (sweeps >= max_sweeps) break;

        int cnt = 0;
        for (int sIn = 0; sIn < n - 1; ++sIn, ++g) {
            const int par = (int)(g & 1);
            float z[MAXB][4];
#pragma unroll
            for (int q = 0; q < MAXB; ++q) {
                if (q < myn) {
                    const float2 ck = csb[par][bk[q]], cl = csb[par][bl[q]];
                    const int e = be[q];
                    const float x0 = A[e], x1 = A[sTB[q]], x2 = A[sBT[q]], x3 = A[S.baseBB + e];
                    // Rows T_k, B_k by R_k^T, then columns T_l, B_l by R_l.
                    const float y0 = ck.x * x0 - ck.y * x2, y1 = ck.x * x1 - ck.y * x3;
                    const float y2 = ck.y * x0 + ck.x * x2, y3 = ck.y * x1 + ck.x * x3;
                    z[q][0] = y0 * cl.x - y1 * cl.y;
                    z[q][1] = y0 * cl.y + y1 * cl.x;
                    z[q][2] = y2 * cl.x - y3 * cl.y;
                    z[q][3] = y2 * cl.y + y3 * cl.x;
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < MAXB; ++q) {
                if (q < myn) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) A[dst[q][c]] = z[q][c];
                }
            }
            // Next step's rotations of the pivots this thread just wrote.
            if (piv0 >= 0) rotate(piv0, A[S.tb(piv0, piv0)], par ^ 1, par, par ^ 1);
            if (piv1 >= 0) rotate(piv1, A[S.tb(piv1, piv1)], par ^ 1, par, par ^ 1);
            if (tid < P) {
                const float2 c = csb[par][tid];
                cnt += c.y != 0.f;
                rlog[g * P + tid] = c;
                const float pv = pvb[par][tid];
                A[pdst] = pv;
                if (pdst_pivot >= 0) rotate(pdst_pivot, pv, par ^ 1, par, par ^ 1);
            }
            __syncthreads();
        }
        ++sweeps;
        const int applied = block_sum_i(cnt, redi);
        rotations += applied;
        if (applied == 0) { converged = 1; floor_hit = 1; break; }
    }

    if (!converged || floor_hit || failed) {
        double part = 0.0;
        for (int e = tid; e < total; e += kJThreads) part += (double)A[e] * (double)A[e];
        off2 = 2.0 * block_sum_d(part, redd);
    }
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

constexpr int kReplayThreads = 512;
constexpr int kReplayMaxRows = 8;
constexpr int kReplayBatch = 16;
constexpr int kReplayPre = (kReplayBatch * kMaxP + kReplayThreads - 1) / kReplayThreads;

// Rows r0 .. r0+R-1 of the eigenvector matrix, in slot coordinates,
// double-buffered: thread (r, k) rotates columns (T_k, B_k) of row r and
// writes them to their permuted places, one barrier per step.
__global__ __launch_bounds__(kReplayThreads) void vreplay_kernel(int n, int rows, const float2 *__restrict__ rlog,
                                                                  const pca_info *__restrict__ info,
                                                                  float *__restrict__ VuT)
{
    __shared__ float vb[2][kReplayMaxRows][256];
    __shared__ float2 lcs[2][kReplayBatch][kMaxP];
    Slots S;
    S.init(n);
    const int P = S.P;
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * rows;
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

// One wave per output column: rank by counting (stable, descending), then the
// sign from the column's largest-magnitude entry (lowest row on ties).
__global__ __launch_bounds__(256) void sort_sign_kernel(int m, int n, const double *__restrict__ lam_u,
                                                        const float *__restrict__ VuT,
                                                        const pca_info *__restrict__ info_ws,
                                                        float *__restrict__ eigvals, float *__restrict__ V,
                                                        pca_info *__restrict__ info_out)
{
    __shared__ int perm[256];
    __shared__ double lam[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = blockIdx.x * 4 + wave;
    if (info_ws->nonfinite) {
        if (blockIdx.x == 0) for (int i = tid; i < m; i += 256) eigvals[i] = NAN;
        if (c < m) for (int r = lane; r < m; r += 64) V[(int64_t)r * m + c] = NAN;
        if (blockIdx.x == 0 && tid == 0 && info_out) *info_out = *info_ws;
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
        if (blockIdx.x == 0) eigvals[rank] = (float)x;
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
    if (blockIdx.x == 0 && tid == 0 && info_out) *info_out = *info_ws;
}

template <int MAXB>
void launch_jac(const float *C, int m, int n, double tol, int max_sweeps, int fp64_angles, double *lam_u,
                float2 *rlog, pca_info *info_ws, hipStream_t st)
{
    hipLaunchKernelGGL(jacobi_kernel<MAXB>, dim3(1), dim3(kJThreads), 0, st, C, m, n, tol, max_sweeps, fp64_angles,
                       lam_u, rlog, info_ws);
}

}  // namespace

JacPlan jac_plan(int m, int max_sweeps)
{
    JacPlan p;
    p.me = m + (m & 1);
    p.npairs = p.me / 2;
    p.log_steps = (int64_t)(max_sweeps > 0 ? max_sweeps : 0) * (p.me - 1);
    p.bytes_log = (size_t)(p.log_steps > 0 ? p.log_steps : 1) * p.npairs * sizeof(float2);
    p.bytes_lam = (size_t)p.me * sizeof(double);
    p.bytes_vu = (size_t)p.me * p.me * sizeof(float);
    p.bytes_info = sizeof(pca_info);
    return p;
}

hipError_t launch_jacobi(const float *C, int m, double tol, int max_sweeps, int fp64_angles, const JacPlan &plan,
                         double *lam_u, float2 *rlog, float *Vu, pca_info *info_ws, float *eigvals, float *V,
                         pca_info *info_out, hipStream_t st)
{
    const int n = plan.me;
    const int P = plan.npairs;
    const int nblocks = P * (P - 1) / 2;
    const int need = (nblocks + kJThreads - 1) / kJThreads;
    if (need <= 1) launch_jac<1>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, st);
    else if (need <= 2) launch_jac<2>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, st);
    else if (need <= 4) launch_jac<4>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, st);
    else if (need <= 8) launch_jac<8>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, st);
    else if (need <= 13) launch_jac<13>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, st);
    else launch_jac<16>(C, m, n, tol, max_sweeps, fp64_angles, lam_u, rlog, info_ws, st);
    int rows = kReplayThreads / P;
    if (rows > kReplayMaxRows) rows = kReplayMaxRows;
    const unsigned nwg = (unsigned)((n + rows - 1) / rows);
    hipLaunchKernelGGL(vreplay_kernel, dim3(nwg), dim3(kReplayThreads), 0, st, n, rows, rlog,
                       (const pca_info *)info_ws, Vu);
    hipLaunchKernelGGL(sort_sign_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, m, n,
                       (const double *)lam_u, (const float *)Vu, (const pca_info *)info_ws, eigvals, V, info_out);
    return hipGetLastError();
}

}  // namespace pca

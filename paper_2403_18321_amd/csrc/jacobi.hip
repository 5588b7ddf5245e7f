// Cyclic Jacobi eigendecomposition of the covariance (Section 2: equations
// (2)-(10) and the parallel-rotation property; the rotation count per sweep
// and the stop rule follow the same section).
//
// jacobi_kernel: one workgroup (1024 threads, one CU) holds the matrix in LDS:
// the strictly upper triangle packed in float32 and the diagonal in float64.
// Each parallel step takes n/2 disjoint pivot pairs from a round-robin
// tournament (n - 1 steps visit every pair once: one sweep). A step has two
// phases separated by workgroup barriers:
//   1. one thread per pair computes the rotation of equations (2)-(5) with the
//      generalised m of equation (7) (evaluated as t = sgn(theta) /
//      (|theta| + sqrt(1 + theta^2)), theta = 1/m, in float64 by default),
//      updates the pivot entries exactly (a_pp - t a_pq, a_qq + t a_pq, 0),
//      and appends (cos, sin) to the rotation log;
//   2. every 2x2 block of rows (p_k, q_k) x columns (p_l, q_l) is replaced by
//      R_k^T B R_l, i.e. the row and column updates of C_k = P^T C P
//      (equation (8)) for all pairs of the step at once.
// Before each sweep the off-diagonal norm is reduced in float64 across the
// workgroup; the iteration stops when it is <= tol ||C||_F, when a sweep
// applied no rotation, or after max_sweeps sweeps.
//
// vreplay_kernel: the eigenvector matrix E = P_1 P_2 ... P_K (equation (10))
// is rebuilt from the rotation log. Rows of E evolve independently under
// E <- E P, so many workgroups each replay the whole log on a few rows; this
// keeps the eigenvector work off the single-CU critical path.
//
// sort_sign_kernel: eigenvalues from the diagonal, sorted in descending order
// (stable), eigenvector columns permuted to match (Code 4.4.3), and the sign
// of each column fixed so its largest-magnitude entry is positive.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace pca {

namespace {

constexpr int kJacThreads = 1024;
constexpr int kMaxPairs = 128;
constexpr int kMaxOff = 256 * 255 / 2;
constexpr int kMaxBlocks = 8;                 // ceil(128 * 127 / 2 / 1024)
constexpr int kLoadPerThread = 64;            // 256 * 256 / 1024
constexpr double kFloorRel = 5.9604644775390625e-08;   // 2^-24

__device__ inline int rowbase(int i, int me) { return i * (2 * me - i - 1) / 2 - i - 1; }

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

__global__ __launch_bounds__(kJacThreads) void jacobi_kernel(
    const float *__restrict__ C, int m, int me, double tol, int max_sweeps, int fp64_angles,
    double *__restrict__ lam_u, float2 *__restrict__ rlog, pca_info *__restrict__ info)
{
    __shared__ float offd[kMaxOff];
    __shared__ double diag[256];
    __shared__ int4 pinfo[kMaxPairs];   // p, q, rowbase(p), rowbase(q)
    __shared__ float2 pcs[kMaxPairs];   // cos, sin (sin == 0: no rotation)
    __shared__ double redd[16];
    __shared__ int redi[16];
    __shared__ int bad;

    const int tid = threadIdx.x;
    const int P = me / 2;
    const int noff = me * (me - 1) / 2;

    if (tid == 0) bad = 0;
    for (int i = tid; i < me; i += kJacThreads) diag[i] = 0.0;
    for (int e = tid; e < noff; e += kJacThreads) offd[e] = 0.f;
    __syncthreads();

    // Load the upper triangle of C (all loads issued before any LDS store).
    {
        float tmp[kLoadPerThread];
        const int mm = m * m;
#pragma unroll
        for (int q = 0; q < kLoadPerThread; ++q) {
            const int e = tid + q * kJacThreads;
            tmp[q] = e < mm ? C[e] : 0.f;
        }
        int nonfin = 0;
#pragma unroll
        for (int q = 0; q < kLoadPerThread; ++q) {
            const int e = tid + q * kJacThreads;
            if (e < mm) {
                const int i = e / m, j = e - (e / m) * m;
                if (j >= i) {
                    if (!isfinite(tmp[q])) nonfin = 1;
                    if (j == i) diag[i] = (double)tmp[q];
                    else offd[rowbase(i, me) + j] = tmp[q];
                }
            }
        }
        if (nonfin) atomicOr(&bad, 1);
    }
    __syncthreads();

    double fro2 = 0.0;
    {
        double part = 0.0;
        for (int e = tid; e < noff; e += kJacThreads) part += 2.0 * (double)offd[e] * (double)offd[e];
        for (int i = tid; i < me; i += kJacThreads) part += diag[i] * diag[i];
        fro2 = block_sum_d(part, redd);
    }
    const bool nonfinite = bad != 0;
    const double floor_abs = kFloorRel * sqrt(fro2) / (double)m;

    // This thread's 2x2 blocks (k, l), k < l, of the pair-indexed matrix.
    int bk[kMaxBlocks], bl[kMaxBlocks];
    const int nblocks = P * (P - 1) / 2;
#pragma unroll
    for (int q = 0; q < kMaxBlocks; ++q) {
        int e = tid + q * kJacThreads;
        int k = 0;
        if (e < nblocks) {
            while (e >= P - 1 - k) { e -= P - 1 - k; ++k; }
            bk[q] = k;
            bl[q] = k + 1 + e;
        } else {
            bk[q] = -1;
            bl[q] = -1;
        }
    }

    int sweeps = 0, converged = 0, floor_hit = 0;
    long long rotations = 0;
    const double lim2 = tol * tol * fro2;
    double off2 = 0.0;
    int64_t g = 0;   // global step index (row of the rotation log)

    while (!nonfinite) {
        {
            double part = 0.0;
            for (int e = tid; e < noff; e += kJacThreads) part += (double)offd[e] * (double)offd[e];
            off2 = 2.0 * block_sum_d(part, redd);
        }
        if (off2 <= lim2) { converged = 1; break; }
        if (sweeps >= max_sweeps) break;

        int cnt = 0;
        for (int step = 0; step < me - 1; ++step, ++g) {
            if (tid < P) {
                int p, q;
                rr_pair(me, step, tid, p, q);
                const int rbp = rowbase(p, me), rbq = rowbase(q, me);
                const float apq = offd[rbp + q];
                const double app = diag[p], aqq = diag[q];
                const double ad = fabs((double)apq);
                float2 cs = make_float2(1.f, 0.f);
                if (apq != 0.f && ad > floor_abs && ad > kFloorRel * sqrt(fabs(app * aqq))) {
                    double t;
                    if (fp64_angles) {
                        const double theta = (aqq - app) / (2.0 * (double)apq);
                        t = fabs(theta) > 1e150 ? 0.5 / theta
                                                : (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                        const double c = 1.0 / sqrt(1.0 + t * t);
                        cs = make_float2((float)c, (float)(t * c));
                        diag[p] = app - t * (double)apq;
                        diag[q] = aqq + t * (double)apq;
                    } else {
                        const float theta = ((float)aqq - (float)app) / (2.f * apq);
                        const float tf = fabsf(theta) > 1e18f ? 0.5f / theta
                                                              : (theta >= 0.f ? 1.f : -1.f) / (fabsf(theta) + sqrtf(1.f + theta * theta));
                        const float c = 1.f / sqrtf(1.f + tf * tf);
                        cs = make_float2(c, tf * c);
                        diag[p] = (double)((float)app - tf * apq);
                        diag[q] = (double)((float)aqq + tf * apq);
                        t = tf;
                    }
                    offd[rbp + q] = 0.f;
                    ++cnt;
                }
                pinfo[tid] = make_int4(p, q, rbp, rbq);
                pcs[tid] = cs;
                rlog[g * P + tid] = cs;
            }
            __syncthreads();
#pragma unroll
            for (int bq = 0; bq < kMaxBlocks; ++bq) {
                const int k = bk[bq];
                if (k < 0) continue;
                const int l = bl[bq];
                const float2 ck = pcs[k], cl = pcs[l];
                if (ck.y == 0.f && cl.y == 0.f) continue;
                const int4 ik = pinfo[k], il = pinfo[l];
                // rows ik.x (p_k), ik.y (q_k); columns il.x (p_l), il.y (q_l)
                const int a11 = ik.x < il.x ? ik.z + il.x : il.z + ik.x;
                const int a12 = ik.x < il.y ? ik.z + il.y : il.w + ik.x;
                const int a21 = ik.y < il.x ? ik.w + il.x : il.z + ik.y;
                const int a22 = ik.y < il.y ? ik.w + il.y : il.w + ik.y;
                const float x11 = offd[a11], x12 = offd[a12], x21 = offd[a21], x22 = offd[a22];
                // Rows: new row p = c row p - s row q, new row q = s row p + c row q.
                const float y11 = ck.x * x11 - ck.y * x21, y12 = ck.x * x12 - ck.y * x22;
                const float y21 = ck.y * x11 + ck.x * x21, y22 = ck.y * x12 + ck.x * x22;
                // Columns: the same combination of columns p and q.
                offd[a11] = y11 * cl.x - y12 * cl.y;
                offd[a12] = y11 * cl.y + y12 * cl.x;
                offd[a21] = y21 * cl.x - y22 * cl.y;
                offd[a22] = y21 * cl.y + y22 * cl.x;
            }
            __syncthreads();
        }
        ++sweeps;
        const int applied = block_sum_i(cnt, redi);
        rotations += applied;
        if (applied == 0) { converged = 1; floor_hit = 1; break; }
    }

    if (!converged || floor_hit || nonfinite) {
        double part = 0.0;
        for (int e = tid; e < noff; e += kJacThreads) part += (double)offd[e] * (double)offd[e];
        off2 = 2.0 * block_sum_d(part, redd);
    }
    for (int i = tid; i < me; i += kJacThreads) lam_u[i] = nonfinite ? (double)NAN : diag[i];
    if (tid == 0) {
        info->sweeps = sweeps;
        info->converged = converged;
        info->nonfinite = nonfinite ? 1 : 0;
        info->floor_hit = floor_hit;
        info->off_rel = nonfinite ? (double)NAN : (fro2 > 0.0 ? sqrt(off2 / fro2) : 0.0);
        info->rotations = rotations;
        info->steps = (int32_t)g;
        info->n_bands = m;
    }
}

constexpr int kReplayRows = 4;
constexpr int kReplayThreads = 512;
constexpr int kReplayBatch = 16;
constexpr int kReplayPre = (kReplayBatch * kMaxPairs + kReplayThreads - 1) / kReplayThreads;

__global__ __launch_bounds__(kReplayThreads) void vreplay_kernel(int me, const float2 *__restrict__ rlog,
                                                                  const pca_info *__restrict__ info,
                                                                  float *__restrict__ Vu)
{
    __shared__ float vr[kReplayRows][256];
    __shared__ float2 lcs[2][kReplayBatch][kMaxPairs];
    const int tid = threadIdx.x;
    const int P = me / 2;
    const int r0 = blockIdx.x * kReplayRows;
    const int nsteps = info->steps;
    const int per = kReplayBatch * P;

    for (int t = tid; t < kReplayRows * 256; t += kReplayThreads) {
        const int r = t >> 8, c = t & 255;
        vr[r][c] = (r0 + r == c) ? 1.f : 0.f;
    }
    for (int t = tid; t < per; t += kReplayThreads) {
        const int gg = t / P, k = t - (t / P) * P;
        lcs[0][gg][k] = gg < nsteps ? rlog[(int64_t)gg * P + k] : make_float2(1.f, 0.f);
    }
    __syncthreads();

    const int task_r = tid / P, task_k = tid - (tid / P) * P;
    const bool has_task = tid < kReplayRows * P;
    const int nbatch = (nsteps + kReplayBatch - 1) / kReplayBatch;
    int step = 0;
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
            if (has_task) {
                const float2 cs = lcs[cur][gg][task_k];
                if (cs.y != 0.f) {
                    int a, b;
                    rr_pair(me, step, task_k, a, b);
                    const float va = vr[task_r][a], vb = vr[task_r][b];
                    vr[task_r][a] = cs.x * va - cs.y * vb;
                    vr[task_r][b] = cs.y * va + cs.x * vb;
                }
            }
            if (++step == me - 1) step = 0;
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < kReplayPre; ++q) {
            const int t = tid + q * kReplayThreads;
            if (t < per) lcs[cur ^ 1][t / P][t - (t / P) * P] = pre[q];
        }
        __syncthreads();
    }
    for (int t = tid; t < kReplayRows * me; t += kReplayThreads) {
        const int r = t / me, c = t - (t / me) * me;
        if (r0 + r < me) Vu[(int64_t)(r0 + r) * me + c] = vr[r][c];
    }
}

__global__ __launch_bounds__(1024) void sort_sign_kernel(int m, int me, const double *__restrict__ lam_u,
                                                         const float *__restrict__ Vu,
                                                         const pca_info *__restrict__ info_ws,
                                                         float *__restrict__ eigvals, float *__restrict__ V,
                                                         pca_info *__restrict__ info_out)
{
    __shared__ int perm[256];
    __shared__ double lam[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool nonfinite = info_ws->nonfinite != 0;
    if (nonfinite) {
        for (int i = tid; i < m; i += 1024) eigvals[i] = NAN;
        for (int e = tid; e < m * m; e += 1024) V[e] = NAN;
        if (tid == 0 && info_out) *info_out = *info_ws;
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
        eigvals[rank] = (float)x;
    }
    __syncthreads();
    for (int c = wave; c < m; c += 16) {
        const int j = perm[c];
        float best = -1.f;
        int bidx = 1 << 30;
        for (int r = lane; r < m; r += 64) {
            const float a = fabsf(Vu[(int64_t)r * me + j]);
            if (a > best) { best = a; bidx = r; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bidx, off, 64);
            if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
        }
        const float sgn = Vu[(int64_t)bidx * me + j] < 0.f ? -1.f : 1.f;
        for (int r = lane; r < m; r += 64) V[(int64_t)r * m + c] = sgn * Vu[(int64_t)r * me + j];
    }
    if (tid == 0 && info_out) *info_out = *info_ws;
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

hipError_t launch_jacobi(const float *C, int m, double tol, int max_sweeps, int fp64_angles,
                         const JacPlan &plan, double *lam_u, float2 *rlog, float *Vu, pca_info *info_ws,
                         float *eigvals, float *V, pca_info *info_out, hipStream_t st)
{
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kJacThreads), 0, st, C, m, plan.me, tol, max_sweeps,
                       fp64_angles, lam_u, rlog, info_ws);
    const unsigned nwg = (unsigned)((plan.me + kReplayRows - 1) / kReplayRows);
    hipLaunchKernelGGL(vreplay_kernel, dim3(nwg), dim3(kReplayThreads), 0, st, plan.me, rlog,
                       (const pca_info *)info_ws, Vu);
    hipLaunchKernelGGL(sort_sign_kernel, dim3(1), dim3(1024), 0, st, m, plan.me, (const double *)lam_u,
                       (const float *)Vu, (const pca_info *)info_ws, eigvals, V, info_out);
    return hipGetLastError();
}

}  // namespace pca

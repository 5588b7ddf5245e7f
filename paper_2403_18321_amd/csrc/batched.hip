// Batched form: many cubes of different pixel and band counts through the
// pipeline of Algorithm 1 in a fixed number of launches.
//
// batch_setup_kernel reads the caller's cube descriptors from device memory
// and writes the task table at the start of the workspace: the cubes in
// decreasing order of covariance work (bands, then pixels), each with its
// covariance plan, its slice of the workspace and the first global work item
// it owns in every batched launch; it also clears the work-queue counter of
// the persistent covariance launch. Every later batched kernel maps its work
// item to a cube through that table (binary search over the first items), so
// the whole sequence needs no host-to-device copy and can be captured in a
// graph once the descriptors are resident.
#include "common.hpp"
#include "kernels.hpp"

namespace pca {

namespace {

constexpr int kSetupThreads = 256;
constexpr int kMaxBatch = 4096;

__global__ __launch_bounds__(kSetupThreads) void batch_setup_kernel(const pca_cube *__restrict__ cubes, int nc,
                                                                    int max_sweeps, int cov_chunk, int proj_tiles,
                                                                    char *__restrict__ ws)
{
    __shared__ int order[kMaxBatch];
    __shared__ int key_m[kMaxBatch];
    __shared__ int64_t key_n[kMaxBatch];
    __shared__ int64_t off[kSetupThreads];        // workspace offset of a cube's slice, then its prefix
    __shared__ int64_t items[kSetupThreads][6];   // work items per launch, then their prefix
    __shared__ int64_t carry[7];                  // slices and work items of the earlier groups
    const int tid = threadIdx.x;
    // The sort keys, read once into LDS.
    for (int i = tid; i < nc; i += kSetupThreads) {
        key_m[i] = cubes[i].n_bands;
        key_n[i] = cubes[i].n_pixels;
    }
    if (tid < 7) carry[tid] = 0;
    __syncthreads();
    // Rank of each cube by (bands, pixels) descending, index ascending on ties.
    for (int i = tid; i < nc; i += kSetupThreads) {
        const int mi = key_m[i];
        const int64_t ni = key_n[i];
        int r = 0;
        for (int j = 0; j < nc; ++j) {
            const int mj = key_m[j];
            const int64_t nj = key_n[j];
            r += (mj > mi) || (mj == mi && (nj > ni || (nj == ni && j < i)));
        }
        order[r] = i;
    }
    __syncthreads();
    BatchHeader *h = reinterpret_cast<BatchHeader *>(ws);
    BatchCube *t = reinterpret_cast<BatchCube *>(ws + sizeof(BatchHeader));
    char *const area0 = ws + batch_table_bytes(nc);
    // The table in groups of kSetupThreads ranks: each thread forms its
    // cube's entry; the slices and first work items are the exclusive prefix
    // sums, in rank order, of the slice sizes and work-item counts.
    for (int base = 0; base < nc; base += kSetupThreads) {
        const int r = base + tid;
        const bool have = r < nc;
        BatchCube c;
        JacPlan jp;
        if (have) {
            const pca_cube d = cubes[order[r]];
            c.Y = d.Y;
            c.n = d.n_pixels;
            c.ld = d.ld_y;
            c.m = d.n_bands;
            c.k = d.k;
            c.mean = d.mean;
            c.eigvals = d.eigvals;
            c.V = d.V;
            c.Q = d.Q;
            c.info = d.info;
            c.cov = batch_cov_plan(c.n, c.m, cov_chunk);
            jp = jac_plan(c.m, max_sweeps);
            off[tid] = (int64_t)batch_cube_bytes(c.cov, jp, c.m);
            int64_t cnt[6];
            batch_counts(c.cov, c.n, c.m, proj_tiles, cnt);
            for (int q = 0; q < 6; ++q) items[tid][q] = cnt[q];
        } else {
            off[tid] = 0;
            for (int q = 0; q < 6; ++q) items[tid][q] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t a = carry[0], w[6];
            for (int q = 0; q < 6; ++q) w[q] = carry[1 + q];
            const int ng = nc - base < kSetupThreads ? nc - base : kSetupThreads;
            for (int i = 0; i < ng; ++i) {
                const int64_t sz = off[i];
                off[i] = a;
                a += sz;
                for (int q = 0; q < 6; ++q) {
                    const int64_t v = items[i][q];
                    items[i][q] = w[q];
                    w[q] += v;
                }
            }
            carry[0] = a;
            for (int q = 0; q < 6; ++q) carry[1 + q] = w[q];
        }
        __syncthreads();
        if (have) {
            char *a = area0 + off[tid];
            c.partS = reinterpret_cast<float *>(a);
            a += batch_al(c.cov.bytes_S);
            c.partSum = reinterpret_cast<double *>(a);
            a += batch_al(c.cov.bytes_sum);
            c.partShift = reinterpret_cast<float *>(a);
            a += batch_al(c.cov.bytes_shift);
            c.srow = reinterpret_cast<float *>(a);
            a += batch_al(c.cov.bytes_srow);
            c.part2 = reinterpret_cast<double *>(a);
            a += batch_al(c.cov.bytes_part2);
            c.C = reinterpret_cast<float *>(a);
            a += batch_al((size_t)c.m * c.m * sizeof(float));
            c.rlog = reinterpret_cast<float2 *>(a);
            a += batch_al(jp.bytes_log);
            c.lam_u = reinterpret_cast<double *>(a);
            a += batch_al(jp.bytes_lam);
            c.Vu = reinterpret_cast<float *>(a);
            a += batch_al(jp.bytes_vu);
            c.info_ws = reinterpret_cast<pca_info *>(a);
            c.rows = follow_rows(jp.me);
            c.proj_tiles = proj_tiles;
            c.w_cov = items[tid][0];
            c.w_fin1 = items[tid][1];
            c.w_fin2 = items[tid][2];
            c.w_rep = items[tid][3];
            c.w_sort = items[tid][4];
            c.w_proj = items[tid][5];
            t[r] = c;
        }
        __syncthreads();
    }
    if (tid == 0) {
        h->n_cubes = nc;
        h->pad = 0;
        for (int q = 0; q < 6; ++q) h->total[q] = carry[1 + q];
        for (int q = 0; q < 4; ++q) h->counter[q] = 0u;
    }
}

}  // namespace

hipError_t launch_batch_setup(const pca_cube *cubes_dev, int n_cubes, int mode, int max_sweeps, int cov_chunk,
                              int proj_tiles, char *ws, hipStream_t st)
{
    (void)mode;
    hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(kSetupThreads), 0, st, cubes_dev, n_cubes, max_sweeps,
                       cov_chunk, proj_tiles, ws);
    return hipGetLastError();
}

}  // namespace pca

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
    const int tid = threadIdx.x;
    // Rank of each cube by (bands, pixels) descending, index ascending on ties.
    for (int i = tid; i < nc; i += kSetupThreads) {
        const int mi = cubes[i].n_bands;
        const int64_t ni = cubes[i].n_pixels;
        int r = 0;
        for (int j = 0; j < nc; ++j) {
            const int mj = cubes[j].n_bands;
            const int64_t nj = cubes[j].n_pixels;
            r += (mj > mi) || (mj == mi && (nj > ni || (nj == ni && j < i)));
        }
        order[r] = i;
    }
    __syncthreads();
    if (tid != 0) return;
    BatchHeader *h = reinterpret_cast<BatchHeader *>(ws);
    BatchCube *t = reinterpret_cast<BatchCube *>(ws + sizeof(BatchHeader));
    char *area = ws + batch_table_bytes(nc);
    int64_t w[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < nc; ++r) {
        const pca_cube d = cubes[order[r]];
        BatchCube c;
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
        const JacPlan jp = jac_plan(c.m, max_sweeps);
        char *a = area;
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
        a += batch_al(jp.bytes_info);
        area += batch_cube_bytes(c.cov, jp, c.m);
        c.rows = follow_rows(jp.me);
        c.proj_tiles = proj_tiles;
        int64_t cnt[6];
        batch_counts(c.cov, c.n, c.m, proj_tiles, cnt);
        c.w_cov = w[0];
        c.w_fin1 = w[1];
        c.w_fin2 = w[2];
        c.w_rep = w[3];
        c.w_sort = w[4];
        c.w_proj = w[5];
        for (int q = 0; q < 6; ++q) w[q] += cnt[q];
        t[r] = c;
    }
    h->n_cubes = nc;
    h->pad = 0;
    for (int q = 0; q < 6; ++q) h->total[q] = w[q];
    for (int q = 0; q < 4; ++q) h->counter[q] = 0u;
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

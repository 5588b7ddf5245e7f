// Covariance of the centred cube, C = X^T X / (N - 1) (Algorithm 1, line 3;
// normalised by PIXELS - 1 as in Code 4.3), with the band-mean removal
// (Algorithm 1, line 2) fused so that the cube is streamed from HBM once.
//
// Pass 0 (cov_shift): a shift row s, the mean of a sample of pixels per band.
// Pass 1 (cov_partial): one workgroup per chunk of pixels. Each chunk is
// shifted by s_w = s, and the workgroup accumulates on chip
//   S_w = sum_{p in w} (y_p - s_w)(y_p - s_w)^T   (upper-triangle 32x32 blocks)
//   t_w = sum_{p in w} (y_p - s_w)               (float64 per band)
// with MFMA: float32 products (v_mfma_f32_32x32x2_f32) or the split-bfloat16
// products (v_mfma_f32_32x32x16_bf16) of x = hi + lo. Splitting the sum over
// pixel chunks and adding the chunk results mirrors the pixel split of
// equation (17); only the upper triangle is formed, as the manycore design
// does for the symmetric result.
// Pass 2 (cov_finalize): in float64 and chunk order,
//   mu = (1/N) sum_w (n_w s_w + t_w),  e_w = s_w - mu,
//   N_2 = sum_w [S_w + t_w e_w^T + e_w t_w^T + n_w e_w e_w^T]
//       = sum_p (y_p - mu)(y_p - mu)^T          (exact algebra),
//   C = N_2 / (N - 1), mirrored to a full symmetric matrix.
//
// Pass-1 kernels by layout: cov_partial_dma_kernel (band-interleaved float32
// or uint16 rows of whole 16-byte pieces, copied straight into LDS),
// cov_partial_dma4_kernel (other band-interleaved float32 cubes, the same
// kernel with 4-byte copies), cov_partial_bsq_dma_kernel (band-sequential
// rows of whole 16-byte pieces, split forms, likewise),
// cov_partial_bsq_kernel (other band-sequential cubes, register-staged),
// cov_partial_kernel (other band-interleaved uint16 layouts,
// register-staged) and the batched form's persistent launches
// (cov_partial_batched_dma_kernel, cov_partial_batched_bsq_kernel,
// cov_partial_batched_kernel).
#include "common.hpp"
#include "kernels.hpp"
#include "loader.hpp"

namespace pca {

namespace {

constexpr int kThreads = 256;   // 4 waves; wave w loads pixel group w of a stage
constexpr int KT = kCovTile;    // 32 pixels per stage = 4 groups of 8
constexpr int kMaxSlots = 9;    // accumulator blocks per wave at 8 blocks per side (36 / 4 waves)
constexpr int kFlush = 8;       // stages per first-level MFMA accumulation (float32 mode)
constexpr int kBfPitch = KT + 8;  // bf16 per band row in LDS (80 bytes)

enum { MODE_F32 = 0, MODE_BF16X3 = 1, MODE_BF16X4 = 2, MODE_FP16X3 = 3 };

// Pixel-major float32 stage pitch (floats): pitch % 64 == 32 so the two
// half-waves of an MFMA operand read fall on disjoint LDS banks.
__host__ __device__ constexpr int f32_pitch(int mpad) { return (mpad % 64 == 0) ? mpad + 32 : mpad; }

// Work order of the upper-triangle 32x32 blocks: block (bi, bj), bi <= bj,
// has id bj (bj + 1) / 2 + bi (column by column), so a matrix of nb blocks per
// side uses exactly the ids below nb (nb + 1) / 2, whatever nb is. Wave w
// owns ids w, w + 4, w + 8, ...; its slot e holds id 4 e + w.
__device__ inline void block_of_id(int id, int &bi, int &bj)
{
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= id) ++j;
    bj = j;
    bi = id - j * (j + 1) / 2;
}
// Accumulator slots per wave for nb blocks per side (a kernel variant each).
__host__ __device__ inline int cov_slots(int nb)
{
    const int per_wave = (nb * (nb + 1) / 2 + 3) / 4;
    return per_wave <= 3 ? 3 : (per_wave <= 6 ? 6 : (per_wave <= 7 ? 7 : kMaxSlots));
}
// Compact id for nb blocks per side (the layout of the partial results).
__device__ inline int compact_block(int bi, int bj, int nb) { return bi * nb - bi * (bi - 1) / 2 + (bj - bi); }

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(2))) _Float16 f16x2;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;

// The split forms. bfloat16: x = hi + lo (+ a remainder below 2^-16 |x|).
// float16 (MODE_FP16X3): x sc = hi + lo, sc the band's power-of-two scale
// (a float16 keeps 11 significant bits but only exponents -14..15, so each
// band is scaled into that range first; the pair then holds about 22 bits).
// Both store 16-bit patterns in the same tiles (bfloat16 storage type).
template <int MODE>
__device__ __forceinline__ void split2(f32x2 v, float sc, bf16x2 &h, bf16x2 &l)
{
    if constexpr (MODE == MODE_FP16X3) {
        const f32x2 t = {v[0] * sc, v[1] * sc};
        const f16x2 hh = __builtin_convertvector(t, f16x2);
        const f32x2 r = t - __builtin_convertvector(hh, f32x2);
        const f16x2 ll = __builtin_convertvector(r, f16x2);
        h = __builtin_bit_cast(bf16x2, hh);
        l = __builtin_bit_cast(bf16x2, ll);
    } else {
        h = __builtin_convertvector(v, bf16x2);
        const f32x2 r = v - __builtin_convertvector(h, f32x2);
        l = __builtin_convertvector(r, bf16x2);
    }
}

template <int MODE>
__device__ __forceinline__ void split1(float x, float sc, __bf16 &hi, __bf16 &lo)
{
    if constexpr (MODE == MODE_FP16X3) {
        const float t = x * sc;
        const _Float16 hh = (_Float16)t;
        hi = __builtin_bit_cast(__bf16, hh);
        lo = __builtin_bit_cast(__bf16, (_Float16)(t - (float)hh));
    } else {
        hi = (__bf16)x;
        lo = (__bf16)(x - (float)hi);
    }
}

// hi_i hi_j + hi_i lo_j + lo_i hi_j (+ lo_i lo_j for bf16x4) added to a.
template <int MODE>
__device__ __forceinline__ f32x16 split_products(bf16x8 hi_i, bf16x8 lo_i, bf16x8 hi_j, bf16x8 lo_j, f32x16 a)
{
    if constexpr (MODE == MODE_FP16X3) {
        const f16x8 hi = __builtin_bit_cast(f16x8, hi_i), li = __builtin_bit_cast(f16x8, lo_i);
        const f16x8 hj = __builtin_bit_cast(f16x8, hi_j), lj = __builtin_bit_cast(f16x8, lo_j);
        a = __builtin_amdgcn_mfma_f32_32x32x16_f16(hi, hj, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_32x32x16_f16(hi, lj, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_32x32x16_f16(li, hj, a, 0, 0, 0);
    } else {
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi_i, hi_j, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi_i, lo_j, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo_i, hi_j, a, 0, 0, 0);
        if constexpr (MODE == MODE_BF16X4) a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo_i, lo_j, a, 0, 0, 0);
    }
    return a;
}

// Per-band scales of the float16 split in the shift buffer: sc at srow + 512,
// 1 / sc at srow + 768 (powers of two, so both are exact).
constexpr int kScaleRow = 512, kInvScaleRow = 768;

// Entry r of a lane's 32x32 block (bi, bj) product in the scale of the data
// (the float16 split's sums carry the factor sc_i sc_j).
template <int MODE>
__device__ __forceinline__ float unscaled(float v, const float *__restrict__ srow, int bi, int bj, int r, int lane)
{
    if constexpr (MODE == MODE_FP16X3) {
        const int i = 32 * bi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);   // MFMA 32x32 result layout
        const int j = 32 * bj + (lane & 31);
        return v * srow[kInvScaleRow + i] * srow[kInvScaleRow + j];
    } else {
        return v;
    }
}

// ---- pass 0: the shift row ------------------------------------------------
//
// s_b = mean of a sample of the pixels of band b: every pixel up to
// kShiftSample of them, else kShiftRuns runs of 32 pixels spread evenly over
// the cube, the pixels of a run an odd stride apart (an odd stride runs
// through every image column of a power-of-two-wide scene, so no single
// detector column is over-represented; a run stays within a few pages, so
// the sample costs few address-translation misses), added in float64 in a
// fixed order. Any shift gives the same covariance in exact arithmetic (pass
// 2 removes it exactly); one close to the band mean keeps the shifted values
// small whatever a single pixel holds (a dead or hot detector column at the
// start of every chunk, for one), and with them the rounding of the
// products, which the split-bfloat16 forms feel most. uint16 cubes round s to
// an integer so that the row can also be held in the cube's own type; float32
// cubes round it to 8 significant bits (a bfloat16 value), which keeps it
// within 2^-9 of the sample mean and makes it an integer from 128 on, so that
// integer-valued cubes (converted sensor counts) stay integer-valued after
// the shift and their bfloat16 hi/lo split stays exact up to 2^16.
// The same pass sets the per-band power-of-two scales of the float16 split:
// 1/2 for uint16 cubes (|y - s| < 2^16, so y - s scaled by 1/2 is below the
// float16 maximum and its 17 significant bits fit the hi/lo pair exactly);
// for float32 cubes the largest sampled |y - s| is scaled to at most 2^4,
// which leaves a factor 2^12 for values beyond the sample before a float16
// overflows (an overflow makes the covariance non-finite, reported as such).
// Shift area: float32 s[256], the cube-type row [256], sc[256], 1/sc[256].
constexpr int kShiftRuns = 8;
constexpr int kShiftSample = 32 * kShiftRuns;   // 256 pixels
constexpr int kShiftThreads = 256;              // one 32-band block a workgroup

// Band block bb (bands 32 bb .. 32 bb + 31) of the shift row. Band-interleaved
// cubes: the 32 lanes of a group read one sampled pixel's 32 bands;
// band-sequential cubes: 8 lanes read 8 sampled pixels of a band. Sample i
// (thread offset i0 = i mod 8, j = i / 8) of a cube of n > kShiftSample
// pixels is pixel start(r) + (i mod 32) stride of run r = i / 32, with
// start(r) = r n / kShiftRuns + 5 r (the small offset keeps the runs' first
// pixels off one image column when n / kShiftRuns is a multiple of the scene
// width) and an odd stride of at most 67, so every sample stays inside its
// run's n / kShiftRuns pixels. Every thread issues all of its 32 loads (at
// clamped addresses) before adding the valid ones.
template <typename T>
__device__ __forceinline__ void cov_shift_body(const T *__restrict__ Y, int64_t n, int m, int64_t ld, bool bsq, int bb,
                               float *__restrict__ srow)
{
    __shared__ double red[32][9];
    __shared__ float svs[32], dev[32][9];
    const int tid = threadIdx.x;
    const bool all = n <= kShiftSample;
    const int ns = all ? (int)n : kShiftSample;
    const int64_t run = n / kShiftRuns;
    const int off = run >= 32 + 36 ? 5 : 0;              // 5 r <= 35 < run - 31 stride
    int64_t stride = off ? (run - 36) / 31 : 1;
    stride = stride > 67 ? 67 : (stride < 1 ? 1 : stride);
    if (stride > 1 && (stride & 1) == 0) --stride;
    const int bl = bsq ? tid >> 3 : tid & 31;
    const int i0 = bsq ? tid & 7 : tid >> 5;
    const int b = 32 * bb + bl;
    const bool bok = b < m;
    const T *base = bsq ? Y + (int64_t)(bok ? b : 0) * ld : Y + (bok ? b : 0);
    const int64_t step = bsq ? 1 : ld;
    float v[kShiftSample / 8];
    if (all) {
#pragma unroll
        for (int j = 0; j < kShiftSample / 8; ++j) {
            const int i = i0 + 8 * j;
            v[j] = load_elem(base + (int64_t)(i < ns ? i : 0) * step);
        }
    } else {
        int64_t start[kShiftRuns];
#pragma unroll
        for (int r = 0; r < kShiftRuns; ++r) start[r] = ((int64_t)r * n / kShiftRuns + off * r) * step;
        const int64_t sstep = stride * step;
#pragma unroll
        for (int j = 0; j < kShiftSample / 8; ++j)   // sample i = i0 + 8 j: run j / 4, place 8 (j mod 4) + i0
            v[j] = load_elem(base + start[j >> 2] + (int64_t)(8 * (j & 3) + i0) * sstep);
    }
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < kShiftSample / 8; ++j) a += (bok && i0 + 8 * j < ns) ? (double)v[j] : 0.0;
    red[bl][i0] = a;
    __syncthreads();
    if (tid < 32) {
        const int bq = 32 * bb + tid;
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) t += red[tid][q];
        T *rowT = reinterpret_cast<T *>(srow + 256);
        float sv = 0.f;
        if (bq < m) {
            const double mean = t / (double)ns;
            if constexpr (sizeof(T) == 2) sv = (float)fmin(fmax(rint(mean), 0.0), 65535.0);
            else sv = (float)(__bf16)(float)mean;   // 8 significant bits (see above)
        }
        srow[bq] = sv;
        svs[tid] = sv;
        if constexpr (sizeof(T) == 2) rowT[bq] = (T)(unsigned)sv;
        else rowT[bq] = sv;
    }
    __syncthreads();
    // Largest sampled deviation from the shift, per band.
    float dmax = 0.f;
#pragma unroll
    for (int j = 0; j < kShiftSample / 8; ++j)
        if (bok && i0 + 8 * j < ns) dmax = fmaxf(dmax, fabsf(v[j] - svs[bl]));
    dev[bl][i0] = dmax;
    __syncthreads();
    if (tid < 32) {
        const int bq = 32 * bb + tid;
        float mx = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) mx = fmaxf(mx, dev[tid][q]);
        int e = 0;
        if constexpr (sizeof(T) == 2) {
            e = -1;
        } else if (bq < m && mx > 0.f && mx <= 3.0e38f) {
            int k;
            (void)frexpf(mx, &k);   // mx < 2^k
            e = 4 - k;
            e = e > 100 ? 100 : (e < -100 ? -100 : e);
        }
        srow[kScaleRow + bq] = ldexpf(1.f, e);
        srow[kInvScaleRow + bq] = ldexpf(1.f, -e);
    }
}

template <typename T>
__global__ __launch_bounds__(kShiftThreads) void cov_shift_kernel(const T *__restrict__ Y, int64_t n, int m,
                                                                  int64_t ld, int bsq, float *__restrict__ srow)
{
    cov_shift_body<T>(Y, n, m, ld, bsq != 0, (int)blockIdx.x, srow);
}

// One chunk c of one cube (the body of the single-cube and the batched
// launches). kSkip: products of slots past the cube's last block are skipped
// (the batched launch sizes S for the widest cube of any batch).
template <typename T, int VEC, int MODE, int S, bool kSkip = false>
__device__ __forceinline__ void cov_partial_body(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int centered, int64_t chunk, int nb,
    int nblk, int mpad, float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow, int64_t c)
{
    constexpr int kF32Max = KT * (256 + 32);
    constexpr int kBfMax = 256 * kBfPitch;
    __shared__ __attribute__((aligned(16))) float tileF[MODE == MODE_F32 ? kF32Max : 4];
    __shared__ __attribute__((aligned(16))) __bf16 hiT[MODE == MODE_F32 ? 8 : kBfMax];
    __shared__ __attribute__((aligned(16))) __bf16 loT[MODE == MODE_F32 ? 8 : kBfMax];
    __shared__ double red[4][256];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t pbeg = c * chunk;
    const int64_t pend = (pbeg + chunk < n) ? pbeg + chunk : n;
    const int pf = f32_pitch(mpad);

    // Shift: the cube's shift row (zero when the cube is centred).
    float shift[4], scs[4];
    double sums[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int b = slot_band<VEC>(lane, s);
        shift[s] = (!centered && b < m) ? srow[b] : 0.f;
        scs[s] = (MODE == MODE_FP16X3 && b < mpad) ? srow[kScaleRow + b] : 1.f;
        sums[s] = 0.0;
    }

    // float32 products accumulate in two levels (the MFMA accumulator is
    // emptied into acc2 every kFlush stages) to keep rounding chains short;
    // a split-bfloat16 MFMA already sums 16 pixels per instruction, so one
    // level keeps its chains as short.
    constexpr bool kTwoLevel = MODE == MODE_F32;
    constexpr int kSlots2 = kTwoLevel ? S : 1;
    f32x16 acc[S], acc2[kSlots2];
#pragma unroll
    for (int e = 0; e < S; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[e][r] = 0.f;
    }
#pragma unroll
    for (int e = 0; e < kSlots2; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[e][r] = 0.f;
    }

    // Register prefetch of PREF stages ahead (float32 mode needs its registers
    // for the two-level accumulators).
    constexpr int PREF = MODE == MODE_F32 ? 1 : 2;
    const int64_t nst = (pend - pbeg + KT - 1) / KT;
    Group<T, VEC> ga, gb;
    ga.load(Y, ld, pbeg + 8 * wave, pend, m, lane);
    if (PREF == 2 && nst > 1) gb.load(Y, ld, pbeg + KT + 8 * wave, pend, m, lane);
    bool bok[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) bok[s] = slot_band<VEC>(lane, s) < m;

    // LDS operand offsets of this wave's blocks (slot e: id 4 e + wave). A slot
    // past the last block multiplies block (0, 0) again and is never stored,
    // so the product loop has no branches.
    const int nbl = nb * (nb + 1) / 2;
    int offI[S], offJ[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
        int bi = 0, bj = 0;
        if (4 * e + wave < nbl) block_of_id(4 * e + wave, bi, bj);
        if constexpr (MODE == MODE_F32) {
            offI[e] = 32 * bi + (lane & 31);
            offJ[e] = 32 * bj + (lane & 31);
        } else {
            offI[e] = (32 * bi + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
            offJ[e] = (32 * bj + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
        }
    }

    auto stage = [&](Group<T, VEC> &v, int64_t st) {
        const int64_t g0 = pbeg + st * KT + 8 * wave;  // first pixel of this wave's group
        const int64_t nval64 = pend - g0;
        const int nval = nval64 < 0 ? 0 : (nval64 > 8 ? 8 : (int)nval64);

        // Centre about the chunk shift, accumulate band sums, stage in LDS.
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int b = slot_band<VEC>(lane, s);
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = (i < nval && bok[s]) ? v.get(i, s) - shift[s] : 0.f;
            double ts = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) ts += (double)x[i];
            sums[s] += ts;
            if constexpr (MODE == MODE_F32) {
                if constexpr (VEC == 1) {
                    if (b < mpad) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) tileF[(8 * wave + i) * pf + b] = x[i];
                    }
                }
            } else {
                if (b < mpad) {
                    bf16x8 h, l;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        __bf16 hh, ll;
                        split1<MODE>(x[i], scs[s], hh, ll);
                        h[i] = hh;
                        l[i] = ll;
                    }
                    *reinterpret_cast<bf16x8 *>(&hiT[b * kBfPitch + 8 * wave]) = h;
                    *reinterpret_cast<bf16x8 *>(&loT[b * kBfPitch + 8 * wave]) = l;
                }
            }
        }
        if constexpr (MODE == MODE_F32 && VEC == 4) {
            const int b = 4 * lane;
            if (b < mpad) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    f32x4 q;
#pragma unroll
                    for (int s = 0; s < 4; ++s) q[s] = (i < nval && bok[s]) ? v.get(i, s) - shift[s] : 0.f;
                    *reinterpret_cast<f32x4 *>(&tileF[(8 * wave + i) * pf + b]) = q;
                }
            }
        }

        // Prefetch a later stage while this one is multiplied.
        if (st + PREF < nst) v.load(Y, ld, g0 + PREF * KT, pend, m, lane);
        __syncthreads();

        if constexpr (MODE == MODE_F32) {
#pragma unroll 2
            for (int kk = 0; kk < KT / 2; ++kk) {
                const float *tr = tileF + (2 * kk + (lane >> 5)) * pf;
#pragma unroll
                for (int e = 0; e < S; ++e) {
                    if (kSkip && 4 * e + wave >= nbl) continue;
                    acc[e] = __builtin_amdgcn_mfma_f32_32x32x2f32(tr[offI[e]], tr[offJ[e]], acc[e], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KT / 16; ++kk) {
#pragma unroll
                for (int e = 0; e < S; ++e) {
                    if (kSkip && 4 * e + wave >= nbl) continue;
                    const bf16x8 hi_i = *reinterpret_cast<const bf16x8 *>(&hiT[offI[e] + 16 * kk]);
                    const bf16x8 lo_i = *reinterpret_cast<const bf16x8 *>(&loT[offI[e] + 16 * kk]);
                    const bf16x8 hi_j = *reinterpret_cast<const bf16x8 *>(&hiT[offJ[e] + 16 * kk]);
                    const bf16x8 lo_j = *reinterpret_cast<const bf16x8 *>(&loT[offJ[e] + 16 * kk]);
                    acc[e] = split_products<MODE>(hi_i, lo_i, hi_j, lo_j, acc[e]);
                }
            }
        }
        __syncthreads();

        if constexpr (kTwoLevel) {
            if ((st + 1) % kFlush == 0) {
#pragma unroll
                for (int e = 0; e < S; ++e) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) { acc2[e][r] += acc[e][r]; acc[e][r] = 0.f; }
                }
            }
        }
    };

    for (int64_t st = 0; st < nst; st += PREF) {
        stage(ga, st);
        if (PREF == 2 && st + 1 < nst) stage(gb, st + 1);
    }

    // Partial second moment of this chunk: [chunk][block][reg][lane], blocks
    // in the row-major compact order the finalisation reads.
#pragma unroll
    for (int e = 0; e < S; ++e) {
        if (4 * e + wave < nbl) {
            int bi, bj;
            block_of_id(4 * e + wave, bi, bj);
            float *dst = partS + ((c * nblk + compact_block(bi, bj, nb)) * 16) * 64 + lane;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                dst[r * 64] = unscaled<MODE>(kTwoLevel ? acc2[e % kSlots2][r] + acc[e][r] : acc[e][r], srow, bi, bj, r,
                                             lane);
        }
    }

    // Band sums: the four waves saw different pixels of the same bands.
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int b = slot_band<VEC>(lane, s);
        if (b < 256) red[wave][b] = sums[s];
    }
    __syncthreads();
    for (int b = tid; b < mpad; b += kThreads) {
        const double t = ((red[0][b] + red[1][b]) + red[2][b]) + red[3][b];
        partSum[c * mpad + b] = t;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int b = slot_band<VEC>(lane, s);
        if (wave == 0 && b < mpad) partShift[c * mpad + b] = shift[s];
    }
}

template <typename T, int VEC, int MODE, int S>
__global__ __launch_bounds__(kThreads) void cov_partial_kernel(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int centered, int64_t chunk, int nb,
    int nblk, int mpad, float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow)
{
    cov_partial_body<T, VEC, MODE, S>(Y, n, m, ld, centered, chunk, nb, nblk, mpad, partS, partSum, partShift, srow,
                                      (int64_t)blockIdx.x);
}

// The split products of one 32-pixel stage for a wave's S blocks, from the
// hi / lo tiles in LDS (hi at hl, lo kHalf further; block e's operand rows at
// offI[e], offJ[e]); only the first ne slots hold blocks (the rest are
// skipped). The (k-step, block) items run in order, and the operands of the
// next item are read while the products of this one run.
template <int MODE, int S>
__device__ __forceinline__ void split_block_products(const __bf16 *hl, const int (&offI)[S], const int (&offJ)[S],
                                                     f32x16 (&acc)[S], int ne = S)
{
    constexpr int kHalf = 256 * kBfPitch;
    constexpr int kItems = (KT / 16) * S;
    bf16x8 cur[4], nxt[4];
    auto operands = [&](int it, bf16x8(&o)[4]) {
        const int kk = it / S, e = it - (it / S) * S;
        o[0] = *reinterpret_cast<const bf16x8 *>(&hl[offI[e] + 16 * kk]);
        o[1] = *reinterpret_cast<const bf16x8 *>(&hl[kHalf + offI[e] + 16 * kk]);
        o[2] = *reinterpret_cast<const bf16x8 *>(&hl[offJ[e] + 16 * kk]);
        o[3] = *reinterpret_cast<const bf16x8 *>(&hl[kHalf + offJ[e] + 16 * kk]);
    };
    operands(0, cur);
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int e = it - (it / S) * S;
        const int en = (it + 1) - ((it + 1) / S) * S;
        if (it + 1 < kItems && en < ne) operands(it + 1, nxt);
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
        if (e < ne) acc[e] = split_products<MODE>(cur[0], cur[1], cur[2], cur[3], acc[e]);
        __builtin_amdgcn_sched_barrier(0);
        if (it + 1 < kItems) {
#pragma unroll
            for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
        }
    }
}

// ---- float32 cubes with 16-byte aligned rows: pixel rows copied into LDS --
//
// The same chunk algorithm, organised for this case:
//  * the raw pixel rows go from HBM straight into LDS through the load unit
//    (global_load_lds_dwordx4: lane l's 16 bytes land at base + 16 l), two
//    stages ahead of use, so no registers are tied up by loads in flight.
//    The FP32 form rotates three ring slots (kRing); the split forms two
//    slots plus two sets of hi / lo tiles. The slots are separate LDS arrays
//    used in a fixed rotation, which lets the compiler see that reading one
//    does not wait on the copies into the others; the copy waits (vmcnt) and
//    the barriers are explicit;
//  * 8 waves of modest register use, two per SIMD, so that one wave's
//    centring and splitting overlaps another's matrix products;
//  * rows past the chunk end, and lanes past the last band, copy the shift
//    row (held in the cube's own type after the float32 row), so they centre
//    to exact zeros without masks.
constexpr int kRing = 3;
constexpr int kDmaWaves = 8;
constexpr int kDmaThreads = 64 * kDmaWaves;
constexpr int kDmaPix = KT / kDmaWaves;   // pixels per wave per stage (copies per wave per stage)

// Accumulator slots per wave (blocks id = kDmaWaves e + wave) for nb blocks
// per side.
__host__ __device__ inline int dma_slots(int nb)
{
    const int per_wave = (nb * (nb + 1) / 2 + kDmaWaves - 1) / kDmaWaves;
    return per_wave <= 2 ? 2 : per_wave;   // 2, 3, 4 or 5
}

// s_waitcnt immediates (gfx9 layout: vmcnt[3:0] and [15:14], expcnt[6:4],
// lgkmcnt[11:8]; all-ones fields do not wait).
constexpr int waitcnt_vm(int n) { return (n & 0xF) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8); }
constexpr int kWaitLgkm0 = 0xF | (0x3 << 14) | (0x7 << 4);

// Workgroup barrier for LDS traffic only: this wave's LDS reads and writes
// complete, then s_barrier (a __syncthreads would also wait for the copies
// in flight). The empty asm statements keep the compiler from moving memory
// operations across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// LDS of the chunk kernel: one set per (element type, mode), shared by the
// slot-count variants that one persistent launch inlines. The three ring
// slots are separate LDS arrays, which lets the compiler see that reading
// one slot does not wait on the copies into the others. The float32 form
// uses three ring slots; the split forms two ring slots and two sets of
// hi / lo tiles (stage k's tiles are read while stage k + 1's are written).
template <typename T, int MODE>
struct DmaLds {
    static constexpr int kPitch = (MODE == MODE_F32 && sizeof(T) == 4) ? 288 : 256;
    static constexpr int kRawElems = KT * kPitch;
    template <int K>
    __device__ static __forceinline__ T *ring()
    {
        __shared__ __attribute__((aligned(16))) T r[kRawElems];
        return r;
    }
    template <int K>
    __device__ static __forceinline__ __bf16 *tiles()
    {
        __shared__ __attribute__((aligned(16))) __bf16 h[MODE == MODE_F32 ? 8 : 2 * 256 * kBfPitch];
        return h;
    }
    __device__ static __forceinline__ float *shift()
    {
        __shared__ float v[256];
        return v;
    }
};

// Chunk c of a cube. CW is the width of one copy: 16 bytes (rows of whole
// 16-byte pieces), or 4 bytes a lane for float32 rows of any band count and
// alignment (a copy then moves 64 consecutive bands of one pixel, and a row
// takes one to four copies). kSkip: a wave that holds no block skips the
// products (narrow cubes of a batch). The stage walk starts at stage
// c nst / spread.
template <typename T, int MODE, int S, int CW, bool kSkip>
__device__ __forceinline__ void cov_dma_body(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int64_t chunk, int nb, int nblk, int mpad,
    float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow, int64_t c, int64_t spread)
{
    // Staged pixel rows of 256 elements (288 floats for the float32 products
    // of a float32 cube, whose two half-waves read rows one apart). A copy
    // instruction moves 16 bytes per lane: one float32 row (4 bands a lane),
    // or two uint16 rows (8 bands a lane, lanes 32-63 on the second pixel).
    static_assert(CW == 16 || (CW == 4 && sizeof(T) == 4), "4-byte copies stage float32 rows");
    constexpr bool kU16 = sizeof(T) == 2;
    constexpr int pitch = (MODE == MODE_F32 && !kU16) ? 288 : 256;
    constexpr int kPerLane = CW / (int)sizeof(T);            // bands per lane and copy
    constexpr int kRowsPerCopy = kU16 ? 2 : 1;
    constexpr int kCopies = kDmaPix / kRowsPerCopy;          // 16-byte copies per wave per stage
    constexpr int kRawElems = KT * pitch;
    constexpr int kHalf = 256 * kBfPitch;   // bf16 per tile (hi, then lo)
    constexpr int kRawWords = (kRawElems * (int)sizeof(T) + 3) / 4;
    T *const raw0 = DmaLds<T, MODE>::template ring<0>();
    T *const raw1 = DmaLds<T, MODE>::template ring<1>();
    float *const shv = DmaLds<T, MODE>::shift();
    static_assert(kRawElems == DmaLds<T, MODE>::kRawElems, "ring slot size");
    static_assert(kRawWords * 4 >= kDmaWaves * 256 * (int)sizeof(double), "band-sum scratch");
    double(*red)[256] = reinterpret_cast<double(*)[256]>(static_cast<void *>(raw0));   // after the ring drains

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t pbeg = c * chunk;
    const int64_t pend = (pbeg + chunk < n) ? pbeg + chunk : n;
    const int64_t nst = (pend - pbeg + KT - 1) / KT;
    const int cl = kU16 ? (lane & 31) : lane;                  // lane within its row
    const int loff = kPerLane * cl < m ? kPerLane * cl : 0;   // m % kPerLane == 0 on this path
    const T *row0 = reinterpret_cast<const T *>(srow + 256);   // the shift row in the cube's type

    // Workgroups walk their chunks from different starting stages (evenly
    // spread over the chunk, wrapping around): chunks are equal power-of-two
    // multiples of bytes apart, and in lockstep every workgroup would hit
    // the same HBM channel at the same moment.
    const int64_t rot = (c * nst) / spread;
    const int nq = (mpad + 63) >> 6;   // 4-byte copies per row
    // Copies of the stage at position t of this walk (pixels pbeg + 32 t'
    // with t' = (t + rot) mod nst; positions past the end copy the first
    // pixel) into ring slot R.
    auto issue = [&](T *R, int64_t t) {
        const int64_t tt = t < nst ? (t + rot < nst ? t + rot : t + rot - nst) : nst;
        if constexpr (CW == 4) {
#pragma unroll
            for (int i = 0; i < kDmaPix; ++i) {
                const int r = kDmaPix * wave + i;
                const int64_t p = pbeg + tt * KT + r;
                const bool pok = p < pend;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q < nq) {
                        // Rows past the chunk end copy the shift row itself
                        // and lanes past the last band its first element, so
                        // both centre to zero.
                        const int b = 64 * q + lane;
                        const T *src = b < m ? (pok ? Y + p * ld : row0) + b : row0;
                        __builtin_amdgcn_global_load_lds(static_cast<const void *>(src),
                                                         static_cast<void *>(R + r * pitch + 64 * q), 4, 0, 0);
                    }
                }
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < kCopies; ++i) {
            const int r = kDmaPix * wave + kRowsPerCopy * i;           // first staged row of this copy
            const int64_t p = pbeg + tt * KT + r + (kU16 ? (lane >> 5) : 0);
            const T *rowp = (p < pend && loff == kPerLane * cl) ? Y + p * ld : row0;
            // (void pointers: the host pass drops kernels whose target
            // builtins take arguments of template-dependent type)
            __builtin_amdgcn_global_load_lds(static_cast<const void *>(rowp + loff), static_cast<void *>(R + r * pitch),
                                             16, 0, 0);
        }
    };

    // Shift per band: the shift row; bands past the last one take the values
    // their lanes copy (row0[b mod kPerLane]), so they centre to zero.
    for (int b = tid; b < 256; b += kDmaThreads) shv[b] = load_elem(row0 + (b < m ? b : b % kPerLane));
    asm volatile("" ::: "memory");   // the shift load and store stay ahead of the copies
    issue(raw0, 0);
    issue(raw1, 1);

    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr bool kTwoLevel = MODE == MODE_F32;
    constexpr int kSlots2 = kTwoLevel ? S : 1;
    f32x16 acc[S], acc2[kSlots2];
#pragma unroll
    for (int e = 0; e < S; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[e][r] = 0.f;
    }
#pragma unroll
    for (int e = 0; e < kSlots2; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[e][r] = 0.f;
    }

    // Operand offsets of this wave's blocks (slot e: id kDmaWaves e + wave; a
    // slot past the last block points at block (0, 0), is skipped by the
    // products and is never stored).
    const int nbl = nb * (nb + 1) / 2;
    // Slots that hold a block (a prefix: the ids grow with the slot); the
    // products of the others are skipped.
    const int nslots = nbl - wave <= 0 ? 0 : ((nbl - wave + kDmaWaves - 1) / kDmaWaves < S ? (nbl - wave + kDmaWaves - 1) / kDmaWaves : S);
    int offI[S], offJ[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
        int bi = 0, bj = 0;
        if (kDmaWaves * e + wave < nbl) block_of_id(kDmaWaves * e + wave, bi, bj);
        if constexpr (MODE == MODE_F32) {
            offI[e] = 32 * bi + (lane & 31);
            offJ[e] = 32 * bj + (lane & 31);
        } else {
            offI[e] = (32 * bi + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
            offJ[e] = (32 * bj + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
        }
    }
    lds_barrier();   // shv visible
    // Centring works on bands lane + 64 s (consecutive lanes, consecutive
    // band rows of the tiles, so their tile stores spread over the banks).
    float shb[4], scb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        shb[s] = shv[lane + 64 * s];
        scb[s] = (MODE == MODE_FP16X3 && lane + 64 * s < mpad) ? srow[kScaleRow + lane + 64 * s] : 1.f;
    }
    float shI[S], shJ[S];
    if constexpr (MODE == MODE_F32) {
#pragma unroll
        for (int e = 0; e < S; ++e) {
            shI[e] = shv[offI[e]];
            shJ[e] = shv[offJ[e]];
        }
    }

    // This wave's pixels of a landed stage, centred: band sums (float32 over
    // the stage's 4 pixels, then float64) and, for the split forms, the hi /
    // lo tiles in LDS, band-major.
    auto centre = [&](const T *R, __bf16 *hl) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int b = lane + 64 * s;
            if (b >= mpad) continue;
            float x[kDmaPix];
#pragma unroll
            for (int i = 0; i < kDmaPix; ++i) x[i] = load_elem(R + (kDmaPix * wave + i) * pitch + b) - shb[s];
            sums[s] += (double)((x[0] + x[1]) + (x[2] + x[3]));
            if constexpr (MODE != MODE_F32) {
                bf16x4 h, l;
#pragma unroll
                for (int q = 0; q < kDmaPix / 2; ++q) {
                    const f32x2 v = {x[2 * q], x[2 * q + 1]};
                    bf16x2 hh, ll;
                    split2<MODE>(v, scb[s], hh, ll);
                    h[2 * q] = hh[0];
                    h[2 * q + 1] = hh[1];
                    l[2 * q] = ll[0];
                    l[2 * q + 1] = ll[1];
                }
                *reinterpret_cast<bf16x4 *>(&hl[b * kBfPitch + kDmaPix * wave]) = h;
                *reinterpret_cast<bf16x4 *>(&hl[kHalf + b * kBfPitch + kDmaPix * wave]) = l;
            }
        }
    };

    auto products = [&](const T *R, const __bf16 *hl) {
        if constexpr (MODE == MODE_F32) {
            // The operands of pixel pair kk + 1 are read while the products
            // of pair kk run, so that no product waits for its LDS reads.
            // Slots past nslots hold no block and are skipped.
            float xa[S] = {}, xb[S] = {};
#pragma unroll
            for (int e = 0; e < S; ++e) {
                if (e < nslots) {
                    xa[e] = load_elem(R + (lane >> 5) * pitch + offI[e]);
                    xb[e] = load_elem(R + (lane >> 5) * pitch + offJ[e]);
                }
            }
#pragma unroll
            for (int kk = 0; kk < KT / 2; ++kk) {
                float ya[S] = {}, yb[S] = {};
                if (kk + 1 < KT / 2) {
                    const T *tr = R + (2 * kk + 2 + (lane >> 5)) * pitch;
#pragma unroll
                    for (int e = 0; e < S; ++e) {
                        if (e < nslots) {
                            ya[e] = load_elem(tr + offI[e]);
                            yb[e] = load_elem(tr + offJ[e]);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
#pragma unroll
                for (int e = 0; e < S; ++e)
                    if (e < nslots)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[e] - shI[e], xb[e] - shJ[e], acc[e], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                if (kk + 1 < KT / 2) {
#pragma unroll
                    for (int e = 0; e < S; ++e) {
                        xa[e] = ya[e];
                        xb[e] = yb[e];
                    }
                }
            }
        } else {
            split_block_products<MODE, S>(hl, offI, offJ, acc, nslots);
        }
    };

    // Wait until this wave's copies of the oldest stage in flight have landed
    // (the copies of the stage after it may still be in flight).
    auto wait_one = [&]() {
        if constexpr (CW == 4) {
            switch (nq) {
            case 1: __builtin_amdgcn_s_waitcnt(waitcnt_vm(kDmaPix)); break;
            case 2: __builtin_amdgcn_s_waitcnt(waitcnt_vm(2 * kDmaPix)); break;
            case 3: __builtin_amdgcn_s_waitcnt(waitcnt_vm(3 * kDmaPix)); break;
            default: __builtin_amdgcn_s_waitcnt(waitcnt_vm(4 * kDmaPix)); break;
            }
        } else {
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(kCopies));
        }
    };
    // Stage counts are rounded up to a multiple of the ring: stages past the
    // chunk end are copies of its first pixel, which centre to exact zeros
    // and add nothing, so every step is the same straight-line code.
    if constexpr (MODE == MODE_F32) {
        // One stage in ring slot `cur`; the copies for two stages ahead go
        // into `nxt` (the slot of the previous stage, which every wave has
        // finished reading once past the barrier).
        // Each wave centres only its own rows, so once past the barrier the
        // band sums and the products of a stage may come in either order:
        // waves 4-7 multiply first, so that the two waves of a SIMD (w and
        // w + 4) overlap one's centring with the other's products.
        T *const raw2 = DmaLds<T, MODE>::template ring<2>();
        const bool prod_first = (wave & 4) != 0;
        auto step = [&](T *cur, T *nxt, int64_t st) {
            wait_one();
            lds_barrier();
            issue(nxt, st + 2);
            if (prod_first && (!kSkip || nbl > wave)) products(cur, nullptr);
            centre(cur, nullptr);
            if (!prod_first && (!kSkip || nbl > wave)) products(cur, nullptr);
            if ((st + 1) % kFlush == 0) {
#pragma unroll
                for (int e = 0; e < S; ++e) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) { acc2[e][r] += acc[e][r]; acc[e][r] = 0.f; }
                }
            }
        };
        for (int64_t st = 0; st < nst; st += kRing) {
            step(raw0, raw2, st);
            step(raw1, raw0, st + 1);
            step(raw2, raw1, st + 2);
        }
    } else {
        // Split forms: two ring slots and two tile sets. Step k centres stage
        // k + 1 (its raw slot to tile set (k + 1) mod 2) and multiplies stage
        // k (tile set k mod 2), with one barrier: the tiles written in step k
        // are read in step k + 1, and the tile set read in step k is written
        // again in step k + 1. Each wave centres only the rows its own copies
        // bring in, so a raw slot needs only this wave's copy wait, and the
        // copies for stage k + 2 may go into stage k's slot once this wave
        // has centred it. Waves 4-7 multiply before they centre, so that the
        // two waves of a SIMD (w and w + 4) overlap one's centring and
        // splitting (vector ALU) with the other's products (matrix cores).
        __bf16 *const t0 = DmaLds<T, MODE>::template tiles<0>();
        __bf16 *const t1 = DmaLds<T, MODE>::template tiles<1>();
        const bool prod_first = (wave & 4) != 0;
        const bool has_blocks = !kSkip || nbl > wave;
        wait_one();
        centre(raw0, t0);
        lds_barrier();
        auto step = [&](T *slot_k, T *slot_k1, const __bf16 *tk, __bf16 *tk1, int64_t k) {
            issue(slot_k, k + 2);
            if (prod_first && has_blocks) products(nullptr, tk);
            wait_one();
            centre(slot_k1, tk1);
            if (!prod_first && has_blocks) products(nullptr, tk);
            lds_barrier();
        };
        for (int64_t k = 0; k < nst; k += 2) {
            step(raw0, raw1, t0, t1, k);
            step(raw1, raw0, t1, t0, k + 1);
        }
    }
    // The stages copied ahead past the end must land before the workgroup's
    // LDS is reused (the band sums below, or another workgroup).
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __syncthreads();

#pragma unroll
    for (int e = 0; e < S; ++e) {
        if (kDmaWaves * e + wave < nbl) {
            int bi, bj;
            block_of_id(kDmaWaves * e + wave, bi, bj);
            float *dst = partS + ((c * nblk + compact_block(bi, bj, nb)) * 16) * 64 + lane;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                dst[r * 64] = unscaled<MODE>(kTwoLevel ? acc2[e % kSlots2][r] + acc[e][r] : acc[e][r], srow, bi, bj, r,
                                             lane);
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) red[wave][lane + 64 * s] = sums[s];
    __syncthreads();
    for (int b = tid; b < mpad; b += kDmaThreads) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kDmaWaves; ++w) t += red[w][b];
        partSum[c * mpad + b] = t;
        partShift[c * mpad + b] = shv[b];
    }
}

template <typename T, int MODE, int S>
__global__ __launch_bounds__(kDmaThreads) void cov_partial_dma_kernel(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int64_t chunk, int nb, int nblk, int mpad,
    float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow)
{
    cov_dma_body<T, MODE, S, 16, false>(Y, n, m, ld, chunk, nb, nblk, mpad, partS, partSum, partShift, srow,
                                        (int64_t)blockIdx.x, (int64_t)gridDim.x);
}

// Float32 cubes whose rows are not whole 16-byte pieces (any band count, any
// row pitch): the same kernel with 4-byte copies.
template <int MODE, int S>
__global__ __launch_bounds__(kDmaThreads) void cov_partial_dma4_kernel(
    const float *__restrict__ Y, int64_t n, int m, int64_t ld, int64_t chunk, int nb, int nblk, int mpad,
    float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow)
{
    cov_dma_body<float, MODE, S, 4, false>(Y, n, m, ld, chunk, nb, nblk, mpad, partS, partSum, partShift, srow,
                                           (int64_t)blockIdx.x, (int64_t)gridDim.x);
}

// ---- band-sequential cubes: Y[b * ld + p] --------------------------------
//
// The same chunk algorithm for cubes stored band by band (the layout of the
// paper's GPU design, Section 4: BANDS x PIXELS, a band's pixels contiguous).
// A stage is the chunk's next 32 pixels of every band, read row by row (16
// lanes x 2 pixels cover one band's 32 pixels), and is already band-major,
// the operand layout of the products, so centring and splitting are
// elementwise: thread t holds pixels 2 (t mod 16), +1 of bands t / 16 + 32 j.
// Loads run one stage ahead in registers. 8 waves; block ownership and the
// bf16 products are those of cov_partial_dma_kernel (slot e of wave w: block
// id idbase + 8 e + w), the float32 products read a band-major tile (pitch
// 34 floats: the two half-waves of an operand read land on disjoint banks).
// The float32 form keeps at most 3 slots (its two-level accumulators must
// stay in registers) and covers wider matrices in several passes over the
// cube, each with its own range of block ids.
constexpr int kBsqPitchF = 34;

template <typename T, int MODE, int S>
__device__ __forceinline__ void cov_bsq_body(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int64_t chunk, int nb, int nblk, int mpad, int idbase,
    float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow, int64_t c)
{
    constexpr int kHalf = 256 * kBfPitch;
    __shared__ __attribute__((aligned(16))) float tileF[MODE == MODE_F32 ? 256 * kBsqPitchF : 4];
    __shared__ __attribute__((aligned(16))) __bf16 hl[MODE == MODE_F32 ? 8 : 2 * kHalf];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pp = tid & 15;      // pixel pair within a stage
    const int bg = tid >> 4;      // band group: bands bg + 32 j
    const int64_t pbeg = c * chunk;
    const int64_t pend = (pbeg + chunk < n) ? pbeg + chunk : n;
    const int64_t nst = (pend - pbeg + KT - 1) / KT;

    // Shift: the cube's shift row, per band.
    float sh[8], scj[8];
    double sums[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int b = bg + 32 * j;
        sh[j] = b < m ? srow[b] : 0.f;
        scj[j] = (MODE == MODE_FP16X3 && b < mpad) ? srow[kScaleRow + b] : 1.f;
        sums[j] = 0.0;
    }

    constexpr bool kTwoLevel = MODE == MODE_F32;
    constexpr int kSlots2 = kTwoLevel ? S : 1;
    f32x16 acc[S], acc2[kSlots2];
#pragma unroll
    for (int e = 0; e < S; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[e][r] = 0.f;
    }
#pragma unroll
    for (int e = 0; e < kSlots2; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[e][r] = 0.f;
    }
    const int nbl = nb * (nb + 1) / 2;
    // Slots that hold a block (a prefix: the ids grow with the slot).
    const int nrem = nbl - idbase - wave;
    const int nslots = nrem <= 0 ? 0 : ((nrem + kDmaWaves - 1) / kDmaWaves < S ? (nrem + kDmaWaves - 1) / kDmaWaves : S);
    int offI[S], offJ[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
        int bi = 0, bj = 0;
        if (idbase + kDmaWaves * e + wave < nbl) block_of_id(idbase + kDmaWaves * e + wave, bi, bj);
        if constexpr (MODE == MODE_F32) {
            offI[e] = (32 * bi + (lane & 31)) * kBsqPitchF + (lane >> 5);
            offJ[e] = (32 * bj + (lane & 31)) * kBsqPitchF + (lane >> 5);
        } else {
            offI[e] = (32 * bi + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
            offJ[e] = (32 * bj + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
        }
    }

    // Raw values of stage st for this thread (pixels past the chunk end and
    // bands past the last one read as the shift, so they centre to zero).
    auto load = [&](float (&v)[16], int64_t st) {
        const int64_t p0 = pbeg + st * KT + 2 * pp;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = bg + 32 * j;
            const T *row = Y + (int64_t)(b < m ? b : 0) * ld;
            v[2 * j] = (b < m && p0 < pend) ? load_elem(row + p0) : sh[j];
            v[2 * j + 1] = (b < m && p0 + 1 < pend) ? load_elem(row + p0 + 1) : sh[j];
        }
    };

    auto stage = [&](const float (&v)[16], int64_t st) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = bg + 32 * j;
            const float x0 = v[2 * j] - sh[j], x1 = v[2 * j + 1] - sh[j];
            sums[j] += (double)(x0 + x1);
            if (b < mpad) {
                if constexpr (MODE == MODE_F32) {
                    *reinterpret_cast<f32x2 *>(&tileF[b * kBsqPitchF + 2 * pp]) = f32x2{x0, x1};
                } else {
                    const f32x2 xv = {x0, x1};
                    bf16x2 hh, ll;
                    split2<MODE>(xv, scj[j], hh, ll);
                    *reinterpret_cast<bf16x2 *>(&hl[b * kBfPitch + 2 * pp]) = hh;
                    *reinterpret_cast<bf16x2 *>(&hl[kHalf + b * kBfPitch + 2 * pp]) = ll;
                }
            }
        }
        __syncthreads();
        if constexpr (MODE == MODE_F32) {
#pragma unroll 2
            for (int kk = 0; kk < KT / 2; ++kk) {
#pragma unroll
                for (int e = 0; e < S; ++e)
                    acc[e] = __builtin_amdgcn_mfma_f32_32x32x2f32(tileF[offI[e] + 2 * kk], tileF[offJ[e] + 2 * kk],
                                                                 acc[e], 0, 0, 0);
            }
            if ((st + 1) % kFlush == 0) {
#pragma unroll
                for (int e = 0; e < S; ++e) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) { acc2[e][r] += acc[e][r]; acc[e][r] = 0.f; }
                }
            }
        } else {
            split_block_products<MODE, S>(hl, offI, offJ, acc, nslots);
        }
        __syncthreads();
    };

    float va[16], vb[16];
    load(va, 0);
    for (int64_t st = 0; st < nst; st += 2) {
        if (st + 1 < nst) load(vb, st + 1);
        stage(va, st);
        if (st + 1 < nst) {
            if (st + 2 < nst) load(va, st + 2);
            stage(vb, st + 1);
        }
    }

#pragma unroll
    for (int e = 0; e < S; ++e) {
        if (idbase + kDmaWaves * e + wave < nbl) {
            int bi, bj;
            block_of_id(idbase + kDmaWaves * e + wave, bi, bj);
            float *dst = partS + ((c * nblk + compact_block(bi, bj, nb)) * 16) * 64 + lane;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                dst[r * 64] = unscaled<MODE>(kTwoLevel ? acc2[e % kSlots2][r] + acc[e][r] : acc[e][r], srow, bi, bj, r,
                                             lane);
        }
    }
    // Band sums: the 16 threads of a band group (consecutive lanes) hold
    // different pixels of the same bands.
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double t = sums[j];
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) t += __shfl_xor(t, o, 16);
        const int b = bg + 32 * j;
        if (pp == 0 && b < mpad) {
            partSum[c * mpad + b] = t;
            partShift[c * mpad + b] = sh[j];
        }
    }
}

template <typename T, int MODE, int S>
__global__ __launch_bounds__(kDmaThreads) void cov_partial_bsq_kernel(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int64_t chunk, int nb, int nblk, int mpad, int idbase,
    float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow)
{
    cov_bsq_body<T, MODE, S>(Y, n, m, ld, chunk, nb, nblk, mpad, idbase, partS, partSum, partShift, srow,
                             (int64_t)blockIdx.x);
}

// Band-sequential cubes with 16-byte aligned band rows (ld and the pixel
// count multiples of 16 bytes' worth of pixels), split-bfloat16 forms: the
// stages are copied straight into LDS, as in cov_partial_dma_kernel. A copy
// moves 16 bytes a lane, kPix pixels (4 float32 or 8 uint16): lane l takes
// band kRows q + l / (32 / kPix), pixels kPix (l mod (32 / kPix)) onwards,
// landing at slot + 16 l bytes, so one copy is kRows = 2 kPix band rows of
// the stage's 32 pixels; 256 / kRows copies a stage, shared by the 8 waves.
// A ring slot holds 256 band rows x 32 pixels, band-major like the tiles;
// centring and the split then read LDS. Bands past the last one and pixels
// past the chunk (or copied from its start in their place) are masked to
// zero.
template <typename T, int MODE, int S>
__global__ __launch_bounds__(kDmaThreads) void cov_partial_bsq_dma_kernel(
    const T *__restrict__ Y, int64_t n, int m, int64_t ld, int64_t chunk, int nb, int nblk, int mpad,
    float *__restrict__ partS, double *__restrict__ partSum, float *__restrict__ partShift,
    const float *__restrict__ srow)
{
    static_assert(MODE != MODE_F32, "split forms only");
    constexpr int kPix = 16 / (int)sizeof(T);        // pixels per lane and copy
    constexpr int kLanesPerRow = KT / kPix;          // 8 (float32) or 4 (uint16)
    constexpr int kRows = 64 / kLanesPerRow;         // band rows per copy
    constexpr int kBsqCopies = 256 / kRows / kDmaWaves;   // copies per wave per stage: 4 or 2
    constexpr int kHalf = 256 * kBfPitch;
    constexpr int kSlot = 256 * KT;
    __shared__ __attribute__((aligned(16))) T raw0[kSlot];
    __shared__ __attribute__((aligned(16))) T raw1[kSlot];
    __shared__ __attribute__((aligned(16))) T raw2[kSlot];
    __shared__ __attribute__((aligned(16))) __bf16 hl[2 * kHalf];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pp = tid & 15;      // pixel pair within a stage
    const int bg = tid >> 4;      // band group: bands bg + 32 j
    const int64_t c = blockIdx.x;
    const int64_t pbeg = c * chunk;
    const int64_t pend = (pbeg + chunk < n) ? pbeg + chunk : n;
    const int64_t nst = (pend - pbeg + KT - 1) / KT;
    // Staggered walk over the chunk's stages (see cov_partial_dma_kernel).
    const int64_t rot = (c * nst) / gridDim.x;
    auto first_pixel = [&](int64_t t) -> int64_t {
        const int64_t tt = t < nst ? (t + rot < nst ? t + rot : t + rot - nst) : 0;
        return pbeg + tt * KT;
    };

    float sh[8], scj[8];
    double sums[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int b = bg + 32 * j;
        sh[j] = b < m ? srow[b] : 0.f;
        scj[j] = (MODE == MODE_FP16X3 && b < mpad) ? srow[kScaleRow + b] : 1.f;
        sums[j] = 0.0;
    }
    asm volatile("" ::: "memory");   // the shift loads stay ahead of the copies

    auto issue = [&](T *R, int64_t t) {
        const int64_t p = first_pixel(t) + kPix * (lane % kLanesPerRow);
#pragma unroll
        for (int i = 0; i < kBsqCopies; ++i) {
            const int q = wave + kDmaWaves * i;                 // copy index: band rows kRows q onwards
            const int b = kRows * q + lane / kLanesPerRow;
            const bool ok = t < nst && b < m && p < pend;      // p < pend <= n, p and n multiples of kPix
            const T *src = ok ? Y + (int64_t)b * ld + p : Y;
            // (void pointers: the host pass drops kernels whose target
            // builtins take arguments of template-dependent type)
            __builtin_amdgcn_global_load_lds(static_cast<const void *>(src),
                                             static_cast<void *>(R + kRows * q * KT), 16, 0, 0);
        }
    };

    f32x16 acc[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[e][r] = 0.f;
    }
    const int nbl = nb * (nb + 1) / 2;
    // Slots that hold a block (a prefix: the ids grow with the slot).
    const int nslots = nbl - wave <= 0 ? 0 : ((nbl - wave + kDmaWaves - 1) / kDmaWaves < S ? (nbl - wave + kDmaWaves - 1) / kDmaWaves : S);
    int offI[S], offJ[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
        int bi = 0, bj = 0;
        if (kDmaWaves * e + wave < nbl) block_of_id(kDmaWaves * e + wave, bi, bj);
        offI[e] = (32 * bi + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
        offJ[e] = (32 * bj + (lane & 31)) * kBfPitch + 8 * (lane >> 5);
    }

    auto centre = [&](const T *R, int64_t t) {
        const int64_t p0 = first_pixel(t) + 2 * pp;
        const bool v0 = t < nst && p0 < pend, v1 = t < nst && p0 + 1 < pend;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = bg + 32 * j;
            if (b >= mpad) continue;
            float r0, r1;
            if constexpr (sizeof(T) == 4) {
                const f32x2 raw = *reinterpret_cast<const f32x2 *>(&R[b * KT + 2 * pp]);
                r0 = raw[0];
                r1 = raw[1];
            } else {
                const uint32_t w = *reinterpret_cast<const uint32_t *>(&R[b * KT + 2 * pp]);
                r0 = (float)(w & 0xffffu);
                r1 = (float)(w >> 16);
            }
            const float x0 = (b < m && v0) ? r0 - sh[j] : 0.f;
            const float x1 = (b < m && v1) ? r1 - sh[j] : 0.f;
            sums[j] += (double)(x0 + x1);
            const f32x2 xv = {x0, x1};
            bf16x2 hh, ll;
            split2<MODE>(xv, scj[j], hh, ll);
            *reinterpret_cast<bf16x2 *>(&hl[b * kBfPitch + 2 * pp]) = hh;
            *reinterpret_cast<bf16x2 *>(&hl[kHalf + b * kBfPitch + 2 * pp]) = ll;
        }
    };

    auto products = [&]() { split_block_products<MODE, S>(hl, offI, offJ, acc, nslots); };

    // Wait for this stage's copies, barrier, start the copies two stages
    // ahead into the slot read last step, centre and split, barrier,
    // multiply (one tile set; cov_partial_dma_kernel's split forms keep two
    // and need one barrier a stage).
    auto step = [&](T *cur, T *nxt, int64_t st) {
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(kBsqCopies));
        lds_barrier();
        issue(nxt, st + 2);
        centre(cur, st);
        lds_barrier();
        products();
    };

    issue(raw0, 0);
    issue(raw1, 1);
    for (int64_t st = 0; st < nst; st += kRing) {
        step(raw0, raw2, st);
        step(raw1, raw0, st + 1);
        step(raw2, raw1, st + 2);
    }
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    __syncthreads();

#pragma unroll
    for (int e = 0; e < S; ++e) {
        if (kDmaWaves * e + wave < nbl) {
            int bi, bj;
            block_of_id(kDmaWaves * e + wave, bi, bj);
            float *dst = partS + ((c * nblk + compact_block(bi, bj, nb)) * 16) * 64 + lane;
#pragma unroll
            for (int r = 0; r < 16; ++r) dst[r * 64] = unscaled<MODE>(acc[e][r], srow, bi, bj, r, lane);
        }
    }
    // Band sums: the 16 threads of a band group (consecutive lanes) hold
    // different pixels of the same bands.
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double t = sums[j];
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) t += __shfl_xor(t, o, 16);
        const int b = bg + 32 * j;
        if (pp == 0 && b < mpad) {
            partSum[c * mpad + b] = t;
            partShift[c * mpad + b] = sh[j];
        }
    }
}

// Pass 2a: grid (block, chunk group). Every workgroup forms the band means of
// its block's 64 bands (all chunks, float64, fixed order: identical in every
// workgroup), then the centred second moment of its range of chunks.
__device__ __forceinline__ void cov_finalize_part_body(
    int64_t n, int m, int centered, int64_t chunk, int64_t nchunks, int nb, int nblk, int mpad,
    const float *__restrict__ partS, const double *__restrict__ partSum, const float *__restrict__ partShift,
    double *__restrict__ part2, int e, int gi, int G)
{
    constexpr int kBatch = 32;
    __shared__ double mu[64];
    __shared__ double mred[16][64];
    __shared__ float shv[kBatch][64];
    __shared__ double smv[kBatch][64];

    int bi = 0, rem = e;
    while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
    const int bj = bi + rem;
    const int tid = threadIdx.x;
    const int r = tid >> 6, lane = tid & 63;
    const int il = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);   // MFMA 32x32 result layout
    const int jl = lane & 31;
    auto band = [&](int q) { return q < 32 ? 32 * bi + q : 32 * bj + (q - 32); };
    auto pixels = [&](int64_t w) { return (double)((w * chunk + chunk < n ? w * chunk + chunk : n) - w * chunk); };

    {
        const int b = band(lane);
        const int64_t w0 = (int64_t)r * nchunks / 16, w1 = (int64_t)(r + 1) * nchunks / 16;
        double a = 0.0;
        if (b < m && !centered) {
            // Eight chunks' loads in flight at once, added in chunk order.
            for (int64_t w = w0; w < w1; w += 8) {
                float hv[8];
                double sv8[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int64_t wi = w + i < w1 ? w + i : w0;
                    hv[i] = partShift[wi * mpad + b];
                    sv8[i] = partSum[wi * mpad + b];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (w + i < w1) a += pixels(w + i) * (double)hv[i] + sv8[i];
            }
        }
        mred[r][lane] = a;
    }
    __syncthreads();
    if (tid < 64) {
        double a = 0.0;
        for (int w = 0; w < 16; ++w) a += mred[w][tid];
        mu[tid] = (band(tid) < m && !centered) ? a / (double)n : 0.0;
    }
    __syncthreads();

    const int64_t c0 = (int64_t)gi * nchunks / G, c1 = (int64_t)(gi + 1) * nchunks / G;
    double acc = 0.0;
    for (int64_t w0 = c0; w0 < c1; w0 += kBatch) {
        const int nbatch = (int)((c1 - w0) < kBatch ? (c1 - w0) : kBatch);
        for (int t = tid; t < kBatch * 64; t += 1024) {
            const int cc = t >> 6, q = t & 63;
            const int b = band(q);
            const bool ok = cc < nbatch && b < mpad;
            const int64_t w = ok ? w0 + cc : 0;
            const int bb = ok ? b : 0;
            const double sm = partSum[w * mpad + bb];
            const float sh = partShift[w * mpad + bb];
            smv[cc][q] = ok ? sm : 0.0;
            shv[cc][q] = ok ? sh : 0.f;   // any shift is exact algebra; centred cubes may store one too
        }
        float sv[kBatch];
#pragma unroll
        for (int cc = 0; cc < kBatch; ++cc) {
            const int64_t w = cc < nbatch ? w0 + cc : w0;
            sv[cc] = partS[(w * nblk + e) * 1024 + tid];
        }
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < kBatch; ++cc) {
            if (cc < nbatch) {
                const double nw = pixels(w0 + cc);
                const double ei = (double)shv[cc][il] - mu[il];
                const double ej = (double)shv[cc][32 + jl] - mu[32 + jl];
                acc += (double)sv[cc] + smv[cc][il] * ej + ei * smv[cc][32 + jl] + nw * ei * ej;
            }
        }
        __syncthreads();
    }
    part2[((int64_t)gi * nblk + e) * 1024 + tid] = acc;
    if (gi == 0 && e == 0 && tid == 0) part2[(int64_t)G * nblk * 1024] = 0.0;   // unused pad
    if (gi == 0 && bi == bj && tid < 32) part2[(int64_t)G * nblk * 1024 + 1 + 32 * bi + tid] = mu[tid];
}

__global__ __launch_bounds__(1024) void cov_finalize_part_kernel(
    int64_t n, int m, int centered, int64_t chunk, int64_t nchunks, int nb, int nblk, int mpad,
    const float *__restrict__ partS, const double *__restrict__ partSum, const float *__restrict__ partShift,
    double *__restrict__ part2)
{
    cov_finalize_part_body(n, m, centered, chunk, nchunks, nb, nblk, mpad, partS, partSum, partShift, part2,
                           (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.y);
}

// Pass 2b: the chunk groups added in order, divided by N - 1, mirrored.
__device__ __forceinline__ void cov_finalize_sum_body(int64_t n, int m, int centered, int nb, int nblk, int G,
                                             const double *__restrict__ part2, float *__restrict__ C,
                                             float *__restrict__ mean, int e)
{
    int bi = 0, rem = e;
    while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
    const int bj = bi + rem;
    const int tid = threadIdx.x;
    const int r = tid >> 6, lane = tid & 63;
    const int il = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int jl = lane & 31;
    double acc = 0.0;
    for (int gi = 0; gi < G; ++gi) acc += part2[((int64_t)gi * nblk + e) * 1024 + tid];
    const int i = 32 * bi + il, j = 32 * bj + jl;
    if (i < m && j < m && !(bi == bj && i > j)) {
        const float val = (float)(acc / (double)(n - 1));
        C[(int64_t)i * m + j] = val;
        C[(int64_t)j * m + i] = val;
    }
    if (mean && !centered && bi == bj && tid < 32 && 32 * bi + tid < m)
        mean[32 * bi + tid] = (float)part2[(int64_t)G * nblk * 1024 + 1 + 32 * bi + tid];
}

__global__ __launch_bounds__(1024) void cov_finalize_sum_kernel(int64_t n, int m, int centered, int nb, int nblk,
                                                                int G, const double *__restrict__ part2,
                                                                float *__restrict__ C, float *__restrict__ mean)
{
    cov_finalize_sum_body(n, m, centered, nb, nblk, G, part2, C, mean, (int)blockIdx.x);
}

// ---- batched form: task table in the workspace (see kernels.hpp) ----------
__device__ inline const BatchCube *batch_table(const char *ws)
{
    return reinterpret_cast<const BatchCube *>(ws + sizeof(BatchHeader));
}

// Cube whose range of work items [w, w + count) holds `item` (entries are
// sorted by their first item).
template <int64_t BatchCube::*W>
__device__ inline int batch_find(const BatchCube *t, int nc, int64_t item)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (t[mid].*W <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Persistent: workgroups take (cube, chunk) items from a queue until it is
// empty; each item's results land in fixed slots, so the order in which
// items are taken does not change them.
// Shift rows of every cube of a batch: workgroup (bb, r) takes band block bb
// of the cube at table position r.
template <typename T>
__global__ __launch_bounds__(kShiftThreads) void cov_shift_batched_kernel(const char *ws, int bsq)
{
    const BatchCube &cb = batch_table(ws)[blockIdx.y];
    if ((int)blockIdx.x >= cb.cov.nb) return;
    cov_shift_body<T>(static_cast<const T *>(cb.Y), cb.n, cb.m, cb.ld, bsq != 0, (int)blockIdx.x, cb.srow);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void cov_partial_batched_kernel(char *ws, int nc, int64_t total)
{
    __shared__ int64_t item_sh;
    BatchHeader *h = reinterpret_cast<BatchHeader *>(ws);
    const BatchCube *t = batch_table(ws);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(&h->counter[0], 1u);
        __syncthreads();
        const int64_t item = item_sh;
        if (item >= total) break;
        const BatchCube &cb = t[batch_find<&BatchCube::w_cov>(t, nc, item)];
        cov_partial_body<T, 1, MODE, kMaxSlots, true>(static_cast<const T *>(cb.Y), cb.n, cb.m, cb.ld, 0,
                                                      cb.cov.chunk, cb.cov.nb, cb.cov.nblk, cb.cov.mpad, cb.partS,
                                                      cb.partSum, cb.partShift, cb.srow, item - cb.w_cov);
    }
}

// Float32 cubes of the batch: the same queue over the 4-byte-copy chunk
// kernel, with the slot count of each item's cube.
template <int MODE>
__global__ __launch_bounds__(kDmaThreads) void cov_partial_batched_dma_kernel(char *ws, int nc, int64_t total)
{
    __shared__ int64_t item_sh;
    BatchHeader *h = reinterpret_cast<BatchHeader *>(ws);
    const BatchCube *t = batch_table(ws);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(&h->counter[0], 1u);
        __syncthreads();
        const int64_t item = item_sh;
        if (item >= total) break;
        const BatchCube &cb = t[batch_find<&BatchCube::w_cov>(t, nc, item)];
#define PCA_BATCH_BODY(S)                                                                                          \
    cov_dma_body<float, MODE, S, 4, true>(static_cast<const float *>(cb.Y), cb.n, cb.m, cb.ld, cb.cov.chunk, cb.cov.nb, \
                                          cb.cov.nblk, cb.cov.mpad, cb.partS, cb.partSum, cb.partShift, cb.srow,       \
                                          item - cb.w_cov, cb.cov.nchunks)
        switch (dma_slots(cb.cov.nb)) {
        case 2: PCA_BATCH_BODY(2); break;
        case 3: PCA_BATCH_BODY(3); break;
        case 4: PCA_BATCH_BODY(4); break;
        default: PCA_BATCH_BODY(5); break;
        }
#undef PCA_BATCH_BODY
    }
}

// Band-sequential cubes of the batch: the same queue over the register-staged
// band-sequential chunk body, three slots a wave; a cube of more than 24
// blocks takes its chunk in several passes (block ids 24 apart).
template <typename T, int MODE>
__global__ __launch_bounds__(kDmaThreads) void cov_partial_batched_bsq_kernel(char *ws, int nc, int64_t total)
{
    __shared__ int64_t item_sh;
    BatchHeader *h = reinterpret_cast<BatchHeader *>(ws);
    const BatchCube *t = batch_table(ws);
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(&h->counter[0], 1u);
        __syncthreads();
        const int64_t item = item_sh;
        if (item >= total) break;
        const BatchCube &cb = t[batch_find<&BatchCube::w_cov>(t, nc, item)];
        for (int idbase = 0; idbase < cb.cov.nblk; idbase += 3 * kDmaWaves)
            cov_bsq_body<T, MODE, 3>(static_cast<const T *>(cb.Y), cb.n, cb.m, cb.ld, cb.cov.chunk, cb.cov.nb,
                                     cb.cov.nblk, cb.cov.mpad, idbase, cb.partS, cb.partSum, cb.partShift, cb.srow,
                                     item - cb.w_cov);
    }
}

__global__ __launch_bounds__(1024) void cov_finalize_part_batched_kernel(const char *ws, int nc)
{
    const BatchCube *t = batch_table(ws);
    const int64_t item = blockIdx.x;
    const BatchCube &cb = t[batch_find<&BatchCube::w_fin1>(t, nc, item)];
    const int64_t local = item - cb.w_fin1;
    cov_finalize_part_body(cb.n, cb.m, 0, cb.cov.chunk, cb.cov.nchunks, cb.cov.nb, cb.cov.nblk, cb.cov.mpad, cb.partS,
                           cb.partSum, cb.partShift, cb.part2, (int)(local % cb.cov.nblk), (int)(local / cb.cov.nblk),
                           cb.cov.groups);
}

__global__ __launch_bounds__(1024) void cov_finalize_sum_batched_kernel(const char *ws, int nc)
{
    const BatchCube *t = batch_table(ws);
    const int64_t item = blockIdx.x;
    const BatchCube &cb = t[batch_find<&BatchCube::w_fin2>(t, nc, item)];
    cov_finalize_sum_body(cb.n, cb.m, 0, cb.cov.nb, cb.cov.nblk, cb.cov.groups, cb.part2, cb.C, cb.mean,
                          (int)(item - cb.w_fin2));
}

template <typename T, int VEC, int MODE>
hipError_t launch_partial_m(const T *Y, int64_t n, int m, int64_t ld, int centered, const CovPlan &p,
                            float *partS, double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    dim3 grid((unsigned)p.nchunks), block(kThreads);
    switch (cov_slots(p.nb)) {
    case 3:
        hipLaunchKernelGGL((cov_partial_kernel<T, VEC, MODE, 3>), grid, block, 0, st, Y, n, m, ld, centered, p.chunk,
                           p.nb, p.nblk, p.mpad, partS, partSum, partShift, srow);
        break;
    case 6:
        hipLaunchKernelGGL((cov_partial_kernel<T, VEC, MODE, 6>), grid, block, 0, st, Y, n, m, ld, centered, p.chunk,
                           p.nb, p.nblk, p.mpad, partS, partSum, partShift, srow);
        break;
    case 7:
        hipLaunchKernelGGL((cov_partial_kernel<T, VEC, MODE, 7>), grid, block, 0, st, Y, n, m, ld, centered, p.chunk,
                           p.nb, p.nblk, p.mpad, partS, partSum, partShift, srow);
        break;
    default:
        hipLaunchKernelGGL((cov_partial_kernel<T, VEC, MODE, kMaxSlots>), grid, block, 0, st, Y, n, m, ld, centered,
                           p.chunk, p.nb, p.nblk, p.mpad, partS, partSum, partShift, srow);
        break;
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_dma_m(const T *Y, int64_t n, int m, int64_t ld, const CovPlan &p, float *partS,
                        double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    dim3 grid((unsigned)p.nchunks), block(kDmaThreads);
    switch (dma_slots(p.nb)) {
    case 2:
        hipLaunchKernelGGL((cov_partial_dma_kernel<T, MODE, 2>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.nb, p.nblk,
                           p.mpad, partS, partSum, partShift, srow);
        break;
    case 3:
        hipLaunchKernelGGL((cov_partial_dma_kernel<T, MODE, 3>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.nb, p.nblk,
                           p.mpad, partS, partSum, partShift, srow);
        break;
    case 4:
        hipLaunchKernelGGL((cov_partial_dma_kernel<T, MODE, 4>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.nb, p.nblk,
                           p.mpad, partS, partSum, partShift, srow);
        break;
    default:
        hipLaunchKernelGGL((cov_partial_dma_kernel<T, MODE, 5>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.nb, p.nblk,
                           p.mpad, partS, partSum, partShift, srow);
        break;
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_dma4_m(const float *Y, int64_t n, int m, int64_t ld, const CovPlan &p, float *partS,
                         double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    const dim3 grid((unsigned)p.nchunks), block(kDmaThreads);
#define PCA_DMA4(S)                                                                                                \
    hipLaunchKernelGGL((cov_partial_dma4_kernel<MODE, S>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.nb, p.nblk, \
                       p.mpad, partS, partSum, partShift, srow)
    switch (dma_slots(p.nb)) {
    case 2: PCA_DMA4(2); break;
    case 3: PCA_DMA4(3); break;
    case 4: PCA_DMA4(4); break;
    default: PCA_DMA4(5); break;
    }
#undef PCA_DMA4
    return hipGetLastError();
}

template <typename T, int MODE, int S>
void launch_bsq_s(const T *Y, int64_t n, int m, int64_t ld, const CovPlan &p, int idbase, float *partS,
                  double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    hipLaunchKernelGGL((cov_partial_bsq_kernel<T, MODE, S>), dim3((unsigned)p.nchunks), dim3(kDmaThreads), 0, st, Y, n,
                       m, ld, p.chunk, p.nb, p.nblk, p.mpad, idbase, partS, partSum, partShift, srow);
}

template <typename T, int MODE>
hipError_t launch_bsq_m(const T *Y, int64_t n, int m, int64_t ld, const CovPlan &p, float *partS, double *partSum,
                        float *partShift, const float *srow, hipStream_t st)
{
    const int slots = dma_slots(p.nb);
    if (MODE == MODE_F32 && slots > 3) {
        for (int base = 0; base < p.nblk; base += 3 * kDmaWaves)
            launch_bsq_s<T, MODE, 3>(Y, n, m, ld, p, base, partS, partSum, partShift, srow, st);
        return hipGetLastError();
    }
    switch (slots) {
    case 2: launch_bsq_s<T, MODE, 2>(Y, n, m, ld, p, 0, partS, partSum, partShift, srow, st); break;
    case 3: launch_bsq_s<T, MODE, 3>(Y, n, m, ld, p, 0, partS, partSum, partShift, srow, st); break;
    case 4:
        if constexpr (MODE != MODE_F32) launch_bsq_s<T, MODE, 4>(Y, n, m, ld, p, 0, partS, partSum, partShift, srow, st);
        break;
    default:
        if constexpr (MODE != MODE_F32) launch_bsq_s<T, MODE, 5>(Y, n, m, ld, p, 0, partS, partSum, partShift, srow, st);
        break;
    }
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_bsq_dma_m(const T *Y, int64_t n, int m, int64_t ld, const CovPlan &p, float *partS,
                            double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    const dim3 grid((unsigned)p.nchunks), block(kDmaThreads);
#define PCA_BSQ_DMA(S)                                                                                             \
    hipLaunchKernelGGL((cov_partial_bsq_dma_kernel<T, MODE, S>), grid, block, 0, st, Y, n, m, ld, p.chunk, p.nb,   \
                       p.nblk, p.mpad, partS, partSum, partShift, srow)
    switch (dma_slots(p.nb)) {
    case 2: PCA_BSQ_DMA(2); break;
    case 3: PCA_BSQ_DMA(3); break;
    case 4: PCA_BSQ_DMA(4); break;
    default: PCA_BSQ_DMA(5); break;
    }
#undef PCA_BSQ_DMA
    return hipGetLastError();
}

// Band-sequential cubes whose band rows can be copied 16 bytes a lane
// (pixels per 16 bytes: 4 float32, 8 uint16).
inline bool bsq_dma_ok(const void *Y, int elem_bytes, int mode, int64_t n, int64_t ld)
{
    const int64_t per = 16 / elem_bytes;
    return mode != MODE_F32 && (reinterpret_cast<uintptr_t>(Y) % 16 == 0) && (ld % per == 0) && (n % per == 0);
}

template <typename T>
hipError_t launch_partial_bsq(const T *Y, int64_t n, int m, int64_t ld, int mode, const CovPlan &p, float *partS,
                              double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    if (bsq_dma_ok(Y, (int)sizeof(T), mode, n, ld)) {
        if (mode == MODE_BF16X3) return launch_bsq_dma_m<T, MODE_BF16X3>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
        if (mode == MODE_FP16X3) return launch_bsq_dma_m<T, MODE_FP16X3>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
        return launch_bsq_dma_m<T, MODE_BF16X4>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    }
    switch (mode) {
    case MODE_F32: return launch_bsq_m<T, MODE_F32>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    case MODE_BF16X3: return launch_bsq_m<T, MODE_BF16X3>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    case MODE_FP16X3: return launch_bsq_m<T, MODE_FP16X3>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    default: return launch_bsq_m<T, MODE_BF16X4>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    }
}

template <typename T>
hipError_t launch_partial_dma(const T *Y, int64_t n, int m, int64_t ld, int mode, const CovPlan &p,
                              float *partS, double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    switch (mode) {
    case MODE_F32: return launch_dma_m<T, MODE_F32>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    case MODE_BF16X3: return launch_dma_m<T, MODE_BF16X3>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    case MODE_FP16X3: return launch_dma_m<T, MODE_FP16X3>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    default: return launch_dma_m<T, MODE_BF16X4>(Y, n, m, ld, p, partS, partSum, partShift, srow, st);
    }
}

// Rows that the 16-byte copies can stage: 16-byte aligned, with whole lanes
// (4 float32 or 8 uint16 bands) per row.
inline bool dma_ok(const void *Y, int dt, int m, int64_t ld)
{
    const int per = dt == PCA_IN_F32 ? 4 : 8;
    return (reinterpret_cast<uintptr_t>(Y) % 16 == 0) && m % per == 0 && ld % per == 0;
}

template <typename T, int VEC>
hipError_t launch_partial_t(const T *Y, int64_t n, int m, int64_t ld, int centered, int mode,
                            const CovPlan &p, float *partS, double *partSum, float *partShift, const float *srow, hipStream_t st)
{
    switch (mode) {
    case MODE_F32:
        return launch_partial_m<T, VEC, MODE_F32>(Y, n, m, ld, centered, p, partS, partSum, partShift, srow, st);
    case MODE_BF16X3:
        return launch_partial_m<T, VEC, MODE_BF16X3>(Y, n, m, ld, centered, p, partS, partSum, partShift, srow, st);
    case MODE_FP16X3:
        return launch_partial_m<T, VEC, MODE_FP16X3>(Y, n, m, ld, centered, p, partS, partSum, partShift, srow, st);
    default:
        return launch_partial_m<T, VEC, MODE_BF16X4>(Y, n, m, ld, centered, p, partS, partSum, partShift, srow, st);
    }
}

}  // namespace

CovPlan cov_plan(int64_t n, int m)
{
    int64_t target = (n + kCovTargetChunks - 1) / kCovTargetChunks;
    target = (target + KT - 1) / KT * KT;
    return cov_plan_chunk(n, m, target < KT ? KT : target);
}

hipError_t launch_cov_shift(const void *Y, int dt, int64_t n, int m, int64_t ld, const CovPlan &plan, float *srow,
                            hipStream_t st)
{
    const dim3 grid((unsigned)plan.nb), block(kShiftThreads);
    const int bsq = (dt == PCA_IN_F32_BSQ || dt == PCA_IN_U16_BSQ) ? 1 : 0;
    if (dt == PCA_IN_F32 || dt == PCA_IN_F32_BSQ)
        hipLaunchKernelGGL(cov_shift_kernel<float>, grid, block, 0, st, static_cast<const float *>(Y), n, m, ld, bsq,
                           srow);
    else
        hipLaunchKernelGGL(cov_shift_kernel<uint16_t>, grid, block, 0, st, static_cast<const uint16_t *>(Y), n, m, ld,
                           bsq, srow);
    return hipGetLastError();
}

hipError_t launch_cov_partial(const void *Y, int dt, int64_t n, int m, int64_t ld, int centered,
                              int mode, const CovPlan &plan, float *partS, double *partSum,
                              float *partShift, const float *srow, hipStream_t st)
{
    if (dt == PCA_IN_F32_BSQ)
        return launch_partial_bsq(static_cast<const float *>(Y), n, m, ld, mode, plan, partS, partSum, partShift, srow, st);
    if (dt == PCA_IN_U16_BSQ)
        return launch_partial_bsq(static_cast<const uint16_t *>(Y), n, m, ld, mode, plan, partS, partSum, partShift,
                                  srow, st);
    if (dma_ok(Y, dt, m, ld)) {
        if (dt == PCA_IN_F32)
            return launch_partial_dma(static_cast<const float *>(Y), n, m, ld, mode, plan, partS, partSum, partShift,
                                      srow, st);
        return launch_partial_dma(static_cast<const uint16_t *>(Y), n, m, ld, mode, plan, partS, partSum, partShift,
                                  srow, st);
    }
    if (dt == PCA_IN_F32) {
        const float *y = static_cast<const float *>(Y);
        switch (mode) {
        case MODE_F32: return launch_dma4_m<MODE_F32>(y, n, m, ld, plan, partS, partSum, partShift, srow, st);
        case MODE_BF16X3: return launch_dma4_m<MODE_BF16X3>(y, n, m, ld, plan, partS, partSum, partShift, srow, st);
        case MODE_FP16X3: return launch_dma4_m<MODE_FP16X3>(y, n, m, ld, plan, partS, partSum, partShift, srow, st);
        default: return launch_dma4_m<MODE_BF16X4>(y, n, m, ld, plan, partS, partSum, partShift, srow, st);
        }
    }
    const bool v4 = vec4_ok(Y, dt, m, ld);
    const uint16_t *y = static_cast<const uint16_t *>(Y);
    return v4 ? launch_partial_t<uint16_t, 4>(y, n, m, ld, centered, mode, plan, partS, partSum, partShift, srow, st)
              : launch_partial_t<uint16_t, 1>(y, n, m, ld, centered, mode, plan, partS, partSum, partShift, srow, st);
}

hipError_t launch_cov_finalize(int64_t n, int m, int centered, const CovPlan &plan, const float *partS,
                               const double *partSum, const float *partShift, double *part2, float *C, float *mean,
                               hipStream_t st)
{
    hipLaunchKernelGGL(cov_finalize_part_kernel, dim3((unsigned)plan.nblk, (unsigned)plan.groups), dim3(1024), 0, st,
                       n, m, centered, plan.chunk, plan.nchunks, plan.nb, plan.nblk, plan.mpad, partS, partSum,
                       partShift, part2);
    hipLaunchKernelGGL(cov_finalize_sum_kernel, dim3((unsigned)plan.nblk), dim3(1024), 0, st, n, m, centered,
                       plan.nb, plan.nblk, plan.groups, (const double *)part2, C, mean);
    return hipGetLastError();
}

hipError_t launch_cov_batched(int dt, int mode, const char *ws, const int64_t total[6], int n_cubes, hipStream_t st)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    // Register-staged uint16 kernel: two workgroups a CU; float32 copy
    // kernel: one (its stage ring fills most of the LDS); band-sequential
    // kernel: one (eight waves of up to 256 registers).
    int64_t g = (int64_t)cus * (dt == PCA_IN_U16 ? 2 : 1);
    if (g > total[0]) g = total[0];
    if (g < 1) g = 1;
    char *w = const_cast<char *>(ws);
    const dim3 grid((unsigned)g), block(kThreads), dgrid((unsigned)g), dblock(kDmaThreads);
    const dim3 sgrid(8u, (unsigned)n_cubes);
    const int bsq = (dt == PCA_IN_F32_BSQ || dt == PCA_IN_U16_BSQ) ? 1 : 0;
    if (dt == PCA_IN_F32 || dt == PCA_IN_F32_BSQ)
        hipLaunchKernelGGL(cov_shift_batched_kernel<float>, sgrid, dim3(kShiftThreads), 0, st, ws, bsq);
    else
        hipLaunchKernelGGL(cov_shift_batched_kernel<uint16_t>, sgrid, dim3(kShiftThreads), 0, st, ws, bsq);
#define PCA_COV_B(T, M)                                                                                           \
    hipLaunchKernelGGL((cov_partial_batched_kernel<T, M>), grid, block, 0, st, w, n_cubes, total[0])
#define PCA_COV_BD(M) hipLaunchKernelGGL((cov_partial_batched_dma_kernel<M>), dgrid, dblock, 0, st, w, n_cubes, total[0])
#define PCA_COV_BB(T, M)                                                                                          \
    hipLaunchKernelGGL((cov_partial_batched_bsq_kernel<T, M>), dgrid, dblock, 0, st, w, n_cubes, total[0])
    if (dt == PCA_IN_F32_BSQ || dt == PCA_IN_U16_BSQ) {
        const bool f = dt == PCA_IN_F32_BSQ;
        if (mode == MODE_F32) { if (f) PCA_COV_BB(float, MODE_F32); else PCA_COV_BB(uint16_t, MODE_F32); }
        else if (mode == MODE_BF16X3) { if (f) PCA_COV_BB(float, MODE_BF16X3); else PCA_COV_BB(uint16_t, MODE_BF16X3); }
        else if (mode == MODE_FP16X3) { if (f) PCA_COV_BB(float, MODE_FP16X3); else PCA_COV_BB(uint16_t, MODE_FP16X3); }
        else { if (f) PCA_COV_BB(float, MODE_BF16X4); else PCA_COV_BB(uint16_t, MODE_BF16X4); }
    } else if (dt == PCA_IN_F32) {
        if (mode == MODE_F32) PCA_COV_BD(MODE_F32);
        else if (mode == MODE_BF16X3) PCA_COV_BD(MODE_BF16X3);
        else if (mode == MODE_FP16X3) PCA_COV_BD(MODE_FP16X3);
        else PCA_COV_BD(MODE_BF16X4);
    } else {
        if (mode == MODE_F32) PCA_COV_B(uint16_t, MODE_F32);
        else if (mode == MODE_BF16X3) PCA_COV_B(uint16_t, MODE_BF16X3);
        else if (mode == MODE_FP16X3) PCA_COV_B(uint16_t, MODE_FP16X3);
        else PCA_COV_B(uint16_t, MODE_BF16X4);
    }
#undef PCA_COV_B
#undef PCA_COV_BD
#undef PCA_COV_BB
    hipLaunchKernelGGL(cov_finalize_part_batched_kernel, dim3((unsigned)total[1]), dim3(1024), 0, st, ws, n_cubes);
    hipLaunchKernelGGL(cov_finalize_sum_batched_kernel, dim3((unsigned)total[2]), dim3(1024), 0, st, ws, n_cubes);
    return hipGetLastError();
}

}  // namespace pca

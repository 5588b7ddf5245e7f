/*
 * FP64 reference Jacobi eigensolver for the PCA oracle.
 *
 * TEST INFRASTRUCTURE ONLY: this file is part of the CPU oracle that the GPU
 * path is checked against. Only the tests, the smoke check and the CPU
 * baseline of the benchmark load it; the GPU library never does, and the two
 * share no code.
 *
 * It follows the Jacobi method of Section 2 of the paper:
 *   - the pivot (i, j) rotation parameters of equations (2)-(5), with the
 *     generalised m of equation (7);
 *   - the rotation matrix P of equation (6) (P_ii = P_jj = cos, P_ij = sin,
 *     P_ji = -sin);
 *   - one iteration C_k = P_k^T C P_k (equation (8)), carried out as the row
 *     update followed by the column update described for the manycore design
 *     in Section 5 (Codes 5.3.2 and 5.3.3), after which the annihilated pair
 *     is exactly zero;
 *   - the eigenvector matrix E = P_1 P_2 ... P_K accumulated column-wise
 *     (equation (10));
 *   - iteration until the off-diagonal part falls below the stop factor
 *     (equation (9) and the text around it).
 *
 * Orderings (Section 2 selects the cyclic one; the GPU design of Section 4
 * searches the largest element; the manycore design of Section 5 selects
 * greedy sets of disjoint pairs):
 *   ORD_ROW_CYCLIC  row by row over the upper triangle (the default);
 *   ORD_ROUND_ROBIN sets of n/2 disjoint pairs per round, n-1 rounds per
 *                   sweep (a round-robin tournament, "circle" construction:
 *                   index n-1 stays fixed while the others turn);
 *   ORD_CLASSICAL   the largest off-diagonal element at every rotation;
 *   ORD_GREEDY      Section 5 selection: scan the upper triangle row-wise and
 *                   take every element that is above the threshold, not yet
 *                   zeroed in this sweep and shares no row or column with an
 *                   element already taken in this iteration.
 *
 * Stop rule (the paper leaves the value of the stop factor open): the
 * relative off-norm sqrt(sum_{i != j} a_ij^2) / ||A||_F is compared with
 * `tol` before every sweep (for the greedy ordering, an element counts as
 * above the threshold when |a_ij| > tol ||A||_F / n, which implies the same
 * bound once no element is left).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORD_ROW_CYCLIC = 0, ORD_ROUND_ROBIN = 1, ORD_CLASSICAL = 2, ORD_GREEDY = 3 };

static double sum_sq_offdiag(const double *A, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) s += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    return s;
}

static double sum_sq_all(const double *A, int n)
{
    double s = 0.0;
    for (size_t e = 0; e < (size_t)n * n; ++e) s += A[e] * A[e];
    return s;
}

/*
 * Rotation parameters for the pivot (i, j), i < j, equations (2)-(5) with (7):
 *   m = 2 C_ij / (C_jj - C_ii),  t = (-1 + sqrt(1 + m^2)) / m,
 *   cos = 1 / sqrt(1 + t^2),     sin = t cos.
 * t is evaluated through theta = 1/m as t = sgn(theta) / (|theta| + sqrt(1 +
 * theta^2)), the same number without the cancellation of -1 + sqrt(1 + m^2)
 * for small m; C_ii == C_jj (m infinite) gives t = 1 (a 45 degree rotation).
 */
static void rotation_params(double aii, double ajj, double aij, double *c, double *s)
{
    double theta = (ajj - aii) / (2.0 * aij);
    double t;
    if (fabs(theta) > 1e150)
        t = 0.5 / theta;
    else
        t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
#ifdef ORACLE_MUTANT_TANGENT_SIGN
    t = -t;
#endif
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = t * (*c);
}

/*
 * C <- P^T C P for the pivot (i, j) and E <- E P.
 * Row update (P^T on the left): for every column k
 *   new a_ik = P_ii a_ik + P_ji a_jk = cos a_ik - sin a_jk
 *   new a_jk = P_ij a_ik + P_jj a_jk = sin a_ik + cos a_jk
 * Column update (P on the right): for every row k
 *   new a_ki = a_ki P_ii + a_kj P_ji = cos a_ki - sin a_kj
 *   new a_kj = a_ki P_ij + a_kj P_jj = sin a_ki + cos a_kj
 * and the same column update on the eigenvector matrix.
 */
static void apply_rotation(double *A, double *V, int n, int i, int j, double c, double s)
{
    double *ri = A + (size_t)i * n, *rj = A + (size_t)j * n;
    for (int k = 0; k < n; ++k) {
        double aik = ri[k], ajk = rj[k];
        ri[k] = c * aik - s * ajk;
        rj[k] = s * aik + c * ajk;
    }
    for (int k = 0; k < n; ++k) {
        double *rk = A + (size_t)k * n;
        double aki = rk[i], akj = rk[j];
#ifdef ORACLE_MUTANT_DROP_TERM
        rk[i] = c * aki;
#else
        rk[i] = c * aki - s * akj;
#endif
        rk[j] = s * aki + c * akj;
    }
    A[(size_t)i * n + j] = 0.0;
    A[(size_t)j * n + i] = 0.0;
    for (int k = 0; k < n; ++k) {
        double *vk = V + (size_t)k * n;
        double vki = vk[i], vkj = vk[j];
#ifdef ORACLE_MUTANT_TRANSPOSED_V
        /* rotates rows of E instead of columns: E <- P^T E */
        double *vi = V + (size_t)i * n, *vj = V + (size_t)j * n;
        double a = vi[k], b = vj[k];
        vi[k] = c * a - s * b;
        vj[k] = s * a + c * b;
        (void)vki; (void)vkj;
#else
        vk[i] = c * vki - s * vkj;
        vk[j] = s * vki + c * vkj;
#endif
    }
}

/* Rotate the pivot (i, j) unless its element is already zero. Returns 1 if a
 * rotation was applied. */
static int rotate_pivot(double *A, double *V, int n, int i, int j)
{
    if (i > j) { int t = i; i = j; j = t; }
    double aij = A[(size_t)i * n + j];
    if (aij == 0.0) return 0;
    double c, s;
    rotation_params(A[(size_t)i * n + i], A[(size_t)j * n + j], aij, &c, &s);
    apply_rotation(A, V, n, i, j, c, s);
    return 1;
}

/* Pair k of round r of an n-player round-robin (n even): player n-1 is fixed
 * and meets player r; the others are paired symmetrically around r on a
 * circle of n-1 positions. */
static void round_robin_pair(int n, int r, int k, int *a, int *b)
{
    int m = n - 1;
    if (k == 0) { *a = r; *b = m; return; }
    *a = (r + k) % m;
    *b = ((r - k) % m + m) % m;
}

/*
 * Diagonalise the symmetric n x n matrix A (row-major, overwritten by the
 * final, nearly diagonal iterate) and accumulate the eigenvectors into V
 * (row-major, column j = eigenvector j; set to the identity first).
 * Returns 1 when the stop rule was met, 0 when max_sweeps ran out.
 */
int oracle_jacobi(double *A, double *V, int n, double tol, int max_sweeps, int ordering,
                  int *sweeps_out, long long *rotations_out, double *off_rel_out)
{
    long long rotations = 0;
    int sweeps = 0, converged = 0;
    memset(V, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double fro2 = sum_sq_all(A, n);
    double lim2 = tol * tol * fro2;

    if (ordering == ORD_ROW_CYCLIC || ordering == ORD_ROUND_ROBIN) {
        for (;;) {
            if (sum_sq_offdiag(A, n) <= lim2) { converged = 1; break; }
            if (sweeps >= max_sweeps) break;
            if (ordering == ORD_ROW_CYCLIC) {
                for (int i = 0; i < n - 1; ++i)
                    for (int j = i + 1; j < n; ++j)
                        rotations += rotate_pivot(A, V, n, i, j);
            } else {
                int ne = n + (n & 1); /* odd n: a phantom player n that is skipped */
                for (int r = 0; r < ne - 1; ++r)
                    for (int k = 0; k < ne / 2; ++k) {
                        int a, b;
                        round_robin_pair(ne, r, k, &a, &b);
                        if (a < n && b < n) rotations += rotate_pivot(A, V, n, a, b);
                    }
            }
            ++sweeps;
        }
    } else if (ordering == ORD_CLASSICAL) {
        long long per_sweep = (long long)n * (n - 1) / 2;
        long long limit = per_sweep * max_sweeps;
        for (;;) {
            if (sum_sq_offdiag(A, n) <= lim2) { converged = 1; break; }
            if (rotations >= limit) break;
            int bi = 0, bj = 1;
            double best = -1.0;
            for (int i = 0; i < n - 1; ++i)
                for (int j = i + 1; j < n; ++j) {
                    double v = fabs(A[(size_t)i * n + j]);
                    if (v > best) { best = v; bi = i; bj = j; }
                }
            rotations += rotate_pivot(A, V, n, bi, bj);
        }
        sweeps = per_sweep > 0 ? (int)((rotations + per_sweep - 1) / per_sweep) : 0;
    } else if (ordering == ORD_GREEDY) {
        double eps = n > 0 ? tol * sqrt(fro2) / n : 0.0;
        unsigned char *zeroed = calloc((size_t)n * n + 1, 1);
        unsigned char *used = calloc((size_t)n + 1, 1);
        int *sel = malloc(sizeof(int) * 2 * ((size_t)n / 2 + 1));
        for (;;) {
            memset(used, 0, (size_t)n);
            int nsel = 0;
            for (int i = 0; i < n - 1; ++i)
                for (int j = i + 1; j < n; ++j) {
                    if (fabs(A[(size_t)i * n + j]) > eps && !zeroed[(size_t)i * n + j] &&
                        !used[i] && !used[j]) {
                        used[i] = used[j] = 1;
                        sel[2 * nsel] = i;
                        sel[2 * nsel + 1] = j;
                        ++nsel;
                    }
                }
            if (nsel == 0) {
                int any_marked = 0;
                for (size_t e = 0; e < (size_t)n * n; ++e) any_marked |= zeroed[e];
                if (!any_marked) { converged = 1; break; }  /* nothing above eps */
                memset(zeroed, 0, (size_t)n * n);               /* new sweep */
                ++sweeps;
                if (sweeps >= max_sweeps) break;
                continue;
            }
            for (int e = 0; e < nsel; ++e) {
                int i = sel[2 * e], j = sel[2 * e + 1];
                rotations += rotate_pivot(A, V, n, i, j);
                zeroed[(size_t)i * n + j] = 1;
            }
        }
        free(zeroed);
        free(used);
        free(sel);
    } else {
        return -1;
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (rotations_out) *rotations_out = rotations;
    if (off_rel_out) *off_rel_out = fro2 > 0.0 ? sqrt(sum_sq_offdiag(A, n) / fro2) : 0.0;
    return converged;
}

/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, fp64 implementation of the pivoted LTL^T factorization of a
 * skew-symmetric matrix and of its Pfaffian.  Only tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this file's library; the GPU
 * library shares no code with it.
 *
 * Paper: "Performant Tridiagonal Factorization of Skew-Symmetric Matrices"
 * (arXiv 2411.09859).
 *
 *   - What is computed: Sec. 3.2 (Specification): P X P^T = L T L^T with L
 *     unit lower triangular, first column e_0, T skew-symmetric tridiagonal.
 *   - How: the unblocked right-looking (modified Parlett-Reid) algorithm of
 *     Sec. 2.4, eq. (1): one Gauss transform per column, the skew rank-2
 *     update X33 += l32 x32^T - x32 l32^T, with partial pivoting added as in
 *     Sec. 3.7.2 (largest magnitude of the column swapped to the top, the
 *     rows of the already computed part of L swapped with it) using iamax
 *     and P(pi) of Sec. 3.7.1 (Definitions of iamax and of P(pi)).
 *   - Pfaffian: definition in Sec. 1 (sum over permutations) together with
 *     Pf(B X B^T) = det(B) Pf(X); for P A P^T = L T L^T this gives
 *     Pf(A) = det(P) * Pf(T) = det(P) * prod_i T[2i][2i+1].
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - Full n x n storage of X and L (no implicit structure) so that every
 *     swap and every update is the literal textbook operation.
 *   - iamax returns the FIRST index among equal magnitudes.
 *   - A column whose candidates are all zero gives tau = 0, l = 0, no swap.
 *   - ipiv is absolute and 0-based: ipiv[0] = 0 (the first pivot is never
 *     computed, Fig. 5 caption), ipiv[r] = row swapped with row r at the
 *     step that produces column r of L.
 *   - The Pfaffian uses T[2i][2i+1] = -t[2i] and det(P); the shorter product
 *     printed in Sec. 1 omits both signs.
 *
 * Built with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 * The OpenMP loop splits the trailing update by columns; each element's
 * arithmetic is the same for any thread count, so results are bitwise
 * independent of the number of threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "skltlt_oracle.h"

#define X_(i, j) X[(size_t)(j) * (size_t)n + (size_t)(i)]
#define L_(i, j) L[(size_t)(j) * (size_t)n + (size_t)(i)]

/* Mutations plant a known mistake; used only by the tests that show the pins
 * catch such mistakes.  0 = the oracle proper. */
enum {
    MUT_NONE = 0,
    MUT_DROP_SECOND_TERM = 1, /* X33 += l x^T only (drops - x l^T)        */
    MUT_NO_PIVOTING = 2,      /* never swap                                */
    MUT_NO_L_ROW_SWAP = 3,    /* swap X but not the computed rows of L     */
    MUT_PF_NO_DETP = 4,       /* Pfaffian without det(P)                   */
    MUT_PF_PAPER_PRODUCT = 5, /* Pfaffian = prod t[2i] (no T sign, no P)   */
    MUT_L_FROM_UPPER = 6,     /* l taken from the upper triangle (-x)      */
    MUT_LAST_INDEX_TIES = 7,  /* iamax keeps the last of equal magnitudes  */
    MUT_WRONG_L_COLUMN = 8,   /* l stored one column too far right         */
    MUT_PARTIAL_UPDATE_SIGN = 9, /* partial: X += c l^T - l c^T          */
    MUT_PARTIAL_UNSCALED_L = 10, /* partial: l = x (not divided by tau)     */
    MUT_SECOND_LARGEST = 11      /* iamax takes the second largest magnitude */
};

int oracle_ltlt(int n, const double *A, int lda, double *X, double *L,
                double *t, int *ipiv, int max_steps, int pivot, int nthreads,
                int mutation)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && (!A || !X || !L || !ipiv)))
        return -1;
    if (n > 1 && !t)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    /* X := the full skew matrix whose strict lower triangle is A's
     * (Sec. 2.2: X = -X^T, zero diagonal); L := I. */
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double v;
            if (i > j)
                v = A[(size_t)j * lda + i];
            else if (i < j)
                v = -A[(size_t)i * lda + j];
            else
                v = 0.0;
            if (!isfinite(v))
                return -2;
            X_(i, j) = v;
            L_(i, j) = (i == j) ? 1.0 : 0.0;
        }
    }
    if (n == 0)
        return 0;
    ipiv[0] = 0;
    for (int i = 1; i < n; ++i)
        ipiv[i] = i;
    for (int k = 0; k + 1 < n; ++k)
        t[k] = 0.0;

    int steps = n - 1;
    if (max_steps >= 0 && max_steps < steps)
        steps = max_steps;

    double *l = (double *)malloc(sizeof(double) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    if (!l || !x) {
        free(l);
        free(x);
        return -3;
    }

    for (int k = 0; k < steps; ++k) {
        const int r = k + 1; /* the row that receives the pivot */

        /* iamax over X[r:n, k] (Sec. 3.7.1), first index on ties. */
        int p = r;
        double amax = fabs(X_(r, k));
        for (int i = r + 1; i < n; ++i) {
            double a = fabs(X_(i, k));
            if (mutation == MUT_LAST_INDEX_TIES ? (a >= amax) : (a > amax)) {
                amax = a;
                p = i;
            }
        }
        if (mutation == MUT_SECOND_LARGEST && r + 1 < n) {
            int q = -1;
            double bmax = -1.0;
            for (int i = r; i < n; ++i) {
                const double a = fabs(X_(i, k));
                if (i != p && a > bmax) {
                    bmax = a;
                    q = i;
                }
            }
            p = q;
        }
        /* Without pivoting (the unpivoted algorithms of Sec. 3.5 and 3.6,
         * for inputs known to need none) the pivot row is always r. */
        if (!pivot || mutation == MUT_NO_PIVOTING)
            p = r;
        ipiv[r] = p;

        /* Symmetric pivot P(pi) applied from both sides, and to the rows of
         * the part of L computed so far (columns 0..r-1) (Sec. 3.7.2). */
        if (p != r) {
            for (int j = 0; j < n; ++j) { /* rows r and p of X */
                double s = X_(r, j);
                X_(r, j) = X_(p, j);
                X_(p, j) = s;
            }
            for (int i = 0; i < n; ++i) { /* columns r and p of X */
                double s = X_(i, r);
                X_(i, r) = X_(i, p);
                X_(i, p) = s;
            }
            if (mutation != MUT_NO_L_ROW_SWAP) {
                for (int j = 0; j < r; ++j) {
                    double s = L_(r, j);
                    L_(r, j) = L_(p, j);
                    L_(p, j) = s;
                }
            }
        }

        /* Gauss transform, eq. (1): l32 := x31 / chi21. */
        const double tau = X_(r, k);
        t[k] = tau;
        for (int i = r + 1; i < n; ++i) {
            double xi = (mutation == MUT_L_FROM_UPPER) ? X_(k, i) : X_(i, k);
            l[i] = (tau != 0.0) ? xi / tau : 0.0;
        }
        const int lcol = (mutation == MUT_WRONG_L_COLUMN && r + 1 < n) ? r + 1 : r;
        for (int i = r + 1; i < n; ++i)
            L_(i, lcol) = l[i];

        /* x32 (column r below the pivot) is not changed by this transform
         * since chi22 = 0 (Sec. 3.5.2). */
        for (int i = r + 1; i < n; ++i)
            x[i] = X_(i, r);

        /* X33 := X33 + (l32 x32^T - x32 l32^T), eq. (1), on the whole
         * trailing block (both triangles, literally). */
        const int drop = (mutation == MUT_DROP_SECOND_TERM);
#pragma omp parallel for schedule(static)
        for (int j = r + 1; j < n; ++j) {
            const double xj = x[j], lj = l[j];
            for (int i = r + 1; i < n; ++i) {
                double upd = l[i] * xj;
                if (!drop)
                    upd = upd - x[i] * lj;
                X_(i, j) = X_(i, j) + upd;
            }
        }

        /* x31 := 0 (and its mirror in the upper triangle). */
        for (int i = r + 1; i < n; ++i) {
            X_(i, k) = 0.0;
            X_(k, i) = 0.0;
        }
    }

    free(l);
    free(x);
    return 0;
}

/* The Pfaffian-only reduction (Wimmer's algorithm as described in Sec. 3.5.2,
 * Notes, and Sec. 3.6.5, Note): the two-step right-looking algorithm with the
 * second Gauss transform of each pair (l43) and its tau (tau32) skipped.
 * Per pair of columns k, k+1 (k even):
 *   - iamax over X[k+1:n, k] and the symmetric exchange k+1 <-> p (Sec. 3.7);
 *   - tau = X[k+1][k]; l = X[k+2:n, k] / tau (0 if tau = 0);
 *   - c = X[k+2:n, k+1], the pair's second column, which the pair's own
 *     transform leaves unchanged (chi22 = 0, Sec. 3.5.2);
 *   - X[k+2:n, k+2:n] += l c^T - c l^T: the Schur complement of the 2 x 2
 *     block [[0, -tau], [tau, 0]], since Pf of that block is -tau and
 *     Pf(A) = Pf(block) Pf(complement) for a block-triangular congruence.
 * Pf(A) = det(P) prod_k (-tau_k) over the even k, as for the full
 * factorization. */
int oracle_ltlt_partial(int n, const double *A, int lda, double *t, int *ipiv,
                        int max_pairs, int nthreads, int mutation)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && (!A || !ipiv)))
        return -1;
    if (n > 1 && !t)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    if (n == 0)
        return 0;
    double *X = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *l = (double *)malloc(sizeof(double) * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    if (!X || !l || !c) {
        free(X);
        free(l);
        free(c);
        return -3;
    }
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double v;
            if (i > j)
                v = A[(size_t)j * lda + i];
            else if (i < j)
                v = -A[(size_t)i * lda + j];
            else
                v = 0.0;
            if (!isfinite(v)) {
                free(X);
                free(l);
                free(c);
                return -2;
            }
            X_(i, j) = v;
        }
    }
    ipiv[0] = 0;
    for (int i = 1; i < n; ++i)
        ipiv[i] = i;
    for (int k = 0; k + 1 < n; ++k)
        t[k] = 0.0;

    for (int k = 0; k + 1 < n; k += 2) {
        if (max_pairs >= 0 && k / 2 >= max_pairs)
            break;
        const int r = k + 1;
        int p = r;
        double amax = fabs(X_(r, k));
        for (int i = r + 1; i < n; ++i) {
            double a = fabs(X_(i, k));
            if (a > amax) {
                amax = a;
                p = i;
            }
        }
        ipiv[r] = p;
        if (p != r) {
            for (int j = 0; j < n; ++j) {
                double s = X_(r, j);
                X_(r, j) = X_(p, j);
                X_(p, j) = s;
            }
            for (int i = 0; i < n; ++i) {
                double s = X_(i, r);
                X_(i, r) = X_(i, p);
                X_(i, p) = s;
            }
        }
        const double tau = X_(r, k);
        t[k] = tau;
        for (int i = r + 1; i < n; ++i) {
            if (mutation == MUT_PARTIAL_UNSCALED_L)
                l[i] = X_(i, k);
            else
                l[i] = (tau != 0.0) ? X_(i, k) / tau : 0.0;
            c[i] = X_(i, r);
        }
        const double sg = (mutation == MUT_PARTIAL_UPDATE_SIGN) ? -1.0 : 1.0;
        /* Schur complement of the pair: rows and columns k+2 .. n-1 */
#pragma omp parallel for schedule(static)
        for (int j = r + 1; j < n; ++j) {
            const double cj = c[j], lj = l[j];
            for (int i = r + 1; i < n; ++i)
                X_(i, j) = X_(i, j) + sg * (l[i] * cj - c[i] * lj);
        }
        for (int i = r + 1; i < n; ++i) {
            X_(i, k) = 0.0;
            X_(k, i) = 0.0;
        }
    }
    free(X);
    free(l);
    free(c);
    return 0;
}

int oracle_pfaffian(int n, const double *t, const int *ipiv, double *log_abs_pf,
                    int *sign, int mutation)
{
    if (n < 0 || !log_abs_pf || !sign || (n > 1 && (!t || !ipiv)))
        return -1;
    /* The Pfaffian is defined for even order only (Sec. 1); for odd n the
     * determinant is zero and we report Pf = 0. */
    if (n % 2 != 0) {
        *log_abs_pf = -INFINITY;
        *sign = 0;
        return 0;
    }
    /* det(P): P is the product of the transpositions P(pi) (Sec. 3.7.1),
     * each non-trivial one contributing -1. */
    int s = 1;
    if (mutation != MUT_PF_NO_DETP && mutation != MUT_PF_PAPER_PRODUCT) {
        for (int i = 0; i < n; ++i)
            if (ipiv[i] != i)
                s = -s;
    }
    /* Pf(T) = prod_i T[2i][2i+1] with T[2i][2i+1] = -tau_{2i+1,2i}
     * (the tridiagonal T of Sec. 1 and eq. (TvsS)). */
    double acc = 0.0;
    for (int i = 0; i < n / 2; ++i) {
        double f = (mutation == MUT_PF_PAPER_PRODUCT) ? t[2 * i] : -t[2 * i];
        if (f == 0.0) {
            *log_abs_pf = -INFINITY;
            *sign = 0;
            return 0;
        }
        if (f < 0.0)
            s = -s;
        acc += log(fabs(f));
    }
    *log_abs_pf = acc;
    *sign = s;
    return 0;
}

/* Packs the factors into the in-place output layout of the library: the
 * strict lower triangle of Aout receives t on the first subdiagonal and
 * L[i][j+1] at (i, j) for i >= j+2 (Sec. 4.1, L stored shifted one column
 * left, T moved onto the subdiagonal).  Other entries are left alone. */
int oracle_pack(int n, const double *L, const double *t, double *Aout, int lda)
{
    if (n < 0 || lda < (n > 1 ? n : 1))
        return -1;
    for (int j = 0; j + 1 < n; ++j) {
        Aout[(size_t)j * lda + j + 1] = t[j];
        for (int i = j + 2; i < n; ++i)
            Aout[(size_t)j * lda + i] = L_(i, j + 1);
    }
    return 0;
}

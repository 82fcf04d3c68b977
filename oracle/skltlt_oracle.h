/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY (see skltlt_oracle.c).
 *
 * All matrices are column-major fp64.  Return value 0 on success, -1 for a
 * bad argument, -2 for a non-finite input entry, -3 when out of host memory.
 */
#ifndef SKLTLT_ORACLE_H
#define SKLTLT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Pivoted LTL^T of the skew matrix whose strict lower triangle is A (n x n,
 * leading dimension lda; diagonal and upper triangle are not read).
 *   X    (out, n*n, ld n): state after the steps taken; after all n-1 steps
 *        it holds the skew-tridiagonal T in full storage.
 *   L    (out, n*n, ld n): unit lower triangular, first column e_0.
 *   t    (out, n-1): t[k] = T[k+1][k].
 *   ipiv (out, n): absolute, 0-based, ipiv[0] = 0, ipiv[i] >= i.
 *   max_steps: < 0 for the whole factorization, else stop after that many
 *        column steps (X then holds the partially reduced matrix).
 *   pivot: 1 for partial pivoting (Sec. 3.7), 0 for none (Sec. 3.5-3.6:
 *        every step pivots on its own subdiagonal entry; ipiv[i] = i).
 *   nthreads: OpenMP threads for the trailing update (<= 0: default).
 *   mutation: 0 for the oracle; non-zero values plant known mistakes and are
 *        used only by the tests of the pins. */
int oracle_ltlt(int n, const double *A, int lda, double *X, double *L,
                double *t, int *ipiv, int max_steps, int pivot, int nthreads,
                int mutation);

/* Pf(A) = det(P) * prod_i (-t[2i]) as log|Pf| and sign in {-1, 0, +1}.
 * Odd n or a zero factor give sign 0 and log|Pf| = -inf. */
int oracle_pfaffian(int n, const double *t, const int *ipiv,
                    double *log_abs_pf, int *sign, int mutation);

/* The Pfaffian-only ("partial") reduction: one pivot and one Gauss transform
 * per PAIR of columns, the second transform of each pair and its tau never
 * formed.  Same input as oracle_ltlt.
 *   t    (out, n-1): t[k] = tau of the pivot step k for even k, 0 for odd k.
 *   ipiv (out, n): ipiv[k+1] = pivot row of step k for even k; every other
 *        entry is its own index (no exchange).
 *   max_pairs: < 0 for the whole reduction, else stop after that many pairs.
 * Pf(A) then follows from oracle_pfaffian(n, t, ipiv, ...). */
int oracle_ltlt_partial(int n, const double *A, int lda, double *t, int *ipiv,
                        int max_pairs, int nthreads, int mutation);

/* Writes t and L into the strict lower triangle of Aout in the packed
 * in-place layout (t on the first subdiagonal, L[i][j+1] at (i, j)). */
int oracle_pack(int n, const double *L, const double *t, double *Aout,
                int lda);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain FP64 reference for a series of tridiagonal systems A X_n = F_n,
 * n = 1..N (statement of the problem, section 2 of the paper).  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may call it;
 * the GPU library never links or loads it, and it shares no code with it.
 *
 * Layout: F and X are M x N, RHS-interleaved (row-major): F[i*N + n] is
 * row i of right-hand side n.  A is symmetric: diagonal b[0..M-1],
 * off-diagonal a[0..M-2] with A[i][i+1] = A[i+1][i] = a[i].
 *
 * oracle_thomas follows the sequential sweep ("Thomas") method the paper
 * builds on (introduction; Lemma 1's block solves are the same elimination):
 * forward elimination of the sub-diagonal, then back substitution, one
 * right-hand side at a time, no pivoting.  X = A^{-1} F is the plain
 * definition that the paper's parallel method reproduces exactly (Theorem 2).
 *
 * oracle_tridiag_general solves one general (nonsymmetric) tridiagonal
 * system; it serves the Python side of the oracle for the matrices B^R_k,
 * B^L_k of eq. (z_vector) and the identity-bordered block matrices A_i of
 * Lemma 1.
 *
 * oracle_grad is the adjoint of X = A^{-1} F for loss L with dL/dX = gX:
 * gF = A^{-T} gX = A^{-1} gX (A symmetric, Lemma 2), dL/dA = -gF X^T summed
 * over the series, hence gb_i = -sum_n gF[i,n] X[i,n] and
 * ga_i = -sum_n (gF[i,n] X[i+1,n] + gF[i+1,n] X[i,n]).
 *
 * Return value: 0 on success, -1 on bad sizes, -2 when an elimination pivot
 * is zero or not finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static int solve_one(int64_t M, int64_t N, int64_t n, const double* a,
                     const double* b, const double* F, double* X,
                     double* cp, double* dp)
{
    /* forward elimination: row i becomes x_i + cp[i] x_{i+1} = dp[i] */
    double den = b[0];
    if (den == 0.0 || !isfinite(den)) return -2;
    cp[0] = (M > 1) ? a[0] / den : 0.0;
    dp[0] = F[0 * N + n] / den;
    for (int64_t i = 1; i < M; ++i) {
        den = b[i] - a[i - 1] * cp[i - 1];
        if (den == 0.0 || !isfinite(den)) return -2;
        cp[i] = (i < M - 1) ? a[i] / den : 0.0;
        dp[i] = (F[i * N + n] - a[i - 1] * dp[i - 1]) / den;
    }
    /* back substitution */
    X[(M - 1) * N + n] = dp[M - 1];
    for (int64_t i = M - 2; i >= 0; --i)
        X[i * N + n] = dp[i] - cp[i] * X[(i + 1) * N + n];
    return 0;
}

int oracle_thomas(int64_t M, int64_t N, const double* a, const double* b,
                  const double* F, double* X)
{
    if (M < 1 || N < 0) return -1;
    if (N == 0) return 0;
    int status = 0;
#pragma omp parallel
    {
        double* cp = (double*)malloc(sizeof(double) * (size_t)M);
        double* dp = (double*)malloc(sizeof(double) * (size_t)M);
        int local = (cp && dp) ? 0 : -1;
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            if (local == 0) local = solve_one(M, N, n, a, b, F, X, cp, dp);
        }
#pragma omp critical
        {
            if (local != 0 && status == 0) status = local;
        }
        free(cp);
        free(dp);
    }
    return status;
}

int oracle_tridiag_general(int64_t n, const double* lower, const double* diag,
                           const double* upper, const double* rhs, double* x)
{
    /* row i: lower[i] x_{i-1} + diag[i] x_i + upper[i] x_{i+1} = rhs[i]
       (lower[0] and upper[n-1] are ignored) */
    if (n < 1) return -1;
    double* cp = (double*)malloc(sizeof(double) * (size_t)n);
    double* dp = (double*)malloc(sizeof(double) * (size_t)n);
    if (!cp || !dp) { free(cp); free(dp); return -1; }
    int rc = 0;
    double den = diag[0];
    if (den == 0.0 || !isfinite(den)) { rc = -2; goto done; }
    cp[0] = (n > 1) ? upper[0] / den : 0.0;
    dp[0] = rhs[0] / den;
    for (int64_t i = 1; i < n; ++i) {
        den = diag[i] - lower[i] * cp[i - 1];
        if (den == 0.0 || !isfinite(den)) { rc = -2; goto done; }
        cp[i] = (i < n - 1) ? upper[i] / den : 0.0;
        dp[i] = (rhs[i] - lower[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
done:
    free(cp);
    free(dp);
    return rc;
}

int oracle_grad(int64_t M, int64_t N, const double* a, const double* b,
                const double* X, const double* gX, double* gF, double* ga,
                double* gb)
{
    int rc = oracle_thomas(M, N, a, b, gX, gF);
    if (rc != 0) return rc;
    for (int64_t i = 0; i < M; ++i) {
        double s = 0.0;
        for (int64_t n = 0; n < N; ++n) s += gF[i * N + n] * X[i * N + n];
        gb[i] = -s;
    }
    for (int64_t i = 0; i + 1 < M; ++i) {
        double s = 0.0;
        for (int64_t n = 0; n < N; ++n)
            s += gF[i * N + n] * X[(i + 1) * N + n] + gF[(i + 1) * N + n] * X[i * N + n];
        ga[i] = -s;
    }
    return 0;
}

int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

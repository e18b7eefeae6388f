/*
 * psp_oracle.c -- plain CPU FP64 oracle for perturbation-induced static
 * pivoting (arXiv 2311.11833).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only tests/, the smoke check and the benchmark's CPU-baseline
 * leg load it.  It shares no code with the GPU path.
 *
 * Everything is plain loops in IEEE binary64, round to nearest even.  Where
 * a multiply-add appears it is written as an explicit fma() and the file is
 * compiled with -ffp-contract=off, so the operation sequence below is the
 * one that is executed.  Division is IEEE division (never a reciprocal
 * multiply).
 *
 * Contents and the passage each part follows:
 *   weights      Sec. III-A, Remark 2 and its proof (Vandermonde system
 *                Gamma^T beta = e1), generalised to any distinct node set
 *                as the Lagrange weights at zero.
 *   dense LU     Sec. II-C / III-A: factorisation with a static pivot
 *                sequence (no row exchange) of A + eps D.
 *   solves       Alg. 1 step 2 (factor and solve each perturbed system);
 *                transposed solves for the adjoint.
 *   combine      Alg. 1 steps 3-4, eq. (x_star): x = sum_k c_k x_k.
 *   estimate     Alg. 1 step 5 from the perturbed solutions alone: divided
 *                differences give the expansion's next term (Sec. II-B,
 *                Theorem 1); node scale from truncation vs rounding (Sec. V).
 *   pivoted LU   ground truth x* = A^{-1} b of Sec. III (problem statement).
 *   symbolic     static pivot sequence computed once and reused (Sec. II-C):
 *                minimum-degree order, elimination tree, fill, level sets.
 *   sparse LU    the same factorisation restricted to the symbolic fill
 *                (the sparse batched factorisation of Sec. IV / V).
 *   gradient     adjoint of x = sum_k c_k (A + eps_k D)^{-1} b.
 *   residual     Alg. 1 step 5 (optional error test): r = b - A x and the
 *                2-norms of r and b (the residual norm of Fig. 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* Number of OpenMP threads the batched routines use from now on (the CPU
 * baseline is timed at one thread and at all threads). */
EXPORT void oracle_set_threads(int t) {
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* Weights.  Remark 2: beta = (Gamma_m^T)^{-1} e1 makes the combination  */
/* keep the A^{-1} term with unit coefficient and cancel the next powers */
/* of eps.  For nodes eps_1..eps_K the same conditions read              */
/*   sum_k c_k eps_k^j = delta_{j0},  j = 0..K-1,                         */
/* whose unique solution is the Lagrange basis evaluated at zero:         */
/*   c_k = prod_{l != k} eps_l / (eps_l - eps_k).                         */
/* Returns 0, or -1 when the nodes are not distinct, zero or finite.     */
/* ------------------------------------------------------------------ */
EXPORT int oracle_weights(int K, const double* eps, double* c) {
    if (K < 1) return -1;
    for (int k = 0; k < K; ++k) {
        if (!isfinite(eps[k]) || eps[k] == 0.0) return -1;
        for (int l = 0; l < k; ++l)
            if (eps[l] == eps[k]) return -1;
    }
    for (int k = 0; k < K; ++k) {
        double p = 1.0;
        for (int l = 0; l < K; ++l) {
            if (l == k) continue;
            p = p * (eps[l] / (eps[l] - eps[k]));
        }
        c[k] = p;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dense pivot-free LU (Doolittle), column-major, in place.              */
/* For k = 0..n-1: the pivot a_kk must be nonzero and finite; the        */
/* multipliers are l_ik = a_ik / a_kk; every trailing entry is updated   */
/* a_ij <- fma(-l_ik, a_kj, a_ij).  Each entry therefore receives its    */
/* updates in ascending k.  Returns 0, or j+1 for the first pivot that   */
/* is zero or not finite (the factorisation stops there).                */
/* ------------------------------------------------------------------ */
EXPORT int oracle_lu_nopiv(int n, double* a, int lda) {
    for (int k = 0; k < n; ++k) {
        const double piv = a[k + (size_t)k * lda];
        if (piv == 0.0 || !isfinite(piv)) return k + 1;
        for (int i = k + 1; i < n; ++i) a[i + (size_t)k * lda] = a[i + (size_t)k * lda] / piv;
        for (int j = k + 1; j < n; ++j) {
            const double u = a[k + (size_t)j * lda];
            double* col = a + (size_t)j * lda;
            const double* l = a + (size_t)k * lda;
            for (int i = k + 1; i < n; ++i) col[i] = fma(-l[i], u, col[i]);
        }
    }
    return 0;
}

/* L y = b with L unit lower (strict lower part of lu); y overwrites b.
 * Column-oriented: for k ascending, y_i <- fma(-l_ik, y_k, y_i), i > k. */
EXPORT void oracle_fwd_unit_lower(int n, const double* lu, int lda, double* y) {
    for (int k = 0; k < n; ++k) {
        const double yk = y[k];
        const double* l = lu + (size_t)k * lda;
        for (int i = k + 1; i < n; ++i) y[i] = fma(-l[i], yk, y[i]);
    }
}

/* U x = y with U upper (upper part of lu incl. diagonal); x overwrites y.
 * Column-oriented: for j descending, x_j = y_j / u_jj, then
 * y_i <- fma(-u_ij, x_j, y_i), i < j. */
EXPORT void oracle_back_upper(int n, const double* lu, int lda, double* y) {
    for (int j = n - 1; j >= 0; --j) {
        const double* u = lu + (size_t)j * lda;
        const double xj = y[j] / u[j];
        y[j] = xj;
        for (int i = 0; i < j; ++i) y[i] = fma(-u[i], xj, y[i]);
    }
}

/* U^T z = w (U^T lower with diagonal u_kk); z overwrites w.
 * For k ascending: z_k = w_k / u_kk, then w_i <- fma(-u_ki, z_k, w_i), i > k. */
EXPORT void oracle_fwd_upper_trans(int n, const double* lu, int lda, double* w) {
    for (int k = 0; k < n; ++k) {
        const double zk = w[k] / lu[k + (size_t)k * lda];
        w[k] = zk;
        for (int i = k + 1; i < n; ++i) w[i] = fma(-lu[k + (size_t)i * lda], zk, w[i]);
    }
}

/* L^T v = z (L^T unit upper); v overwrites z.
 * For k descending: v_k = z_k, then z_i <- fma(-l_ki, v_k, z_i), i < k. */
EXPORT void oracle_back_lower_trans(int n, const double* lu, int lda, double* z) {
    for (int k = n - 1; k >= 0; --k) {
        const double vk = z[k];
        for (int i = 0; i < k; ++i) z[i] = fma(-lu[k + (size_t)i * lda], vk, z[i]);
    }
}

/* x = sum_k c_k x_k, ascending k, as an fma chain starting from zero.
 * xk is K blocks of len values. */
EXPORT void oracle_combine(int K, int64_t len, const double* c, const double* xk, double* x) {
    for (int64_t i = 0; i < len; ++i) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc = fma(c[k], xk[(size_t)k * len + i], acc);
        x[i] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* A-posteriori error estimate of the combination (Alg. 1 step 5 done    */
/* without the unperturbed matrix).  By the expansion of Sec. II-B the   */
/* perturbed solutions are x(eps) = sum_j (-eps)^j M^j x*, M = A^{-1} D, */
/* so the divided difference of x over the first j+1 nodes,               */
/*   f[eps_0..eps_j] = sum_{k<=j} x_k / prod_{l<=j, l!=k} (eps_k - eps_l),*/
/* is (-1)^j M^j x* up to terms of order eps, and the combination's       */
/* leading error is -(prod_k eps_k) M^K x* (Theorem 1 for general nodes). */
/* With m_j = ||f[eps_0..eps_j]||_inf the ratio m_{K-1} / m_{K-2} is one  */
/* more power of M (a growth factor rho_hat), and                         */
/*   est = |prod_k eps_k| m_{K-1} rho_hat / ||x_hat||_inf                 */
/* estimates the relative error of x_hat.  Operation order: the weights   */
/* multiply (eps_k - eps_l) in ascending l and take one reciprocal; each  */
/* entry of f is an fma chain over ascending k from zero; the product of  */
/* |eps_k| runs in ascending k; est = ((P m1) (m1 / m2)) / mx.            */
/* ------------------------------------------------------------------ */

/* f[eps_0..eps_j] of the K blocks xk (each len values) into out. */
EXPORT void oracle_divided_difference(int j, const double* eps, int64_t len, const double* xk, double* out) {
    double w[64];
    for (int k = 0; k <= j; ++k) {
        double p = 1.0;
        for (int l = 0; l <= j; ++l)
            if (l != k) p = p * (eps[k] - eps[l]);
        w[k] = 1.0 / p;
    }
    for (int64_t i = 0; i < len; ++i) {
        double acc = 0.0;
        for (int k = 0; k <= j; ++k) acc = fma(w[k], xk[(size_t)k * len + i], acc);
        out[i] = acc;
    }
}

static double max_abs(int64_t len, const double* v) {
    double m = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        const double a = fabs(v[i]);
        if (a != a) return a;          /* NaN propagates */
        if (a > m) m = a;
    }
    return m;
}

/* est and rho_hat of one system from its K (>= 3) perturbed solutions xk
 * (K blocks of len) and the combination x.  m_{K-1} = 0 gives est = 0,
 * rho_hat = 0; a NaN anywhere gives NaN. */
EXPORT void oracle_error_estimate(int K, const double* eps, int64_t len, const double* xk, const double* x,
                                  double* est, double* rho_hat) {
    double* f = (double*)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
    oracle_divided_difference(K - 1, eps, len, xk, f);
    const double m1 = max_abs(len, f);
    oracle_divided_difference(K - 2, eps, len, xk, f);
    const double m2 = max_abs(len, f);
    free(f);
    const double mx = max_abs(len, x);
    if (m1 != m1 || m2 != m2 || mx != mx) {
        *est = *rho_hat = m1 + m2 + mx;
        return;
    }
    if (m1 == 0.0) {
        *est = *rho_hat = 0.0;
        return;
    }
    double P = 1.0;
    for (int k = 0; k < K; ++k) P = P * fabs(eps[k]);
    const double r = m1 / m2;
    *rho_hat = r;
    *est = ((P * m1) * r) / mx;
}

/* ------------------------------------------------------------------ */
/* Node scale for a system whose estimate is above the tolerance (the    */
/* perturbation strategy Sec. V leaves open).  The nodes become s eps_k   */
/* with s = 2^-j, j >= 1 (the weights do not change).  The error at s is  */
/* modelled as truncation + rounding,                                     */
/*   T(s) = a s^K   with a = est when est < 1e-2 (the series converges   */
/*                  and est is its leading term), else                    */
/*                  a = |prod_k eps_k| rho_hat^K (a from the growth rate) */
/*   R(s) = b / s   with b = gamma u / max_k |eps_k|, u = 2^-53,          */
/* the rounding of the pivot-free solves growing like 1/eps once eps      */
/* controls the smallest pivot (gamma = 50).  T + R is smallest at        */
/* s* = q^{1/(K+1)}, q = b / (K a); j is the smallest j >= 1 with          */
/* 2^{-j(K+1)} <= q, i.e. s is the largest power of two <= min(s*, 1/2),  */
/* found from the binary exponent e of q (2^e <= q < 2^{e+1}):             */
/* j = max(1, ceil(-e / (K+1))), at most 60.  A NaN est, or q zero or not */
/* finite, gives j = 10.                                                  */
/* ------------------------------------------------------------------ */
EXPORT int oracle_scale_exponent(int K, const double* eps, double est, double rho_hat) {
    if (est != est) return 10;
    double emax = 0.0, P = 1.0;
    for (int k = 0; k < K; ++k) {
        const double a = fabs(eps[k]);
        if (a > emax) emax = a;
        P = P * a;
    }
    double a = est;
    if (!(est < 1e-2)) {
        a = P;
        for (int k = 0; k < K; ++k) a = a * rho_hat;
    }
    const double b = (50.0 * 0x1p-53) / emax;
    const double q = b / ((double)K * a);
    if (!(q > 0.0) || !isfinite(q)) return 10;
    const int e = ilogb(q);
    int j = e >= 0 ? 1 : (-e + K) / (K + 1);
    if (j < 1) j = 1;
    if (j > 60) j = 60;
    return j;
}

/* ------------------------------------------------------------------ */
/* Error test (Alg. 1 step 5): r = b - A x for CSR A, each r_i taken as   */
/* b_i followed by fma(-a_ie, x_j, .) over row i in CSR order; ||r||_2 and */
/* ||b||_2 as sqrt of the sum of squares accumulated by fma in ascending   */
/* row order.  b, x, r are n x nrhs row-major; rnorm, bnorm are nrhs long; */
/* r and bnorm may be NULL.                                                */
/* ------------------------------------------------------------------ */
EXPORT void oracle_residual(int n, const int* rowptr, const int* colidx, const double* val, int nrhs,
                            const double* b, const double* x, double* r, double* rnorm, double* bnorm) {
    for (int q = 0; q < nrhs; ++q) {
        double sr = 0.0, sb = 0.0;
        for (int i = 0; i < n; ++i) {
            double acc = b[(size_t)i * nrhs + q];
            for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc = fma(-val[e], x[(size_t)colidx[e] * nrhs + q], acc);
            if (r) r[(size_t)i * nrhs + q] = acc;
            sr = fma(acc, acc, sr);
            sb = fma(b[(size_t)i * nrhs + q], b[(size_t)i * nrhs + q], sb);
        }
        rnorm[q] = sqrt(sr);
        if (bnorm) bnorm[q] = sqrt(sb);
    }
}

/* 2-norm as the square root of the fma sum of squares in ascending order
 * (the norm used by the error test and the rho power iteration). */
EXPORT double oracle_norm2(int n, const double* x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = fma(x[i], x[i], s);
    return sqrt(s);
}

/* ------------------------------------------------------------------ */
/* Ground truth: LU with partial pivoting (largest |a_ik| in the column, */
/* ties to the smallest row index), then the two substitutions.          */
/* piv[k] = row swapped with row k at step k.  Returns 0 or k+1 if the   */
/* column is exactly zero.                                                */
/* ------------------------------------------------------------------ */
EXPORT int oracle_lu_partial(int n, double* a, int lda, int* piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k + (size_t)k * lda]);
        for (int i = k + 1; i < n; ++i) {
            const double v = fabs(a[i + (size_t)k * lda]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return k + 1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = a[k + (size_t)j * lda];
                a[k + (size_t)j * lda] = a[p + (size_t)j * lda];
                a[p + (size_t)j * lda] = t;
            }
        const double d = a[k + (size_t)k * lda];
        for (int i = k + 1; i < n; ++i) a[i + (size_t)k * lda] = a[i + (size_t)k * lda] / d;
        for (int j = k + 1; j < n; ++j) {
            const double u = a[k + (size_t)j * lda];
            for (int i = k + 1; i < n; ++i)
                a[i + (size_t)j * lda] = fma(-a[i + (size_t)k * lda], u, a[i + (size_t)j * lda]);
        }
    }
    return 0;
}

EXPORT void oracle_lu_partial_solve(int n, const double* lu, int lda, const int* piv, double* b) {
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    oracle_fwd_unit_lower(n, lu, lda, b);
    oracle_back_upper(n, lu, lda, b);
}

/* ------------------------------------------------------------------ */
/* One perturbed dense system, end to end: A_k = P (A + eps D) P^T from  */
/* CSR, pivot-free LU, then x = P^T U^{-1} L^{-1} P b for nrhs columns.   */
/* perm[q] = original index placed at position q (NULL = identity);       */
/* d = diagonal of D (NULL = identity).  b and x are n x nrhs row-major.  */
/* lu (n x n, column-major, lda = n) receives the factors when non-NULL.  */
/* Returns the LU info.                                                   */
/* ------------------------------------------------------------------ */
EXPORT int oracle_dense_system(int n, const int* rowptr, const int* colidx, const double* val,
                               const int* perm, double eps, const double* d,
                               int nrhs, const double* b, double* x, double* lu_out) {
    int* ip = (int*)malloc(sizeof(int) * (size_t)n);
    for (int q = 0; q < n; ++q) ip[perm ? perm[q] : q] = q;
    double* a = lu_out ? lu_out : (double*)malloc(sizeof(double) * (size_t)n * n);
    memset(a, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
            a[ip[i] + (size_t)ip[colidx[e]] * n] = val[e];
    for (int i = 0; i < n; ++i) a[ip[i] + (size_t)ip[i] * n] += eps * (d ? d[i] : 1.0);
    const int info = oracle_lu_nopiv(n, a, n);
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    for (int r = 0; r < nrhs; ++r) {
        for (int q = 0; q < n; ++q) t[q] = b[(size_t)(perm ? perm[q] : q) * nrhs + r];
        if (info == 0) {
            oracle_fwd_unit_lower(n, a, n, t);
            oracle_back_upper(n, a, n, t);
        } else {
            for (int q = 0; q < n; ++q) t[q] = NAN;
        }
        for (int q = 0; q < n; ++q) x[(size_t)(perm ? perm[q] : q) * nrhs + r] = t[q];
    }
    free(t);
    if (!lu_out) free(a);
    free(ip);
    return info;
}

/* The whole method for a batch of Jacobians sharing one pattern, dense:
 * for each Jacobian s and node k, solve (A_s + eps_k D) x_sk = b_s, then
 * x_s = sum_k c_k x_sk.  Systems are independent, so the (s, k) loop is
 * spread over OpenMP threads; the combine is done per s in ascending k.
 * vals: batch x nnz; b, x: batch x n x nrhs; xk (optional): batch x K x n x nrhs;
 * info: batch x K.  Returns the number of threads used. */
EXPORT int oracle_dense_batch(int n, const int* rowptr, const int* colidx, int batch,
                              const double* vals, const int* perm, int K, const double* eps,
                              const double* c, const double* d, int nrhs, const double* b,
                              double* x, double* xk_out, int* info) {
    const size_t nn = (size_t)n * nrhs;
    const int64_t nnz = rowptr[n];
    double* xk = xk_out ? xk_out : (double*)malloc(sizeof(double) * (size_t)batch * K * nn);
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            used = omp_get_num_threads();
#endif
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < (int64_t)batch * K; ++t) {
            const int s = (int)(t / K), k = (int)(t % K);
            info[t] = oracle_dense_system(n, rowptr, colidx, vals + (size_t)s * nnz, perm, eps[k], d,
                                          nrhs, b + (size_t)s * nn, xk + (size_t)t * nn, NULL);
        }
    }
    for (int s = 0; s < batch; ++s) oracle_combine(K, (int64_t)nn, c, xk + (size_t)s * K * nn, x + (size_t)s * nn);
    if (!xk_out) free(xk);
    return used;
}

/*
 * hh_oracle.c -- FP64 CPU oracle for the Householder-reflector hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or constant with the HIP
 * implementation.
 *
 * It is written to be read against the paper (Rusu, "Approximate eigenvalue
 * decompositions of linear transformations with a few Householder
 * reflectors", arXiv 1811.07624): every routine is the plain definition,
 * evaluated in double precision with straightforward loops.
 *
 * Conventions (all matrices column-major, leading dimensions as in BLAS):
 *   U(i,k) = U[i + k*ldu]   reflector vectors u_1..u_h are the columns of U
 *   X(i,j) = X[i + j*ldx]   vector j of the batch is column j
 *   H_k    = I - 2 uh_k uh_k^T with uh_k = u_k / ||u_k||_2  (Sec. II-A, eq. 2:
 *            the paper constrains ||u_k|| = 1; we normalise the given vector)
 *   u_k = 0 gives H_k = I  (Sec. II-B, Result 1: a zero reflector vector is
 *            the identity factor)
 *   Q      = H_1 H_2 ... H_h   (the product order of eq. 1 as used by Result 3,
 *            eq. theU2: Ubar_2 = J_1 ... J_h).  Q x applies H_h first.
 *   Sym    = Q diag(lam) Q^T  (Sec. III-A, eq. thesbar, with D = I)
 *   Mahal  d = sum_i lam_i ((Q^T (x - y))_i)^2  (Sec. IV-C: the metric
 *            S = L^T L with L = sqrt(Lambda) U_paper, U_paper = Q^T)
 *
 * Backward passes are the per-vector chain rule written out step by step,
 * storing every intermediate vector (no recomputation tricks), followed by the
 * chain rule through the normalisation uh = u / ||u||.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* Normalisation (eq. 2: unit reflector vectors).  Uh is n x h, ld = n.
 * nrm[k] receives ||u_k||_2 (0 for a zero column).                      */
EXPORT void orc_normalize(int64_t n, int64_t h, const double *U, int64_t ldu,
                          double *Uh, double *nrm) {
    for (int64_t k = 0; k < h; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += U[i + k * ldu] * U[i + k * ldu];
        double r = sqrt(s);
        if (nrm) nrm[k] = r;
        for (int64_t i = 0; i < n; ++i)
            Uh[i + k * n] = (r > 0.0) ? U[i + k * ldu] / r : 0.0;
    }
}

/* z <- (I - 2 u u^T) z for one unit (or zero) vector u.  Returns u^T z. */
static double reflect(int64_t n, const double *u, double *z) {
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) a += u[i] * z[i];
    for (int64_t i = 0; i < n; ++i) z[i] -= 2.0 * a * u[i];
    return a;
}

/* Reflector index used at step r (0-based) of a chain.
 * trans = 0 : Q x   = H_1 (H_2 (... (H_h x)))  -> steps use k = h-1, ..., 0
 * trans = 1 : Q^T x = H_h (... (H_1 x))        -> steps use k = 0, ..., h-1 */
static int64_t chain_index(int64_t h, int trans, int64_t r) {
    return trans ? r : (h - 1 - r);
}

/* ------------------------------------------------------------------ */
/* Forward: Y = Q X (trans = 0) or Y = Q^T X (trans = 1).  Sec. II-A,
 * eqs. 1-2; each step is one dot product and one update (4n operations per
 * reflector, as counted in Sec. II-A).                                   */
EXPORT void orc_apply(int64_t n, int64_t h, const double *U, int64_t ldu,
                      int trans, const double *X, int64_t ldx, int64_t N,
                      double *Y, int64_t ldy) {
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * (h > 0 ? h : 1)));
    orc_normalize(n, h, U, ldu, Uh, NULL);
#pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t i = 0; i < n; ++i) z[i] = X[i + j * ldx];
            for (int64_t r = 0; r < h; ++r)
                reflect(n, Uh + chain_index(h, trans, r) * n, z);
            for (int64_t i = 0; i < n; ++i) Y[i + j * ldy] = z[i];
        }
        free(z);
    }
    free(Uh);
}

/* Dense Q = H_1 H_2 ... H_h as an explicit n x n matrix (ld = n), built by
 * multiplying the explicit reflector matrices left to right.  Only for small
 * n: O(h n^3).                                                           */
EXPORT void orc_dense_Q(int64_t n, int64_t h, const double *U, int64_t ldu,
                        double *Q) {
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * (h > 0 ? h : 1)));
    double *Hk = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *T = (double *)malloc(sizeof(double) * (size_t)(n * n));
    orc_normalize(n, h, U, ldu, Uh, NULL);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) Q[i + j * n] = (i == j) ? 1.0 : 0.0;
    for (int64_t k = 0; k < h; ++k) {
        const double *u = Uh + k * n;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                Hk[i + j * n] = ((i == j) ? 1.0 : 0.0) - 2.0 * u[i] * u[j];
        /* T = Q * Hk */
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int64_t l = 0; l < n; ++l) s += Q[i + l * n] * Hk[l + j * n];
                T[i + j * n] = s;
            }
        memcpy(Q, T, sizeof(double) * (size_t)(n * n));
    }
    free(T);
    free(Hk);
    free(Uh);
}

/* ------------------------------------------------------------------ */
/* Symmetric form: Y = Q diag(lam) Q^T X.  Sec. III-A, eq. thesbar with
 * D = I: first Q^T (H_1 first), then the diagonal, then Q (H_h first);
 * (8h + 1) n operations per vector as counted there.                     */
EXPORT void orc_sym(int64_t n, int64_t h, const double *U, int64_t ldu,
                    const double *lam, const double *X, int64_t ldx, int64_t N,
                    double *Y, int64_t ldy) {
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * (h > 0 ? h : 1)));
    orc_normalize(n, h, U, ldu, Uh, NULL);
#pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t i = 0; i < n; ++i) z[i] = X[i + j * ldx];
            for (int64_t r = 0; r < h; ++r) reflect(n, Uh + chain_index(h, 1, r) * n, z);
            for (int64_t i = 0; i < n; ++i) z[i] *= lam[i];
            for (int64_t r = 0; r < h; ++r) reflect(n, Uh + chain_index(h, 0, r) * n, z);
            for (int64_t i = 0; i < n; ++i) Y[i + j * ldy] = z[i];
        }
        free(z);
    }
    free(Uh);
}

/* ------------------------------------------------------------------ */
/* Mahalanobis distance of the metric-learning application (Sec. IV-C):
 * d_j = || sqrt(Lambda) Q^T (xa_j - xb_j) ||^2
 *     = sum_i lam_i ((Q^T (xa_j - xb_j))_i)^2.                           */
EXPORT void orc_mahal(int64_t n, int64_t h, const double *U, int64_t ldu,
                      const double *lam, const double *Xa, int64_t lda,
                      const double *Xb, int64_t ldb, int64_t N, double *d) {
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * (h > 0 ? h : 1)));
    orc_normalize(n, h, U, ldu, Uh, NULL);
#pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t i = 0; i < n; ++i) z[i] = Xa[i + j * lda] - Xb[i + j * ldb];
            for (int64_t r = 0; r < h; ++r) reflect(n, Uh + chain_index(h, 1, r) * n, z);
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += lam[i] * z[i] * z[i];
            d[j] = s;
        }
        free(z);
    }
    free(Uh);
}

/* ------------------------------------------------------------------ */
/* Backward machinery.
 *
 * One chain step maps s_{r-1} to s_r = s_{r-1} - 2 (uh^T s_{r-1}) uh.
 * With upstream gradient g_r = dL/ds_r:
 *   dL/ds_{r-1} = H g_r = g_r - 2 (uh^T g_r) uh
 *   dL/duh     += -2 [ (uh^T s_{r-1}) g_r + (uh^T g_r) s_{r-1} ]
 * (product rule on the two occurrences of uh; H is symmetric).
 * Then dL/du = (I - uh uh^T) dL/duh / ||u|| (chain rule through uh = u/||u||),
 * and 0 for a zero column.                                               */

/* Reverse sweep over a chain of h steps.  S holds s_0..s_h (each n long,
 * S + r*n); g holds g_h on entry and g_0 on exit; dUh (n x h) accumulates. */
static void chain_backward(int64_t n, int64_t h, const double *Uh, int trans,
                           const double *S, double *g, double *dUh) {
    for (int64_t r = h; r >= 1; --r) {
        int64_t k = chain_index(h, trans, r - 1);
        const double *u = Uh + k * n;
        const double *sp = S + (r - 1) * n;
        double a = 0.0, b = 0.0;
        for (int64_t i = 0; i < n; ++i) { a += u[i] * sp[i]; b += u[i] * g[i]; }
        for (int64_t i = 0; i < n; ++i) dUh[i + k * n] += -2.0 * (a * g[i] + b * sp[i]);
        for (int64_t i = 0; i < n; ++i) g[i] -= 2.0 * b * u[i];
    }
}

/* Forward sweep storing s_0..s_h in S (s_0 already in S). */
static void chain_forward(int64_t n, int64_t h, const double *Uh, int trans,
                          double *S) {
    for (int64_t r = 1; r <= h; ++r) {
        memcpy(S + r * n, S + (r - 1) * n, sizeof(double) * (size_t)n);
        reflect(n, Uh + chain_index(h, trans, r - 1) * n, S + r * n);
    }
}

static void normalize_backward(int64_t n, int64_t h, const double *Uh,
                               const double *nrm, const double *dUh, double *dU,
                               int64_t lddu) {
    for (int64_t k = 0; k < h; ++k) {
        const double *u = Uh + k * n;
        const double *gu = dUh + k * n;
        if (!(nrm[k] > 0.0)) {
            for (int64_t i = 0; i < n; ++i) dU[i + k * lddu] = 0.0;
            continue;
        }
        double p = 0.0;
        for (int64_t i = 0; i < n; ++i) p += u[i] * gu[i];
        for (int64_t i = 0; i < n; ++i) dU[i + k * lddu] = (gu[i] - p * u[i]) / nrm[k];
    }
}

/* Sum per-thread partial arrays into dst (fixed thread order). */
static void sum_partials(int64_t len, int nthr, const double *parts, double *dst) {
    for (int64_t i = 0; i < len; ++i) dst[i] = 0.0;
    for (int t = 0; t < nthr; ++t)
        for (int64_t i = 0; i < len; ++i) dst[i] += parts[(size_t)t * (size_t)len + i];
}

static int max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
static int thread_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* Backward of Y = Q X (trans = 0) or Y = Q^T X (trans = 1).
 * dY: upstream gradient.  dX (nullable) and dU (nullable, n x h) are
 * overwritten.                                                           */
EXPORT void orc_apply_bwd(int64_t n, int64_t h, const double *U, int64_t ldu,
                          int trans, const double *X, int64_t ldx,
                          const double *dY, int64_t lddy, int64_t N, double *dX,
                          int64_t lddx, double *dU, int64_t lddu) {
    int64_t hh = h > 0 ? h : 1;
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * hh));
    double *nrm = (double *)malloc(sizeof(double) * (size_t)hh);
    orc_normalize(n, h, U, ldu, Uh, nrm);
    int nthr = max_threads();
    double *parts = (double *)calloc((size_t)nthr * (size_t)(n * hh), sizeof(double));
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)(n * (h + 1)));
        double *g = (double *)malloc(sizeof(double) * (size_t)n);
        double *my = parts + (size_t)thread_id() * (size_t)(n * hh);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t i = 0; i < n; ++i) S[i] = X[i + j * ldx];
            chain_forward(n, h, Uh, trans, S);
            for (int64_t i = 0; i < n; ++i) g[i] = dY[i + j * lddy];
            chain_backward(n, h, Uh, trans, S, g, my);
            if (dX)
                for (int64_t i = 0; i < n; ++i) dX[i + j * lddx] = g[i];
        }
        free(g);
        free(S);
    }
    if (dU && h > 0) {
        double *dUh = (double *)malloc(sizeof(double) * (size_t)(n * h));
        sum_partials(n * h, nthr, parts, dUh);
        normalize_backward(n, h, Uh, nrm, dUh, dU, lddu);
        free(dUh);
    }
    free(parts);
    free(nrm);
    free(Uh);
}

/* Backward of Y = Q diag(lam) Q^T X.  dX, dU, dlam nullable, overwritten. */
EXPORT void orc_sym_bwd(int64_t n, int64_t h, const double *U, int64_t ldu,
                        const double *lam, const double *X, int64_t ldx,
                        const double *dY, int64_t lddy, int64_t N, double *dX,
                        int64_t lddx, double *dU, int64_t lddu, double *dlam) {
    int64_t hh = h > 0 ? h : 1;
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * hh));
    double *nrm = (double *)malloc(sizeof(double) * (size_t)hh);
    orc_normalize(n, h, U, ldu, Uh, nrm);
    int nthr = max_threads();
    int64_t plen = n * hh + n; /* dUh then dlam */
    double *parts = (double *)calloc((size_t)nthr * (size_t)plen, sizeof(double));
#pragma omp parallel
    {
        double *S1 = (double *)malloc(sizeof(double) * (size_t)(n * (h + 1)));
        double *S2 = (double *)malloc(sizeof(double) * (size_t)(n * (h + 1)));
        double *g = (double *)malloc(sizeof(double) * (size_t)n);
        double *my = parts + (size_t)thread_id() * (size_t)plen;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            /* forward: S1 = chain of Q^T, scale, S2 = chain of Q */
            for (int64_t i = 0; i < n; ++i) S1[i] = X[i + j * ldx];
            chain_forward(n, h, Uh, 1, S1);
            const double *z = S1 + h * n;
            for (int64_t i = 0; i < n; ++i) S2[i] = lam[i] * z[i];
            chain_forward(n, h, Uh, 0, S2);
            /* backward */
            for (int64_t i = 0; i < n; ++i) g[i] = dY[i + j * lddy];
            chain_backward(n, h, Uh, 0, S2, g, my);
            for (int64_t i = 0; i < n; ++i) {
                my[n * hh + i] += g[i] * z[i]; /* d(lam_i z_i)/d lam_i = z_i */
                g[i] *= lam[i];
            }
            chain_backward(n, h, Uh, 1, S1, g, my);
            if (dX)
                for (int64_t i = 0; i < n; ++i) dX[i + j * lddx] = g[i];
        }
        free(g);
        free(S2);
        free(S1);
    }
    double *tot = (double *)malloc(sizeof(double) * (size_t)plen);
    sum_partials(plen, nthr, parts, tot);
    if (dU && h > 0) normalize_backward(n, h, Uh, nrm, tot, dU, lddu);
    if (dlam)
        for (int64_t i = 0; i < n; ++i) dlam[i] = tot[n * hh + i];
    free(tot);
    free(parts);
    free(nrm);
    free(Uh);
}

/* Backward of d_j = sum_i lam_i ((Q^T (xa_j - xb_j))_i)^2 with upstream
 * dd_j = dL/dd_j.  dXa, dXb (share lddx), dU, dlam nullable, overwritten. */
EXPORT void orc_mahal_bwd(int64_t n, int64_t h, const double *U, int64_t ldu,
                          const double *lam, const double *Xa, int64_t lda,
                          const double *Xb, int64_t ldb, const double *dd,
                          int64_t N, double *dXa, double *dXb, int64_t lddx,
                          double *dU, int64_t lddu, double *dlam) {
    int64_t hh = h > 0 ? h : 1;
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(n * hh));
    double *nrm = (double *)malloc(sizeof(double) * (size_t)hh);
    orc_normalize(n, h, U, ldu, Uh, nrm);
    int nthr = max_threads();
    int64_t plen = n * hh + n;
    double *parts = (double *)calloc((size_t)nthr * (size_t)plen, sizeof(double));
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)(n * (h + 1)));
        double *g = (double *)malloc(sizeof(double) * (size_t)n);
        double *my = parts + (size_t)thread_id() * (size_t)plen;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t i = 0; i < n; ++i) S[i] = Xa[i + j * lda] - Xb[i + j * ldb];
            chain_forward(n, h, Uh, 1, S);
            const double *z = S + h * n;
            for (int64_t i = 0; i < n; ++i) {
                my[n * hh + i] += dd[j] * z[i] * z[i];
                g[i] = 2.0 * dd[j] * lam[i] * z[i];
            }
            chain_backward(n, h, Uh, 1, S, g, my);
            if (dXa)
                for (int64_t i = 0; i < n; ++i) dXa[i + j * lddx] = g[i];
            if (dXb)
                for (int64_t i = 0; i < n; ++i) dXb[i + j * lddx] = -g[i];
        }
        free(g);
        free(S);
    }
    double *tot = (double *)malloc(sizeof(double) * (size_t)plen);
    sum_partials(plen, nthr, parts, tot);
    if (dU && h > 0) normalize_backward(n, h, Uh, nrm, tot, dU, lddu);
    if (dlam)
        for (int64_t i = 0; i < n; ++i) dlam[i] = tot[n * hh + i];
    free(tot);
    free(parts);
    free(nrm);
    free(Uh);
}

/* ------------------------------------------------------------------ */
/* Householder QR (Golub & Van Loan, Sec. 5.1-5.2, cited by Sec. II-D).
 * Input A (n x n, ld lda) is copied; on return
 *   V (n x (n-1), ld n): unit reflector vectors j_k, with j_k(i) = 0 for
 *     i < k (the leading-zero structure noted after Result 3),
 *   R (n x n, ld n): upper triangular, R = J_{n-1} ... J_1 A,
 * so that A = J_1 ... J_{n-1} R.  For k whose sub-column is already zero
 * the reflector is the zero vector (J_k = I).  v = x + sign(x_1)||x|| e_1
 * with sign(0) = +1.                                                     */
EXPORT void orc_householder_qr(int64_t n, const double *A, int64_t lda,
                               double *V, double *R) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) R[i + j * n] = A[i + j * lda];
    for (int64_t k = 0; k + 1 < n; ++k) {
        double *v = V + k * n;
        for (int64_t i = 0; i < n; ++i) v[i] = 0.0;
        double s = 0.0;
        for (int64_t i = k; i < n; ++i) s += R[i + k * n] * R[i + k * n];
        double nx = sqrt(s);
        if (nx == 0.0) continue;
        double x1 = R[k + k * n];
        double sg = (x1 >= 0.0) ? 1.0 : -1.0;
        for (int64_t i = k; i < n; ++i) v[i] = R[i + k * n];
        v[k] += sg * nx;
        double vv = 0.0;
        for (int64_t i = k; i < n; ++i) vv += v[i] * v[i];
        double vn = sqrt(vv);
        if (vn == 0.0) { v[k] = 0.0; continue; }
        for (int64_t i = k; i < n; ++i) v[i] /= vn;
        /* R <- (I - 2 v v^T) R */
        for (int64_t j = 0; j < n; ++j) {
            double a = 0.0;
            for (int64_t i = k; i < n; ++i) a += v[i] * R[i + j * n];
            for (int64_t i = k; i < n; ++i) R[i + j * n] -= 2.0 * a * v[i];
        }
    }
}

EXPORT int orc_num_threads(void) { return max_threads(); }

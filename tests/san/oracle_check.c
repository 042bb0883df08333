/*
 * Memory and undefined-behaviour check of the FP64 oracle (test
 * infrastructure): built together with oracle/hh_oracle.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer, it calls every exported
 * routine on small inputs in buffers of exactly the documented sizes (leading
 * dimensions larger than n, h = 0, N = 0, a zero reflector) and checks two
 * identities so that a routine that silently did nothing would be noticed:
 * Q^T (Q X) = X, and d(x, x) = 0.  Exit status 0 means clean.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_normalize(int64_t n, int64_t h, const double *U, int64_t ldu, double *Uh, double *nrm);
void orc_apply(int64_t n, int64_t h, const double *U, int64_t ldu, int trans, const double *X,
               int64_t ldx, int64_t N, double *Y, int64_t ldy);
void orc_dense_Q(int64_t n, int64_t h, const double *U, int64_t ldu, double *Q);
void orc_sym(int64_t n, int64_t h, const double *U, int64_t ldu, const double *lam,
             const double *X, int64_t ldx, int64_t N, double *Y, int64_t ldy);
void orc_mahal(int64_t n, int64_t h, const double *U, int64_t ldu, const double *lam,
               const double *Xa, int64_t lda, const double *Xb, int64_t ldb, int64_t N, double *d);
void orc_apply_bwd(int64_t n, int64_t h, const double *U, int64_t ldu, int trans, const double *X,
                   int64_t ldx, const double *dY, int64_t lddy, int64_t N, double *dX,
                   int64_t lddx, double *dU, int64_t lddu);
void orc_sym_bwd(int64_t n, int64_t h, const double *U, int64_t ldu, const double *lam,
                 const double *X, int64_t ldx, const double *dY, int64_t lddy, int64_t N,
                 double *dX, int64_t lddx, double *dU, int64_t lddu, double *dlam);
void orc_mahal_bwd(int64_t n, int64_t h, const double *U, int64_t ldu, const double *lam,
                   const double *Xa, int64_t lda, const double *Xb, int64_t ldb, const double *dd,
                   int64_t N, double *dXa, double *dXb, int64_t lddx, double *dU, int64_t lddu,
                   double *dlam);
void orc_householder_qr(int64_t n, const double *A, int64_t lda, double *V, double *R);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* splitmix64 -> [-1, 1) */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
/* exactly `count` doubles (at least one, so that malloc never returns NULL) */
static double *buf(int64_t count) {
    double *p = (double *)malloc(sizeof(double) * (size_t)(count > 0 ? count : 1));
    for (int64_t i = 0; i < count; ++i) p[i] = urand();
    return p;
}

static int failures = 0;
#define CHECK(c, ...) do { if (!(c)) { ++failures; printf("FAIL: " __VA_ARGS__); printf("\n"); } } while (0)

static void run(int64_t n, int64_t h, int64_t N, int64_t pad, int zero_col) {
    const int64_t ld = n + pad, ldu = n + pad;
    /* a column-major m x c matrix with leading dimension l occupies (c-1) l + m */
    const int64_t sx = N > 0 ? (N - 1) * ld + n : 0, su = h > 0 ? (h - 1) * ldu + n : 0;
    double *U = buf(su), *X = buf(sx), *Xb = buf(sx), *G = buf(sx), *lam = buf(n), *dd = buf(N);
    double *Y = buf(sx), *Z = buf(sx), *dX = buf(sx), *dXb = buf(sx);
    double *dU = buf(su), *dl = buf(n), *d = buf(N), *Uh = buf(n * h), *nrm = buf(h);
    if (zero_col && h > 1)
        for (int64_t i = 0; i < n; ++i) U[i + ldu] = 0.0;
    for (int64_t i = 0; i < n; ++i) lam[i] = 0.5 + fabs(lam[i]);
    orc_normalize(n, h, U, ldu, Uh, nrm);
    orc_apply(n, h, U, ldu, 0, X, ld, N, Y, ld);
    orc_apply(n, h, U, ldu, 1, Y, ld, N, Z, ld);
    double err = 0.0;
    for (int64_t j = 0; j < N; ++j)
        for (int64_t i = 0; i < n; ++i) err = fmax(err, fabs(Z[i + j * ld] - X[i + j * ld]));
    CHECK(err < 1e-12, "Q^T Q X != X (n=%lld h=%lld N=%lld): %g", (long long)n, (long long)h,
          (long long)N, err);
    orc_sym(n, h, U, ldu, lam, X, ld, N, Y, ld);
    orc_mahal(n, h, U, ldu, lam, X, ld, X, ld, N, d);
    for (int64_t j = 0; j < N; ++j) CHECK(d[j] == 0.0, "d(x, x) = %g", d[j]);
    orc_mahal(n, h, U, ldu, lam, X, ld, Xb, ld, N, d);
    for (int trans = 0; trans < 2; ++trans)
        orc_apply_bwd(n, h, U, ldu, trans, X, ld, G, ld, N, dX, ld, dU, ldu);
    orc_sym_bwd(n, h, U, ldu, lam, X, ld, G, ld, N, dX, ld, dU, ldu, dl);
    orc_mahal_bwd(n, h, U, ldu, lam, X, ld, Xb, ld, dd, N, dX, dXb, ld, dU, ldu, dl);
    if (n <= 64) {
        double *Q = buf(n * n);
        orc_dense_Q(n, h, U, ldu, Q);
        double *A = buf((n - 1) * ld + n), *V = buf(n * n), *R = buf(n * n);
        orc_householder_qr(n, A, ld, V, R);
        free(Q); free(A); free(V); free(R);
    }
    free(U); free(X); free(Xb); free(G); free(lam); free(dd); free(Y); free(Z); free(dX);
    free(dXb); free(dU); free(dl); free(d); free(Uh); free(nrm);
}

int main(void) {
    static const int64_t shapes[][3] = {{1, 1, 1}, {2, 3, 5}, {7, 2, 9}, {16, 4, 8}, {33, 0, 4},
                                        {40, 7, 0}, {64, 4, 17}, {5, 9, 3}, {129, 6, 11}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (int64_t pad = 0; pad <= 3; pad += 3)
            for (int zc = 0; zc < 2; ++zc) run(shapes[s][0], shapes[s][1], shapes[s][2], pad, zc);
    printf("oracle sanitizer check: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}

// Symmetric Householder Factorisation (paper Sec. III-B, Algorithm 1: SHF,
// and SHF-SU with the spectrum update of eq. updateofsbar), FP64 on the GPU:
// reflectors u_1 .. u_h, a spectrum sbar and a +-1 diagonal d such that
//   Sbar = D U_1 ... U_h diag(sbar) U_h ... U_1 D      (eq. thesbar)
// approximates a symmetric S in the Frobenius norm; the transform kernels then
// apply Sbar as the symmetric form with d on both sides.
//
// Per reflector k, with A_k = U_{k-1} ... U_1 D S D U_1 ... U_{k-1} (eq. ak)
// and B_k = U_{k+1} ... U_h diag(sbar) U_h ... U_{k+1} (eq. bk), the error is
// ||A_k||^2 + ||B_k||^2 - 2 tr(A_k B_k) + 4 C(u_k) (eq. objectivefunctionS3)
// with C(u) = u^T M u - 2 (u^T A u)(u^T B u), M = A B + B A (eq. theRk).
//   Initialisation (eq. combine): u_dagger, the eigenvector of the smallest
//   eigenvalue of M; u_ddagger from the largest eigenvalue of B (x) A: the
//   extreme eigenpairs of A_k are those of S carried by D and the reflectors
//   before k, those of B_k are sbar's entries carried by the reflectors after k
//   (no eigensolver needed), and V = a b^T has its best symmetric rank-one
//   approximation along a + b or a - b; u_ddagger is made orthogonal to
//   u_dagger and C is minimised over the arc between them.
//   Descent (eqs. gradient and iterate): steps along the great circle through
//   u and the normalised projected gradient, the step length minimising C.
//   D (eq. optimaldiagonal): one entry at a time, the sign that lowers
//   ||S - D B_0 D||^2.
// Along an arc u(gamma) = x1 p + x2 q (p, q orthonormal) C is a quartic in
// (x1, x2) whose coefficients are the 2 x 2 projections of M, A and B, so each
// trial point of a line search costs a few flops after one pass over the
// matrices.  The line searches (the paper uses Matlab's fminbnd) are a
// 65-point grid on [0, sqrt 2] followed by 40 golden-section steps around the
// best grid point; gamma = 0 is on the grid, so no step raises C.
//
// The whole algorithm is one 512-thread block (a set-up step, O(n^3) work
// per initial reflector and O(h n^2) per descent step): matrices live in the
// caller's workspace, eigendecompositions (of S and of each initial M) are a
// cyclic two-sided Jacobi method inside the block.
#include <cmath>

#include "hh_internal.h"

namespace hh {
namespace {

constexpr int kST = 512;
constexpr int kGrid = 65;
constexpr int kGolden = 40;
constexpr int kInner = 20;
constexpr double kInnerTol = 1e-12;
constexpr double kOuterTol = 1e-8;
constexpr int kJacSweeps = 30;
constexpr int kMaxN = 512;

struct ShfWs {
    size_t S, A, B, M, J, V, T, R, s, vmin, vmax, vec, total;
};
constexpr int kVecs = 10;

__host__ __device__ inline ShfWs shf_ws(int64_t n, int64_t h) {
    ShfWs w{};
    const size_t nn = align256((size_t)n * n * 8), v = align256((size_t)n * 8);
    size_t off = 0;
    w.S = off; off += nn;
    w.A = off; off += nn;
    w.B = off; off += nn;
    w.M = off; off += nn;
    w.J = off; off += nn;
    w.V = off; off += nn;
    w.T = off; off += nn;
    w.R = off; off += align256((size_t)n * (h > 0 ? h : 1) * 8);
    w.s = off; off += v;
    w.vmin = off; off += v;
    w.vmax = off; off += v;
    w.vec = off; off += kVecs * v;
    w.total = off;
    return w;
}

struct Shared {
    double red[kST / 64];
    double rc[kMaxN / 2], rs[kMaxN / 2], rp[kMaxN / 2], rq[kMaxN / 2];
    double bcast[8];
};

// Sum over the block; every thread gets the result.
__device__ double bsum(double v, Shared &sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh.red[w] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kST / 64; ++i) r += sh.red[i];
    return r;
}

__device__ double dot(const double *x, const double *y, int n, Shared &sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kST) s += x[i] * y[i];
    return bsum(s, sh);
}

// y = X x for a symmetric (or any, column-major) n x n X.
__device__ void matvec(const double *X, const double *x, double *y, int n) {
    for (int i = threadIdx.x; i < n; i += kST) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += X[i + (int64_t)j * n] * x[j];
        y[i] = s;
    }
    __syncthreads();
}

// X <- (I - 2 u u^T) X (I - 2 u u^T) for symmetric X; w is scratch (n).
__device__ void two_sided(double *X, const double *u, double *w, int n, Shared &sh) {
    matvec(X, u, w, n);
    const double al = dot(u, w, n, sh);
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kST) {
        const int i = (int)(e % n), j = (int)(e / n);
        X[e] -= 2.0 * (u[i] * w[j] + w[i] * u[j]) - 4.0 * al * u[i] * u[j];
    }
    __syncthreads();
}

// x <- (I - 2 u u^T) x
__device__ void reflect_vec(double *x, const double *u, int n, Shared &sh) {
    const double a = dot(u, x, n, sh);
    for (int i = threadIdx.x; i < n; i += kST) x[i] -= 2.0 * a * u[i];
    __syncthreads();
}

// M = A B + B A (A, B symmetric: columns serve as rows).
__device__ void sym_product(const double *A, const double *B, double *M, int n) {
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kST) {
        const int i = (int)(e % n), j = (int)(e / n);
        const double *ai = A + (int64_t)i * n, *bj = B + (int64_t)j * n;
        const double *bi = B + (int64_t)i * n, *aj = A + (int64_t)j * n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += ai[k] * bj[k] + bi[k] * aj[k];
        M[e] = s;
    }
    __syncthreads();
}

// Cyclic two-sided Jacobi on the symmetric J (destroyed: its diagonal ends up
// holding the eigenvalues), eigenvectors in the columns of V.
__device__ void jacobi(double *J, double *V, int n, Shared &sh) {
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kST)
        V[e] = (e % n) == (e / n) ? 1.0 : 0.0;
    __syncthreads();
    if (n < 2) return;
    const int m = n + (n & 1), np = m / 2;
    for (int sweep = 0; sweep < kJacSweeps; ++sweep) {
        double off = 0.0, all = 0.0;
        for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kST) {
            const double v = J[e] * J[e];
            all += v;
            if (e % n != e / n) off += v;
        }
        off = bsum(off, sh);
        all = bsum(all, sh);
        if (off <= 1e-30 * all) break;
        for (int r = 0; r < m - 1; ++r) {
            for (int j = threadIdx.x; j < np; j += kST) {
                int p, q;
                if (j == 0) {
                    p = r;
                    q = m - 1;
                } else {
                    p = (r + j) % (m - 1);
                    q = (r - j + (m - 1)) % (m - 1);
                }
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double app = J[p + (int64_t)p * n], aqq = J[q + (int64_t)q * n];
                    const double apq = J[p + (int64_t)q * n];
                    double t = 0.0;
                    if (apq != 0.0) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                    sh.rp[j] = app - t * apq;  // rotated diagonal entries
                    sh.rq[j] = aqq + t * apq;
                }
                sh.rc[j] = c;
                sh.rs[j] = s;
            }
            __syncthreads();
            // columns p, q of J and V
            for (int64_t e = threadIdx.x; e < (int64_t)np * n; e += kST) {
                const int j = (int)(e / n), i = (int)(e % n);
                const double s = sh.rs[j];
                if (s == 0.0) continue;
                int p, q;
                if (j == 0) { p = r; q = m - 1; } else { p = (r + j) % (m - 1); q = (r - j + (m - 1)) % (m - 1); }
                if (p > q) { const int t = p; p = q; q = t; }
                const double c = sh.rc[j];
                double *jp = J + (int64_t)p * n, *jq = J + (int64_t)q * n;
                const double x = jp[i], y = jq[i];
                jp[i] = c * x - s * y;
                jq[i] = s * x + c * y;
                double *vp = V + (int64_t)p * n, *vq = V + (int64_t)q * n;
                const double u = vp[i], w = vq[i];
                vp[i] = c * u - s * w;
                vq[i] = s * u + c * w;
            }
            __syncthreads();
            // rows p, q of J; the 2 x 2 block set to its exact rotated value
            for (int64_t e = threadIdx.x; e < (int64_t)np * n; e += kST) {
                const int j = (int)(e / n), i = (int)(e % n);
                const double s = sh.rs[j];
                if (s == 0.0) continue;
                int p, q;
                if (j == 0) { p = r; q = m - 1; } else { p = (r + j) % (m - 1); q = (r - j + (m - 1)) % (m - 1); }
                if (p > q) { const int t = p; p = q; q = t; }
                const double c = sh.rc[j];
                if (i == p || i == q) {
                    if (i == p) {
                        J[p + (int64_t)p * n] = sh.rp[j];
                        J[q + (int64_t)q * n] = sh.rq[j];
                        J[p + (int64_t)q * n] = 0.0;
                        J[q + (int64_t)p * n] = 0.0;
                    }
                    continue;
                }
                const double x = J[p + (int64_t)i * n], y = J[q + (int64_t)i * n];
                J[p + (int64_t)i * n] = c * x - s * y;
                J[q + (int64_t)i * n] = s * x + c * y;
            }
            __syncthreads();
        }
    }
}

// The 2 x 2 projections along the arc through orthonormal p, q:
// P[0..2] = (p^T X p, p^T X q, q^T X q) for X = M, A, B.
struct Arc {
    double m0, m1, m2, a0, a1, a2, b0, b1, b2;
    __device__ double c_at(double g, double sg) const {
        const double x1 = 1.0 - 0.5 * g * g;
        const double x2 = sg * sqrt(fmax(g * g - 0.25 * g * g * g * g, 0.0));
        const double qm = x1 * x1 * m0 + 2.0 * x1 * x2 * m1 + x2 * x2 * m2;
        const double qa = x1 * x1 * a0 + 2.0 * x1 * x2 * a1 + x2 * x2 * a2;
        const double qb = x1 * x1 * b0 + 2.0 * x1 * x2 * b1 + x2 * x2 * b2;
        return qm - 2.0 * qa * qb;
    }
};

// pX = X p, qX = X q are given (matvecs); returns the projections.
__device__ Arc arc_of(const double *p, const double *q, const double *Mp, const double *Mq,
                      const double *Ap, const double *Aq, const double *Bp, const double *Bq,
                      int n, Shared &sh) {
    Arc a;
    a.m0 = dot(p, Mp, n, sh);
    a.m1 = dot(p, Mq, n, sh);
    a.m2 = dot(q, Mq, n, sh);
    a.a0 = dot(p, Ap, n, sh);
    a.a1 = dot(p, Aq, n, sh);
    a.a2 = dot(q, Aq, n, sh);
    a.b0 = dot(p, Bp, n, sh);
    a.b1 = dot(p, Bq, n, sh);
    a.b2 = dot(q, Bq, n, sh);
    return a;
}

// Grid plus golden section over gamma in [0, sqrt 2]; every thread computes
// the same (uniform) result.
__device__ void line_search(const Arc &arc, double sg, double *gbest, double *cbest) {
    const double top = sqrt(2.0);
    int bi = 0;
    double bv = arc.c_at(0.0, sg);
    for (int i = 1; i < kGrid; ++i) {
        const double v = arc.c_at(top * i / (kGrid - 1), sg);
        if (v < bv) {
            bv = v;
            bi = i;
        }
    }
    double lo = top * (bi > 0 ? bi - 1 : 0) / (kGrid - 1);
    double hi = top * (bi < kGrid - 1 ? bi + 1 : kGrid - 1) / (kGrid - 1);
    double bx = top * bi / (kGrid - 1);
    const double r = (sqrt(5.0) - 1.0) / 2.0;
    double x1 = hi - r * (hi - lo), x2 = lo + r * (hi - lo);
    double f1 = arc.c_at(x1, sg), f2 = arc.c_at(x2, sg);
    for (int it = 0; it < kGolden; ++it) {
        if (f1 <= f2) {
            hi = x2; x2 = x1; f2 = f1;
            x1 = hi - r * (hi - lo);
            f1 = arc.c_at(x1, sg);
        } else {
            lo = x1; x1 = x2; f1 = f2;
            x2 = lo + r * (hi - lo);
            f2 = arc.c_at(x2, sg);
        }
    }
    if (f1 < bv) { bv = f1; bx = x1; }
    if (f2 < bv) { bv = f2; bx = x2; }
    *gbest = bx;
    *cbest = bv;
}

struct ShfArgs {
    const double *S_in;
    int64_t lds;
    double *R;      // n x h output reflectors, ld ldr
    int64_t ldr;
    double *sbar_out, *d_out, *err;
    char *ws;
    int n, h, K, su;
};

__global__ __launch_bounds__(kST) void k_shf(ShfArgs a) {
    __shared__ Shared sh;
    const int n = a.n, h = a.h, tid = threadIdx.x;
    const ShfWs L = shf_ws(n, h);
    double *S = reinterpret_cast<double *>(a.ws + L.S);
    double *A = reinterpret_cast<double *>(a.ws + L.A);
    double *B = reinterpret_cast<double *>(a.ws + L.B);
    double *M = reinterpret_cast<double *>(a.ws + L.M);
    double *J = reinterpret_cast<double *>(a.ws + L.J);
    double *V = reinterpret_cast<double *>(a.ws + L.V);
    double *T = reinterpret_cast<double *>(a.ws + L.T);
    double *U = reinterpret_cast<double *>(a.ws + L.R);  // reflector k at U + k n
    double *sv = reinterpret_cast<double *>(a.ws + L.s);
    double *vmin = reinterpret_cast<double *>(a.ws + L.vmin);
    double *vmax = reinterpret_cast<double *>(a.ws + L.vmax);
    double *vec = reinterpret_cast<double *>(a.ws + L.vec);
    const size_t vs = align256((size_t)n * 8) / 8;
    double *p = vec, *q = vec + vs, *Mp = vec + 2 * vs, *Mq = vec + 3 * vs, *Ap = vec + 4 * vs,
           *Aq = vec + 5 * vs, *Bp = vec + 6 * vs, *Bq = vec + 7 * vs, *w = vec + 8 * vs,
           *w2 = vec + 9 * vs;
    double *sbar = a.sbar_out, *d = a.d_out;

    // Step 1: eigenvalues of S, ordered by decreasing magnitude, and its
    // extreme eigenvectors.
    for (int64_t e = tid; e < (int64_t)n * n; e += kST) {
        const double v = a.S_in[(e % n) + (e / n) * a.lds];
        S[e] = v;
        J[e] = v;
    }
    __syncthreads();
    jacobi(J, V, n, sh);
    for (int i = tid; i < n; i += kST) {
        const double zi = J[i + (int64_t)i * n];
        int rank = 0, rlo = 0, rhi = 0;
        for (int j = 0; j < n; ++j) {
            const double zj = J[j + (int64_t)j * n];
            // |z| descending, ties by ascending value, then index
            const bool before = fabs(zj) > fabs(zi) || (fabs(zj) == fabs(zi) && (zj < zi || (zj == zi && j < i)));
            rank += before ? 1 : 0;
            rlo += (zj < zi || (zj == zi && j < i)) ? 1 : 0;
            rhi += (zj > zi || (zj == zi && j < i)) ? 1 : 0;
        }
        sbar[rank] = zi;
        if (rlo == 0) sh.bcast[1] = (double)i;  // smallest eigenvalue's index
        if (rhi == 0) sh.bcast[2] = (double)i;  // largest
    }
    __syncthreads();
    {
        const int imin = (int)sh.bcast[1], imax = (int)sh.bcast[2];
        for (int i = tid; i < n; i += kST) {
            sv[i] = sbar[i];
            vmin[i] = V[i + (int64_t)imin * n];
            vmax[i] = V[i + (int64_t)imax * n];
        }
        if (tid == 0) {
            sh.bcast[3] = J[imin + (int64_t)imin * n];
            sh.bcast[4] = J[imax + (int64_t)imax * n];
        }
    }
    for (int i = tid; i < n; i += kST) d[i] = 1.0;
    for (int64_t e = tid; e < (int64_t)n * h; e += kST) U[e] = 0.0;
    __syncthreads();
    const double smin = sh.bcast[3], smax = sh.bcast[4];

    auto build_DSD = [&]() {  // A = D S D
        for (int64_t e = tid; e < (int64_t)n * n; e += kST) A[e] = d[e % n] * S[e] * d[e / n];
        __syncthreads();
    };
    auto build_B = [&](int k, double *X) {  // X = U_{k+1} .. U_h diag(sbar) U_h .. U_{k+1}
        for (int64_t e = tid; e < (int64_t)n * n; e += kST)
            X[e] = (e % n) == (e / n) ? sbar[e % n] : 0.0;
        __syncthreads();
        for (int j = h - 1; j > k; --j) two_sided(X, U + (int64_t)j * n, w, n, sh);
    };
    auto error = [&]() {  // ||S - D B_0 D||_F^2
        build_B(-1, T);
        double s = 0.0;
        for (int64_t e = tid; e < (int64_t)n * n; e += kST) {
            const double r = S[e] - d[e % n] * T[e] * d[e / n];
            s += r * r;
        }
        return bsum(s, sh);
    };
    auto update_D = [&]() {  // eq. optimaldiagonal, one entry at a time
        build_B(-1, T);
        for (int i = 0; i < n; ++i) {
            double sp = 0.0, sm = 0.0;
            for (int j = tid; j < n; j += kST) {
                if (j == i) continue;
                const double b = d[i] * d[j] * T[i + (int64_t)j * n], s = S[i + (int64_t)j * n];
                sp += (s + b) * (s + b);
                sm += (s - b) * (s - b);
            }
            sp = bsum(sp, sh);
            sm = bsum(sm, sh);
            if (sqrt(sp) < sqrt(sm) && tid == 0) d[i] = -d[i];
            __syncthreads();
        }
    };
    auto spectrum_update = [&]() {  // eq. updateofsbar: sbar = diag(Ubar^T S Ubar)
        build_DSD();
        for (int j = 0; j < h; ++j) two_sided(A, U + (int64_t)j * n, w, n, sh);
        for (int i = tid; i < n; i += kST) sbar[i] = A[i + (int64_t)i * n];
        __syncthreads();
    };
    // u = x1 p + x2 q into dst
    auto arc_point = [&](double g, double sg, double *dst) {
        const double x1 = 1.0 - 0.5 * g * g;
        const double x2 = sg * sqrt(fmax(g * g - 0.25 * g * g * g * g, 0.0));
        for (int i = tid; i < n; i += kST) dst[i] = x1 * p[i] + x2 * q[i];
        __syncthreads();
    };
    auto arc_prepare = [&]() {
        matvec(M, p, Mp, n);
        matvec(M, q, Mq, n);
        matvec(A, p, Ap, n);
        matvec(A, q, Aq, n);
        matvec(B, p, Bp, n);
        matvec(B, q, Bq, n);
        return arc_of(p, q, Mp, Mq, Ap, Aq, Bp, Bq, n, sh);
    };

    // Step 2: initial reflectors (eq. combine), then D (and sbar for SHF-SU).
    build_DSD();
    for (int k = 0; k < h; ++k) {
        double *uk = U + (int64_t)k * n;
        build_B(k, B);
        sym_product(A, B, M, n);
        for (int64_t e = tid; e < (int64_t)n * n; e += kST) J[e] = M[e];
        __syncthreads();
        jacobi(J, V, n, sh);
        // u_dagger: eigenvector of the smallest eigenvalue of M
        if (tid == 0) {
            int im = 0;
            for (int j = 1; j < n; ++j)
                if (J[j + (int64_t)j * n] < J[im + (int64_t)im * n]) im = j;
            sh.bcast[5] = (double)im;
        }
        __syncthreads();
        const int im = (int)sh.bcast[5];
        for (int i = tid; i < n; i += kST) p[i] = V[i + (int64_t)im * n];
        // extreme eigenpairs of A_k: those of S carried by D, U_1 .. U_{k-1}
        for (int i = tid; i < n; i += kST) {
            Ap[i] = d[i] * vmin[i];
            Aq[i] = d[i] * vmax[i];
        }
        __syncthreads();
        for (int j = 0; j < k; ++j) {
            reflect_vec(Ap, U + (int64_t)j * n, n, sh);
            reflect_vec(Aq, U + (int64_t)j * n, n, sh);
        }
        // of B_k: sbar's extreme entries carried by U_h .. U_{k+1}
        int bmin = 0, bmax = 0;
        for (int j = 1; j < n; ++j) {
            if (sbar[j] < sbar[bmin]) bmin = j;
            if (sbar[j] > sbar[bmax]) bmax = j;
        }
        for (int i = tid; i < n; i += kST) {
            Bp[i] = i == bmin ? 1.0 : 0.0;
            Bq[i] = i == bmax ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int j = h - 1; j > k; --j) {
            reflect_vec(Bp, U + (int64_t)j * n, n, sh);
            reflect_vec(Bq, U + (int64_t)j * n, n, sh);
        }
        const double lb0 = sbar[bmin], lb1 = sbar[bmax];
        // the largest of the four products (first in the order min.min,
        // min.max, max.min, max.max on ties)
        const double cand[4] = {smin * lb0, smin * lb1, smax * lb0, smax * lb1};
        int ci = 0;
        for (int c = 1; c < 4; ++c)
            if (cand[c] > cand[ci]) ci = c;
        const double *va = ci < 2 ? Ap : Aq, *vb = (ci & 1) ? Bq : Bp;
        // u_ddagger along a + b or a - b, the larger (u^T A u)(u^T B u)
        double bestq = -INFINITY, bsg = 0.0;
        for (int c = 0; c < 2; ++c) {
            const double sg = c == 0 ? 1.0 : -1.0;
            for (int i = tid; i < n; i += kST) w2[i] = va[i] + sg * vb[i];
            __syncthreads();
            const double nv = sqrt(dot(w2, w2, n, sh));
            if (nv < 1e-12) continue;
            for (int i = tid; i < n; i += kST) w2[i] /= nv;
            __syncthreads();
            matvec(A, w2, w, n);
            const double qa = dot(w2, w, n, sh);
            matvec(B, w2, w, n);
            const double qb = dot(w2, w, n, sh);
            if (qa * qb > bestq) {
                bestq = qa * qb;
                bsg = sg;
            }
        }
        for (int i = tid; i < n; i += kST) q[i] = va[i] + bsg * vb[i];
        __syncthreads();
        const double nq0 = sqrt(dot(q, q, n, sh));
        for (int i = tid; i < n; i += kST) q[i] /= nq0;
        __syncthreads();
        const double pq = dot(p, q, n, sh);  // eq. processtheinitial
        for (int i = tid; i < n; i += kST) q[i] -= pq * p[i];
        __syncthreads();
        const double nq = sqrt(dot(q, q, n, sh));
        if (nq < 1e-12) {
            for (int i = tid; i < n; i += kST) uk[i] = p[i];
        } else {
            for (int i = tid; i < n; i += kST) q[i] /= nq;
            __syncthreads();
            const Arc arc = arc_prepare();
            double bg = 0.0, bs = 1.0, bc = arc.c_at(0.0, 1.0);
            for (int c = 0; c < 2; ++c) {
                const double sg = c == 0 ? 1.0 : -1.0;
                double g, cv;
                line_search(arc, sg, &g, &cv);
                if (cv < bc) {
                    bc = cv;
                    bg = g;
                    bs = sg;
                }
            }
            arc_point(bg, bs, uk);
        }
        __syncthreads();
        two_sided(A, uk, w, n, sh);  // A_{k+1}
    }
    update_D();
    if (a.su) spectrum_update();
    double prev = error();
    if (a.err && tid == 0) a.err[0] = prev;
    int done = 0;
    // Step 3: K sweeps of descent over the reflectors, then D (and sbar).
    for (int it = 1; it <= a.K; ++it) {
        if (!done) {
            build_DSD();
            for (int k = 0; k < h; ++k) {
                double *uk = U + (int64_t)k * n;
                build_B(k, B);
                sym_product(A, B, M, n);
                // C at the current point
                for (int i = tid; i < n; i += kST) p[i] = uk[i];
                __syncthreads();
                matvec(M, p, Mp, n);
                matvec(A, p, Ap, n);
                matvec(B, p, Bp, n);
                double c = dot(p, Mp, n, sh) - 2.0 * dot(p, Ap, n, sh) * dot(p, Bp, n, sh);
                for (int step = 0; step < kInner; ++step) {
                    // projected, normalised gradient (eq. gradient)
                    const double pa = dot(p, Ap, n, sh), pb = dot(p, Bp, n, sh);
                    for (int i = tid; i < n; i += kST) q[i] = 2.0 * Mp[i] - 4.0 * (pa * Bp[i] + pb * Ap[i]);
                    __syncthreads();
                    const double pg = dot(p, q, n, sh);
                    for (int i = tid; i < n; i += kST) q[i] -= pg * p[i];
                    __syncthreads();
                    const double ng = sqrt(dot(q, q, n, sh));
                    if (ng < 1e-14) break;
                    for (int i = tid; i < n; i += kST) q[i] /= ng;
                    __syncthreads();
                    matvec(M, q, Mq, n);
                    matvec(A, q, Aq, n);
                    matvec(B, q, Bq, n);
                    const Arc arc = arc_of(p, q, Mp, Mq, Ap, Aq, Bp, Bq, n, sh);
                    double g, cv;
                    line_search(arc, -1.0, &g, &cv);  // eq. iterate
                    const bool last = c - cv <= kInnerTol * fmax(1.0, fabs(c));
                    if (last && !(cv < c)) break;
                    // move: p <- (1 - g^2/2) p - sqrt(g^2 - g^4/4) q, and the
                    // products follow linearly
                    const double x1 = 1.0 - 0.5 * g * g;
                    const double x2 = -sqrt(fmax(g * g - 0.25 * g * g * g * g, 0.0));
                    for (int i = tid; i < n; i += kST) {
                        p[i] = x1 * p[i] + x2 * q[i];
                        Mp[i] = x1 * Mp[i] + x2 * Mq[i];
                        Ap[i] = x1 * Ap[i] + x2 * Aq[i];
                        Bp[i] = x1 * Bp[i] + x2 * Bq[i];
                    }
                    __syncthreads();
                    c = cv;
                    if (last) break;
                }
                for (int i = tid; i < n; i += kST) uk[i] = p[i];
                __syncthreads();
                two_sided(A, uk, w, n, sh);
            }
            update_D();
            if (a.su) spectrum_update();
            const double e = error();
            if (prev - e < kOuterTol * prev) done = 1;
            prev = e;
        }
        if (a.err && tid == 0) a.err[it] = prev;
    }
    for (int64_t e = tid; e < (int64_t)n * h; e += kST)
        a.R[(e % n) + (e / n) * a.ldr] = U[e];
}

}  // namespace
}  // namespace hh

using namespace hh;

extern "C" {

hh_status hh_shf_workspace_size(int64_t n, int64_t h, int64_t K, size_t *bytes) {
    if (!bytes) return set_error(HH_ERR_INVALID_ARG, "bytes must not be null");
    if (n < 1 || h < 0 || K < 0) return set_error(HH_ERR_INVALID_ARG, "need n >= 1, h >= 0, K >= 0");
    if (n > kMaxN) return set_error(HH_ERR_UNSUPPORTED, "SHF supports n <= %d (n = %lld)", kMaxN, (long long)n);
    if (K > 100000) return set_error(HH_ERR_UNSUPPORTED, "K must be <= 100000");
    *bytes = shf_ws(n, h).total;
    return HH_OK;
}

hh_status hh_shf(int64_t n, int64_t h, int64_t K, int spectrum_update, const double *S, int64_t lds,
                 double *R, int64_t ldr, double *sbar, double *d, double *err, void *ws,
                 size_t ws_bytes, hipStream_t st) {
    size_t need = 0;
    const hh_status s = hh_shf_workspace_size(n, h, K, &need);
    if (s != HH_OK) return s;
    if (!S || !sbar || !d || !ws) return set_error(HH_ERR_INVALID_ARG, "S, sbar, d and ws must not be null");
    if (lds < n) return set_error(HH_ERR_INVALID_ARG, "lds must be >= n");
    if (h > 0 && (!R || ldr < n)) return set_error(HH_ERR_INVALID_ARG, "R must not be null and ldr >= n");
    if (ws_bytes < need)
        return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
    ShfArgs a{};
    a.S_in = S;
    a.lds = lds;
    a.R = R;
    a.ldr = ldr;
    a.sbar_out = sbar;
    a.d_out = d;
    a.err = err;
    a.ws = static_cast<char *>(ws);
    a.n = (int)n;
    a.h = (int)h;
    a.K = (int)K;
    a.su = spectrum_update ? 1 : 0;
    hipLaunchKernelGGL(k_shf, dim3(1), dim3(kST), 0, st, a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HH_OK : set_error(HH_ERR_HIP, "SHF launch: %s", hipGetErrorString(e));
}

}  // extern "C"

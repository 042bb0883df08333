// Orthonormal factorisation front-end (paper Sec. II-B to II-D), FP64 on the
// GPU: the reflectors that approximate a given orthonormal n x n matrix U and
// feed the transform kernels.
//
//   HH_FACTOR_CONSTRAINED (Result 1): mutually orthogonal reflectors, the
//     eigenvectors of the negative eigenvalues of Z = U + U^T, smallest first.
//   HH_FACTOR_UNCONSTRAINED (Result 2): along the spectrum of Z, Case 1 (an
//     eigenvalue -1 of U, z = -2) gives one reflector, the eigenvector;
//     Case 2 (a pair lam = alpha +- i beta of U, z = 2 alpha twice) gives two,
//     u1 = sqrt(2) Re t and u2 = 2 (gamma Re t - delta Im t) with t the
//     eigenvector of the beta > 0 member, gamma = -sqrt(1 + alpha) / 2,
//     delta = -sqrt(1 - alpha) / 2 (eq. theu2).  The invariant plane of a pair
//     is the eigenspace of Z at 2 alpha: with a unit a in it, U a = alpha a +
//     s b for the unit b of that plane orthogonal to a, and t = (a + i b) /
//     sqrt(2) is an eigenvector of U for alpha - i s, so b is oriented to make
//     s < 0 (beta > 0); then u1 = a and u2 = sqrt(2) (gamma a - delta b).  The
//     construction multiplies each new reflector on the left (Ubar = U_m ...
//     U_1), so the output lists them in reverse order for Q = H_1 ... H_h.
//   HH_FACTOR_QR (Result 3): the first h reflectors of the textbook
//     Householder QR of U (v = x + sign(x_1) ||x|| e_1, sign(0) = +1) and the
//     +-1 diagonal d of the signs of the diagonal of J_h ... J_1 U, so that
//     U ~ (J_1 ... J_h) diag(d) (eqs. ReflectorStructure and theU2).
//
// The symmetric eigendecomposition is a cyclic two-sided Jacobi method (each
// sweep a round-robin tournament of n - 1 rounds of n/2 disjoint rotations,
// Golub & Van Loan Sec. 8.5): per round one kernel computes the rotations and
// applies them to the columns of Z and of the eigenvector matrix, a second
// applies them to the rows.  After each sweep a one-block kernel compares the
// off-diagonal norm with the whole norm; once converged the remaining launches
// return at once.
#include <cmath>
#include <cstring>

#include "hh_internal.h"

namespace hh {
namespace {

constexpr int kFT = 256;         // threads per block
constexpr int kMaxSweeps = 16;   // cyclic Jacobi in FP64 converges in well under this
constexpr double kOffTol = 1e-15;

struct FactorWs {
    size_t A, V, rot, flag, perm, zs, total;
};

inline FactorWs factor_ws(int64_t n) {
    FactorWs w{};
    const size_t nn = (size_t)n * n * 8, m = (size_t)(n + 1) / 2;
    size_t off = 0;
    w.A = off;    off += align256(nn);
    w.V = off;    off += align256(nn);
    w.rot = off;  off += align256(m * 4 * 8);
    w.flag = off; off += align256(16);
    w.perm = off; off += align256((size_t)n * 4);
    w.zs = off;   off += align256((size_t)n * 8);
    w.total = off;
    return w;
}

// Pair j of round r of the round-robin tournament on m (even) players:
// player m-1 stays, the others rotate.
__device__ __forceinline__ void tour_pair(int r, int j, int m, int *p, int *q) {
    if (j == 0) {
        *p = r;
        *q = m - 1;
    } else {
        *p = (r + j) % (m - 1);
        *q = (r - j + (m - 1)) % (m - 1);
    }
    if (*p > *q) {
        const int t = *p;
        *p = *q;
        *q = t;
    }
}

__device__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kFT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// A = U + U^T, V = I, not converged.
__global__ __launch_bounds__(kFT) void k_sym_sum(const double *__restrict__ U, int64_t ldu, int n,
                                                double *__restrict__ A, double *__restrict__ V,
                                                int *__restrict__ flag) {
    const int64_t e = (int64_t)blockIdx.x * kFT + threadIdx.x;
    if (e == 0) flag[0] = 0;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e % n), j = (int)(e / n);
    A[e] = U[i + j * ldu] + U[j + i * ldu];
    V[e] = i == j ? 1.0 : 0.0;
}

// Round r: rotation of pair (p, q) from the current a_pp, a_qq, a_pq
// (Golub & Van Loan, sym.schur2), then A <- A J and V <- V J on columns p, q.
__global__ __launch_bounds__(kFT) void k_jac_cols(double *__restrict__ A, double *__restrict__ V,
                                                 int n, int m, int r, double *__restrict__ rot,
                                                 const int *__restrict__ flag) {
    if (flag[0]) return;
    int p, q;
    tour_pair(r, blockIdx.x, m, &p, &q);
    if (q >= n) return;  // the idle player of an odd n
    __shared__ double cs[4];
    if (threadIdx.x == 0) {
        const double app = A[p + (int64_t)p * n], aqq = A[q + (int64_t)q * n];
        const double apq = A[p + (int64_t)q * n];
        double c = 1.0, s = 0.0, t = 0.0;
        if (apq != 0.0) {
            const double tau = (aqq - app) / (2.0 * apq);
            t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
        }
        cs[0] = c;
        cs[1] = s;
        double *o = rot + 4 * blockIdx.x;
        o[0] = c;
        o[1] = s;
        o[2] = app - t * apq;  // the rotated diagonal entries
        o[3] = aqq + t * apq;
    }
    __syncthreads();
    const double c = cs[0], s = cs[1];
    if (s == 0.0) return;
    double *ap = A + (int64_t)p * n, *aq = A + (int64_t)q * n;
    double *vp = V + (int64_t)p * n, *vq = V + (int64_t)q * n;
    for (int i = threadIdx.x; i < n; i += kFT) {
        const double x = ap[i], y = aq[i];
        ap[i] = c * x - s * y;
        aq[i] = s * x + c * y;
        const double u = vp[i], w = vq[i];
        vp[i] = c * u - s * w;
        vq[i] = s * u + c * w;
    }
}

// Round r: A <- J^T A on rows p, q; the 2 x 2 block is set to its exact
// rotated value (zero off the diagonal).
__global__ __launch_bounds__(kFT) void k_jac_rows(double *__restrict__ A, int n, int m, int r,
                                                 const double *__restrict__ rot,
                                                 const int *__restrict__ flag) {
    if (flag[0]) return;
    int p, q;
    tour_pair(r, blockIdx.x, m, &p, &q);
    if (q >= n) return;
    const double *o = rot + 4 * blockIdx.x;
    const double c = o[0], s = o[1];
    if (s == 0.0) return;
    for (int i = threadIdx.x; i < n; i += kFT) {
        if (i == p || i == q) continue;
        const double x = A[p + (int64_t)i * n], y = A[q + (int64_t)i * n];
        A[p + (int64_t)i * n] = c * x - s * y;
        A[q + (int64_t)i * n] = s * x + c * y;
    }
    if (threadIdx.x == 0) {
        A[p + (int64_t)p * n] = o[2];
        A[q + (int64_t)q * n] = o[3];
        A[p + (int64_t)q * n] = 0.0;
        A[q + (int64_t)p * n] = 0.0;
    }
}

// Converged when the off-diagonal norm is below kOffTol times the whole norm.
__global__ __launch_bounds__(kFT) void k_jac_check(const double *__restrict__ A, int n,
                                                  int *__restrict__ flag) {
    __shared__ double red[kFT];
    if (flag[0]) return;
    double off = 0.0, all = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kFT) {
        const double v = A[e] * A[e];
        all += v;
        if (e % n != e / n) off += v;
    }
    off = block_sum(off, red);
    all = block_sum(all, red);
    if (threadIdx.x == 0 && off <= kOffTol * kOffTol * all) flag[0] = 1;
}

// Eigenvalues in ascending order (ties by index): zs[rank] = a_ii, perm[rank] = i.
__global__ __launch_bounds__(kFT) void k_eig_sort(const double *__restrict__ A, int n,
                                                 double *__restrict__ zs, int *__restrict__ perm,
                                                 double *__restrict__ zout) {
    for (int i = threadIdx.x; i < n; i += kFT) {
        const double zi = A[i + (int64_t)i * n];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double zj = A[j + (int64_t)j * n];
            rank += (zj < zi || (zj == zi && j < i)) ? 1 : 0;
        }
        zs[rank] = zi;
        perm[rank] = i;
        if (zout) zout[rank] = zi;
    }
}

// Result 1: column k of R is the eigenvector of the k-th smallest eigenvalue
// when that eigenvalue is negative, else zero.
__global__ __launch_bounds__(kFT) void k_constrained(const double *__restrict__ V, int n, int h,
                                                    const double *__restrict__ zs,
                                                    const int *__restrict__ perm,
                                                    double *__restrict__ R, int64_t ldr) {
    const int k = blockIdx.x;
    const bool use = k < n && zs[k] < 0.0;
    const double *v = use ? V + (int64_t)perm[k] * n : nullptr;
    for (int i = threadIdx.x; i < n; i += kFT) R[i + k * ldr] = use ? v[i] : 0.0;
}

// Result 2, one block: walks the sorted spectrum, writes the reflectors in
// construction order into L (n x n), then reverses them into R.
__global__ __launch_bounds__(kFT) void k_unconstrained(const double *__restrict__ U, int64_t ldu,
                                                      const double *__restrict__ V, int n, int h,
                                                      const double *__restrict__ zs,
                                                      const int *__restrict__ perm,
                                                      double *__restrict__ L,
                                                      double *__restrict__ R, int64_t ldr) {
    __shared__ double red[kFT];
    extern __shared__ double wv[];  // U a, n values
    int cnt = 0, mi = 0;
    while (mi < n && cnt < h && zs[mi] < 0.0) {
        const double *a = V + (int64_t)perm[mi] * n;
        if (zs[mi] < -2.0 + 1e-9) {  // Case 1: U a = -a
            for (int i = threadIdx.x; i < n; i += kFT) L[i + (int64_t)cnt * n] = a[i];
            ++cnt;
            ++mi;
            __syncthreads();
            continue;
        }
        // Case 2: w = U a, alpha = a^T U a, b = the unit part of w orthogonal to a
        double da = 0.0;
        for (int i = threadIdx.x; i < n; i += kFT) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += U[i + (int64_t)j * ldu] * a[j];
            wv[i] = s;
            da += s * a[i];
        }
        const double alpha = block_sum(da, red);
        double nw = 0.0;
        for (int i = threadIdx.x; i < n; i += kFT) {
            const double r = wv[i] - alpha * a[i];
            nw += r * r;
        }
        nw = sqrt(block_sum(nw, red));
        const bool from_w = nw > 1e-8;
        const double *a2 = (mi + 1 < n) ? V + (int64_t)perm[mi + 1] * n : a;
        // the partner eigenvector is the fallback b (degenerate plane)
        double sb = 0.0;
        for (int i = threadIdx.x; i < n; i += kFT) {
            const double b = from_w ? (wv[i] - alpha * a[i]) / nw : a2[i];
            sb += b * wv[i];  // s = b^T U a
        }
        sb = block_sum(sb, red);
        const double sg = sb > 0.0 ? -1.0 : 1.0;  // orient b so that s < 0 (beta > 0)
        const double ga = -sqrt(fmax(0.0, 1.0 + alpha)) * 0.5;
        const double de = -sqrt(fmax(0.0, 1.0 - alpha)) * 0.5;
        for (int i = threadIdx.x; i < n; i += kFT) {
            const double b = sg * (from_w ? (wv[i] - alpha * a[i]) / nw : a2[i]);
            L[i + (int64_t)cnt * n] = a[i];
            if (cnt + 1 < h) L[i + (int64_t)(cnt + 1) * n] = sqrt(2.0) * (ga * a[i] - de * b);
        }
        cnt += cnt + 1 < h ? 2 : 1;
        mi += 2;
        __syncthreads();
    }
    __syncthreads();
    for (int k = 0; k < h; ++k)
        for (int i = threadIdx.x; i < n; i += kFT)
            R[i + (int64_t)k * ldr] = k < cnt ? L[i + (int64_t)(cnt - 1 - k) * n] : 0.0;
}

// Result 3, step k: the reflector that zeroes column k of W below row k:
// v = x + sign(x_k) ||x|| e_k over rows k .. n-1, u = v / ||v|| (zero when
// the column is already zero), ||v||^2 = ||x||^2 - x_k^2 + (x_k +- ||x||)^2.
__global__ __launch_bounds__(kFT) void k_qr_refl(const double *__restrict__ W, int n, int k,
                                                double *__restrict__ R, int64_t ldr) {
    __shared__ double red[kFT];
    const double *x = W + (int64_t)k * n;
    double s = 0.0;
    for (int i = k + threadIdx.x; i < n; i += kFT) s += x[i] * x[i];
    const double ss = block_sum(s, red);
    const double nx = sqrt(ss);
    const double x1 = x[k];
    const double top = x1 + (x1 >= 0.0 ? nx : -nx);
    const double nv2 = ss - x1 * x1 + top * top;
    const double nv = (nx == 0.0 || nv2 <= 0.0) ? 0.0 : sqrt(nv2);
    double *u = R + (int64_t)k * ldr;
    for (int i = threadIdx.x; i < n; i += kFT) {
        double v = 0.0;
        if (nv > 0.0 && i >= k) v = (i == k ? top : x[i]) / nv;
        u[i] = v;
    }
}

// Result 3, step k: W <- (I - 2 u u^T) W on columns k .. n-1.
__global__ __launch_bounds__(kFT) void k_qr_apply(double *__restrict__ W, int n, int k,
                                                 const double *__restrict__ R, int64_t ldr) {
    __shared__ double red[kFT];
    const int j = k + blockIdx.x;
    const double *u = R + (int64_t)k * ldr;
    double *w = W + (int64_t)j * n;
    double s = 0.0;
    for (int i = k + threadIdx.x; i < n; i += kFT) s += u[i] * w[i];
    const double a = 2.0 * block_sum(s, red);
    for (int i = k + threadIdx.x; i < n; i += kFT) w[i] -= a * u[i];
}

__global__ __launch_bounds__(kFT) void k_copy_mat(const double *__restrict__ U, int64_t ldu, int n,
                                                 double *__restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * kFT + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    W[e] = U[(e % n) + (e / n) * ldu];
}

__global__ __launch_bounds__(kFT) void k_diag_sign(const double *__restrict__ W, int n,
                                                  double *__restrict__ d, int ones) {
    const int i = blockIdx.x * kFT + threadIdx.x;
    if (i < n) d[i] = (ones || W[i + (int64_t)i * n] >= 0.0) ? 1.0 : -1.0;
}

int mat_blocks(int n) { return (int)(((int64_t)n * n + kFT - 1) / kFT); }

}  // namespace

}  // namespace hh

using namespace hh;

extern "C" {

hh_status hh_factor_workspace_size(hh_factor_method method, int64_t n, int64_t h, size_t *bytes) {
    int mc;
    static_assert(sizeof(method) == sizeof(int), "C enums are int-sized");
    std::memcpy(&mc, &method, sizeof mc);
    if (!bytes) return set_error(HH_ERR_INVALID_ARG, "bytes must not be null");
    if (mc < HH_FACTOR_CONSTRAINED || mc > HH_FACTOR_QR)
        return set_error(HH_ERR_INVALID_ARG, "unknown factorisation method");
    if (n < 1 || h < 0) return set_error(HH_ERR_INVALID_ARG, "need n >= 1 and h >= 0");
    const int64_t nmax = mc == HH_FACTOR_QR ? 4096 : 1024;
    if (n > nmax)
        return set_error(HH_ERR_UNSUPPORTED, "this method supports n <= %lld (n = %lld)",
                         (long long)nmax, (long long)n);
    if (mc == HH_FACTOR_QR && h > n - 1)
        return set_error(HH_ERR_INVALID_ARG, "QR gives at most n - 1 reflectors (h = %lld, n = %lld)",
                         (long long)h, (long long)n);
    *bytes = factor_ws(n).total;
    return HH_OK;
}

hh_status hh_factor_orthonormal(hh_factor_method method, int64_t n, int64_t h, const double *U,
                                int64_t ldu, double *R, int64_t ldr, double *d, double *z,
                                void *ws, size_t ws_bytes, hipStream_t st) {
    size_t need = 0;
    hh_status s = hh_factor_workspace_size(method, n, h, &need);
    if (s != HH_OK) return s;
    int mc;
    std::memcpy(&mc, &method, sizeof mc);
    if (!U) return set_error(HH_ERR_INVALID_ARG, "U must not be null");
    if (ldu < n) return set_error(HH_ERR_INVALID_ARG, "ldu must be >= n");
    if (h > 0 && !R) return set_error(HH_ERR_INVALID_ARG, "R must not be null when h > 0");
    if (h > 0 && ldr < n) return set_error(HH_ERR_INVALID_ARG, "ldr must be >= n");
    if (!ws) return set_error(HH_ERR_INVALID_ARG, "ws must not be null");
    if (ws_bytes < need)
        return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
    const FactorWs w = factor_ws(n);
    char *b = static_cast<char *>(ws);
    double *A = reinterpret_cast<double *>(b + w.A);
    double *V = reinterpret_cast<double *>(b + w.V);
    double *rot = reinterpret_cast<double *>(b + w.rot);
    int *flag = reinterpret_cast<int *>(b + w.flag);
    int *perm = reinterpret_cast<int *>(b + w.perm);
    double *zs = reinterpret_cast<double *>(b + w.zs);
    const int ni = (int)n, hi = (int)h;
    hipError_t e;
    if (mc == HH_FACTOR_QR) {
        hipLaunchKernelGGL(k_copy_mat, dim3(mat_blocks(ni)), dim3(kFT), 0, st, U, ldu, ni, A);
        for (int k = 0; k < hi; ++k) {
            hipLaunchKernelGGL(k_qr_refl, dim3(1), dim3(kFT), 0, st, A, ni, k, R, ldr);
            hipLaunchKernelGGL(k_qr_apply, dim3(ni - k), dim3(kFT), 0, st, A, ni, k, R, ldr);
        }
        if (d) hipLaunchKernelGGL(k_diag_sign, dim3((ni + kFT - 1) / kFT), dim3(kFT), 0, st, A, ni, d, 0);
        e = hipGetLastError();
        return e == hipSuccess ? HH_OK : set_error(HH_ERR_HIP, "factor launch: %s", hipGetErrorString(e));
    }
    // symmetric eigendecomposition of Z = U + U^T
    const int m = ni + (ni & 1);
    hipLaunchKernelGGL(k_sym_sum, dim3(mat_blocks(ni)), dim3(kFT), 0, st, U, ldu, ni, A, V, flag);
    if (ni > 1) {
        for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
            for (int r = 0; r < m - 1; ++r) {
                hipLaunchKernelGGL(k_jac_cols, dim3(m / 2), dim3(kFT), 0, st, A, V, ni, m, r, rot, flag);
                hipLaunchKernelGGL(k_jac_rows, dim3(m / 2), dim3(kFT), 0, st, A, ni, m, r, rot, flag);
            }
            hipLaunchKernelGGL(k_jac_check, dim3(1), dim3(kFT), 0, st, A, ni, flag);
        }
    }
    hipLaunchKernelGGL(k_eig_sort, dim3(1), dim3(kFT), 0, st, A, ni, zs, perm, z);
    if (hi > 0) {
        if (mc == HH_FACTOR_CONSTRAINED)
            hipLaunchKernelGGL(k_constrained, dim3(hi), dim3(kFT), 0, st, V, ni, hi, zs, perm, R, ldr);
        else  // A is free again: it holds the construction-order list
            hipLaunchKernelGGL(k_unconstrained, dim3(1), dim3(kFT), (size_t)ni * 8, st, U, ldu, V, ni,
                               hi, zs, perm, A, R, ldr);
    }
    if (d) hipLaunchKernelGGL(k_diag_sign, dim3((ni + kFT - 1) / kFT), dim3(kFT), 0, st, A, ni, d, 1);
    e = hipGetLastError();
    return e == hipSuccess ? HH_OK : set_error(HH_ERR_HIP, "factor launch: %s", hipGetErrorString(e));
}

}  // extern "C"

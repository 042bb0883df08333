// Reflector setup for the fused kernels, in FP64 on the GPU.
//
// For each column u_k of U (paper Sec. II-A, eq. 2 requires unit reflector
// vectors; a zero vector is the identity factor, Sec. II-B after Result 1):
//   nrm_k = ||u_k||_2                  (FP64)
//   uh_k  = u_k / nrm_k                (FP64, kept for the gradient's chain rule)
//   ut_k  = uh_k rounded to the compute type, zero-padded to npad
//   tau_k = 2 / ||ut_k||^2             (FP64, then rounded; 0 for a zero column)
// With tau_k formed from the rounded vector, z - tau_k (ut_k^T z) ut_k is an
// exact reflection for the vector actually used, so rounding ut_k changes the
// reflector direction slightly but never its orthogonality.
//   lead_k = first i with ut_k[i] != 0 (npad for a zero column): reflectors
// built by Householder QR have k - 1 leading zeros (the remark after
// Result 3), which the fused kernels skip.
#include "hh_internal.h"

namespace hh {
namespace {

constexpr int kSetupThreads = 256;

__device__ int block_min_int(int v, int *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kSetupThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = min(red[t], red[t + s]);
        __syncthreads();
    }
    int r = red[0];
    __syncthreads();
    return r;
}

__device__ double block_sum_f64(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kSetupThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

template <typename P, typename T>
__global__ __launch_bounds__(kSetupThreads) void k_setup_fused(
    const P *__restrict__ U, int64_t ldu, const P *__restrict__ lam, int n, int h,
    int npad, T *__restrict__ ut, T *__restrict__ tau, T *__restrict__ lamp,
    double *__restrict__ uh64, double *__restrict__ nrm64, int *__restrict__ lead) {
    __shared__ double red[kSetupThreads];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    if (k == h) {  // the spectrum, padded with zeros
        if (lamp)
            for (int i = t; i < npad; i += kSetupThreads)
                lamp[i] = (i < n) ? (T)lam[i] : (T)0;
        return;
    }
    const P *u = U + (int64_t)k * ldu;
    double s = 0.0;
    for (int i = t; i < n; i += kSetupThreads) {
        double v = (double)u[i];
        s += v * v;
    }
    s = block_sum_f64(s, red);
    const double r = sqrt(s);
    double s2 = 0.0;
    int first = npad;
    for (int i = t; i < npad; i += kSetupThreads) {
        double v = (i < n && r > 0.0) ? (double)u[i] / r : 0.0;
        T vr = (T)v;
        ut[(int64_t)k * npad + i] = vr;
        if (uh64 && i < n) uh64[(int64_t)k * n + i] = v;
        s2 += (double)vr * (double)vr;
        if (vr != (T)0 && i < first) first = i;
    }
    s2 = block_sum_f64(s2, red);
    if (lead) {
        first = block_min_int(first, reinterpret_cast<int *>(red));
        if (t == 0) lead[k] = first;
    }
    if (t == 0) {
        tau[k] = (s2 > 0.0) ? (T)(2.0 / s2) : (T)0;
        if (nrm64) nrm64[k] = r;
    }
}

}  // namespace

hipError_t launch_setup_fused(hh_dtype t, const void *U, int64_t ldu, const void *lam,
                              int64_t n, int64_t h, int npad, void *ut, void *tau,
                              void *lamp, double *uh64, double *nrm64, int *lead,
                              hipStream_t st) {
    const int blocks = (int)h + 1;
    if (t == HH_F32) {
        hipLaunchKernelGGL((k_setup_fused<float, float>), dim3(blocks), dim3(kSetupThreads), 0,
                           st, (const float *)U, ldu, (const float *)lam, (int)n, (int)h,
                           npad, (float *)ut, (float *)tau, (float *)lamp, uh64, nrm64, lead);
    } else {
        hipLaunchKernelGGL((k_setup_fused<double, double>), dim3(blocks), dim3(kSetupThreads),
                           0, st, (const double *)U, ldu, (const double *)lam, (int)n,
                           (int)h, npad, (double *)ut, (double *)tau, (double *)lamp, uh64,
                           nrm64, lead);
    }
    return hipGetLastError();
}

}  // namespace hh

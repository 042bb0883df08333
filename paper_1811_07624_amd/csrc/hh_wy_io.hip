// FP32 data on the compact-WY path.  The WY kernels read and write vectors in
// their 16-bit compute type; FP32 data is rounded to that type (nearest even)
// into a workspace buffer before the 16-bit path runs and its 16-bit results
// are widened back to FP32 after it.  The arithmetic is that of the 16-bit
// path on the rounded data, bit for bit; the conversion costs one extra pass
// over each FP32 operand.
#include <algorithm>

#include "hh_wy_common.h"

#define HH_CHECK(expr)                \
    do {                              \
        const hh_status _s = (expr);  \
        if (_s != HH_OK) return _s;   \
    } while (0)

namespace hh {
namespace {

constexpr int kCvtThreads = 256;

// dst[j * n + i] = (16-bit) src[j * lds + i] for i < n, j < N; a thread
// converts 8 consecutive elements of one vector (n is a multiple of 8).
template <typename E>
__global__ __launch_bounds__(kCvtThreads) void k_to16(const float *__restrict__ src, int64_t lds,
                                                     int n, int64_t N, typename E::elem *__restrict__ dst) {
    using v8 = typename E::vec8;
    const int64_t per = n / 8;
    for (int64_t t = (int64_t)blockIdx.x * kCvtThreads + threadIdx.x; t < per * N;
         t += (int64_t)gridDim.x * kCvtThreads) {
        const int64_t j = t / per, i = (t % per) * 8;
        const float *s = src + j * lds + i;
        v8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (typename E::elem)s[e];
        *reinterpret_cast<v8 *>(dst + j * n + i) = v;
    }
}

// dst[j * ldd + i] = (FP32) src[j * n + i].
template <typename E>
__global__ __launch_bounds__(kCvtThreads) void k_from16(const typename E::elem *__restrict__ src, int n,
                                                       int64_t N, float *__restrict__ dst, int64_t ldd) {
    using v8 = typename E::vec8;
    const int64_t per = n / 8;
    for (int64_t t = (int64_t)blockIdx.x * kCvtThreads + threadIdx.x; t < per * N;
         t += (int64_t)gridDim.x * kCvtThreads) {
        const int64_t j = t / per, i = (t % per) * 8;
        const v8 v = *reinterpret_cast<const v8 *>(src + j * n + i);
        float *d = dst + j * ldd + i;
#pragma unroll
        for (int e = 0; e < 8; ++e) d[e] = (float)v[e];
    }
}

dim3 cvt_grid(int n, int64_t N) {
    const int64_t work = (int64_t)(n / 8) * N;
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((work + kCvtThreads - 1) / kCvtThreads,
                                                                 (int64_t)8 * device_cu_count())));
}

hipError_t to16(bool bf, const void *src, int64_t lds, int n, int64_t N, void *dst, hipStream_t st) {
    if (N == 0) return hipSuccess;
    if (bf)
        hipLaunchKernelGGL(k_to16<BF16>, cvt_grid(n, N), dim3(kCvtThreads), 0, st,
                           static_cast<const float *>(src), lds, n, N, static_cast<BF16::elem *>(dst));
    else
        hipLaunchKernelGGL(k_to16<F16>, cvt_grid(n, N), dim3(kCvtThreads), 0, st,
                           static_cast<const float *>(src), lds, n, N, static_cast<F16::elem *>(dst));
    return hipGetLastError();
}

hipError_t from16(bool bf, const void *src, int n, int64_t N, void *dst, int64_t ldd, hipStream_t st) {
    if (N == 0) return hipSuccess;
    if (bf)
        hipLaunchKernelGGL(k_from16<BF16>, cvt_grid(n, N), dim3(kCvtThreads), 0, st,
                           static_cast<const BF16::elem *>(src), n, N, static_cast<float *>(dst), ldd);
    else
        hipLaunchKernelGGL(k_from16<F16>, cvt_grid(n, N), dim3(kCvtThreads), 0, st,
                           static_cast<const F16::elem *>(src), n, N, static_cast<float *>(dst), ldd);
    return hipGetLastError();
}

// The descriptor of the 16-bit path for FP32 data.
hh_desc desc16(const hh_desc *d) {
    hh_desc e = *d;
    e.io_dtype = d->compute_dtype;
    return e;
}

bool io32(const hh_desc *d) { return d->io_dtype == HH_F32; }

// One n x N matrix in the compute type, leading dimension n.
size_t buf16(const hh_desc *d) { return align256((size_t)d->n * (size_t)d->N * 2); }

// Buffers of the FP32 path after the 16-bit path's workspace: the forward
// needs one (X, converted in place into Y), the backward three (X, dY, dX).
size_t io_buffers(hh_op op) { return op >= HH_OP_APPLY_BWD ? 3 : 1; }

hh_status check_io32(const hh_desc *d) {
    if (d->n % 8 != 0) return set_error(HH_ERR_UNSUPPORTED, "WY path needs n to be a multiple of 8");
    return HH_OK;
}

// The checks of the 16-bit path that would otherwise come after the
// conversion kernels are enqueued: nothing is enqueued by a failing call.
hh_status check_params(hh_op fop, const hh_desc *d, const void *U, const void *lam, const void *saved,
                       size_t saved_bytes) {
    if (d->h > 0 && !U) return set_error(HH_ERR_INVALID_ARG, "U must not be null");
    if (fop == HH_OP_SYM && !lam) return set_error(HH_ERR_INVALID_ARG, "lam must not be null");
    if (saved) {
        size_t sz = 0;
        HH_CHECK(wy_saved_size(fop, d, &sz));
        if (saved_bytes < sz)
            return set_error(HH_ERR_INVALID_ARG, "saved record needs %zu bytes, got %zu", sz, saved_bytes);
        if (((uintptr_t)saved & 15) != 0)
            return set_error(HH_ERR_INVALID_ARG, "saved record must be 16-byte aligned");
    }
    return HH_OK;
}

}  // namespace

hh_status wy_workspace_size(hh_op op, const hh_desc *d, size_t *bytes) {
    if (!io32(d)) return wy_workspace_size16(op, d, bytes);
    HH_CHECK(check_io32(d));
    const hh_desc e = desc16(d);
    size_t b = 0;
    HH_CHECK(wy_workspace_size16(op, &e, &b));
    *bytes = align256(b) + io_buffers(op) * buf16(d);
    return HH_OK;
}

hh_status wy_forward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                     const void *X, int64_t ldx, const void *Xb, int64_t ldb, void *Y,
                     int64_t ldy, void *saved, size_t saved_bytes, void *ws, size_t ws_bytes,
                     hipStream_t st) {
    if (!io32(d))
        return wy_forward16(op, d, U, ldu, lam, X, ldx, Xb, ldb, Y, ldy, saved, saved_bytes, ws, ws_bytes, st);
    HH_CHECK(check_io32(d));
    if (op == HH_OP_MAHAL)
        return set_error(HH_ERR_UNSUPPORTED, "WY path provides Q X, Q^T X and Q diag(lam) Q^T X");
    const hh_desc e = desc16(d);
    const int64_t n = d->n, N = d->N;
    size_t b = 0;
    HH_CHECK(wy_workspace_size16(op, &e, &b));
    const size_t need = align256(b) + buf16(d);
    if (N == 0 && !saved) return HH_OK;
    HH_CHECK(check_params(op, d, U, lam, saved, saved_bytes));
    if (N > 0 && (!X || !Y)) return set_error(HH_ERR_INVALID_ARG, "X and Y must not be null");
    if (N > 0 && Y == X && ldy != ldx) return set_error(HH_ERR_INVALID_ARG, "in-place call needs ldy == ldx");
    if (!ws) return set_error(HH_ERR_INVALID_ARG, "ws must not be null");
    if (ws_bytes < need) return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
    char *xh = static_cast<char *>(ws) + align256(b);
    const bool bf = d->compute_dtype == HH_BF16;
    hipError_t er = to16(bf, X, ldx, (int)n, N, xh, st);
    if (er != hipSuccess) return set_error(HH_ERR_HIP, "conversion to 16 bits: %s", hipGetErrorString(er));
    // the 16-bit path in place on the converted copy
    HH_CHECK(wy_forward16(op, &e, U, ldu, lam, xh, n, nullptr, 0, xh, n, saved, saved_bytes, ws, b, st));
    er = from16(bf, xh, (int)n, N, Y, ldy, st);
    if (er != hipSuccess) return set_error(HH_ERR_HIP, "conversion to FP32: %s", hipGetErrorString(er));
    return HH_OK;
}

hh_status wy_backward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                      const void *X, int64_t ldx, const void *Xb, int64_t ldb, const void *G,
                      int64_t ldg, void *dX, void *dXb, int64_t lddx, void *dU, int64_t lddu,
                      void *dlam, const void *saved, size_t saved_bytes, void *ws,
                      size_t ws_bytes, hipStream_t st) {
    if (!io32(d))
        return wy_backward16(op, d, U, ldu, lam, X, ldx, Xb, ldb, G, ldg, dX, dXb, lddx, dU, lddu, dlam,
                             saved, saved_bytes, ws, ws_bytes, st);
    HH_CHECK(check_io32(d));
    if (op == HH_OP_MAHAL_BWD)
        return set_error(HH_ERR_UNSUPPORTED, "WY path provides Q X, Q^T X and Q diag(lam) Q^T X");
    const hh_desc e = desc16(d);
    const int64_t n = d->n, N = d->N;
    size_t b = 0;
    HH_CHECK(wy_workspace_size16(op, &e, &b));
    const size_t need = align256(b) + 3 * buf16(d);
    const hh_op fop = op == HH_OP_APPLY_BWD ? HH_OP_APPLY : op == HH_OP_APPLY_T_BWD ? HH_OP_APPLY_T : HH_OP_SYM;
    HH_CHECK(check_params(fop, d, U, lam, saved, saved_bytes));
    if (N > 0 && (!X || !G)) return set_error(HH_ERR_INVALID_ARG, "X and dY must not be null");
    if (!ws) return set_error(HH_ERR_INVALID_ARG, "ws must not be null");
    if (ws_bytes < need) return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
    char *xh = static_cast<char *>(ws) + align256(b);
    char *gh = xh + buf16(d);
    char *dxh = gh + buf16(d);
    const bool bf = d->compute_dtype == HH_BF16;
    hipError_t er = to16(bf, X, ldx, (int)n, N, xh, st);
    if (er == hipSuccess) er = to16(bf, G, ldg, (int)n, N, gh, st);
    if (er != hipSuccess) return set_error(HH_ERR_HIP, "conversion to 16 bits: %s", hipGetErrorString(er));
    HH_CHECK(wy_backward16(op, &e, U, ldu, lam, xh, n, nullptr, 0, gh, n, dX ? dxh : nullptr, nullptr, n, dU,
                           lddu, dlam, saved, saved_bytes, ws, b, st));
    if (dX) {
        er = from16(bf, dxh, (int)n, N, dX, lddx, st);
        if (er != hipSuccess) return set_error(HH_ERR_HIP, "conversion to FP32: %s", hipGetErrorString(er));
    }
    return HH_OK;
}

}  // namespace hh

// Internal declarations shared by the HIP translation units of libhh.so.
// Not part of the public ABI (that is include/hh.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>
#include <utility>

#include "hh.h"

namespace hh {

constexpr int kWave = 64;

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// Calls f(integral_constant<int, i>) for i = 0 .. N-1 (compile-time indices).
template <int N, typename F> __device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// 16-byte vector types: the unit of every global and LDS access of the fused
// kernels (one dwordx4 per lane).
template <typename T> struct V16;
template <> struct V16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
};
template <> struct V16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
};

// Fused multiply-add in the operand type (never promotes float to double).
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Cross-lane sums built from DPP moves (no LDS round trip).
//   quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E,
//   row_ror:4 = 0x124, row_ror:8 = 0x128  -> every lane of a 16-lane row
//   holds the row sum;  row_bcast:15 = 0x142 (rows 1,3), row_bcast:31 = 0x143
//   (rows 2,3) -> lane 63 holds the wave sum.
template <int CTRL, int RM = 0xF, int BM = 0xF>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, RM, BM, false));
}
template <int CTRL, int RM = 0xF, int BM = 0xF>
__device__ __forceinline__ double dpp_mov(double v) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, RM, BM, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, RM, BM, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo);
}

template <typename T> __device__ __forceinline__ T row_sum16(T v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x124>(v);
    v += dpp_mov<0x128>(v);
    return v;
}

__device__ __forceinline__ float read_lane(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the LPV lanes that share one vector; every one of them gets it.
template <int LPV, typename T> __device__ __forceinline__ T group_sum(T v) {
    static_assert(LPV == 16 || LPV == 64, "16 or 64 lanes per vector");
    v = row_sum16(v);
    if constexpr (LPV == 64) {
        v += dpp_mov<0x142, 0xA>(v);
        v += dpp_mov<0x143, 0xC>(v);
        v = read_lane(v, 63);
    }
    return v;
}

// out[y][e] = sum over q < nq of part[(y nq + q) stride + e], e < ne, in FP64
// and in the order q = 0, 1, ...  Each thread sums 4 consecutive elements with
// 16-byte loads, 8 partials in flight (ne and stride multiples of 4, part
// 16-byte aligned).  Launched by launch_sum_parts.
template <typename T> struct Vec4Of;
template <> struct Vec4Of<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec4Of<double> { typedef double type __attribute__((ext_vector_type(4))); };
constexpr int kSumThreads = 256;
template <typename T>
__global__ __launch_bounds__(kSumThreads) void k_sum_parts(const T *__restrict__ part, int nq, size_t stride,
                                                          int ne, double *__restrict__ out) {
    using V = typename Vec4Of<T>::type;
    const int e = 4 * (blockIdx.x * kSumThreads + threadIdx.x);
    if (e >= ne) return;
    const T *p = part + (size_t)blockIdx.y * nq * stride + e;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 8
    for (int q = 0; q < nq; ++q) {
        const V v = *reinterpret_cast<const V *>(p + (size_t)q * stride);
        s0 += (double)v[0];
        s1 += (double)v[1];
        s2 += (double)v[2];
        s3 += (double)v[3];
    }
    typedef double d4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<d4 *>(out + (size_t)blockIdx.y * ne + e) = d4{s0, s1, s2, s3};
}

// ny independent sums of nq partials of ne elements each (ne % 4 == 0).
template <typename T>
inline hipError_t launch_sum_parts(const T *part, int nq, size_t stride, int ne, int ny, double *out,
                                   hipStream_t st) {
    if (ne % 4 || stride % 4) return hipErrorInvalidValue;
    const unsigned bx = (unsigned)((ne / 4 + kSumThreads - 1) / kSumThreads);
    hipLaunchKernelGGL((k_sum_parts<T>), dim3(bx, ny), dim3(kSumThreads), 0, st, part, nq, stride, ne, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kernel selection for the fused (sequential-reflector) kernels: LPV lanes
// (16 or 64) own one vector, each lane NC 16-byte chunks of it; npad = NC*LPV*W >= n.
// The forward kernel may hold VPL vectors per lane group (each reflector
// chunk read from LDS then serves VPL vectors) and run WPB waves per block.
struct FusedShape {
    int lpv;
    int nc;
    int npad;
    int vpl = 1;
    int wpb = 4;
};
bool fused_shape(hh_dtype t, int64_t n, FusedShape *s);

// Records a thread-local message for hh_last_error() and returns s.
hh_status set_error(hh_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Device facts, cached per device.
int device_cu_count();

// Workspace layout helpers.
__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// Launchers (host side, enqueue only).  Each returns hipSuccess or the launch
// error.  Pointers are device pointers; shapes have been validated.
struct FusedPlan {
    hh_dtype t;          // F32 or F64 (compute = io = param)
    int64_t n, h, N;
    FusedShape s;
    int hc;              // reflectors per LDS chunk
    size_t lds_bytes;
};

// Setup: uh (FP64), compute-type padded reflectors, tau, padded lam, and
// (nullable) lead[k] = index of the first nonzero entry of the compute-type
// reflector k (npad for a zero reflector).
hipError_t launch_setup_fused(hh_dtype t, const void *U, int64_t ldu, const void *lam,
                              int64_t n, int64_t h, int npad, void *ut, void *tau,
                              void *lamp, double *uh64, double *nrm64, int *lead,
                              hipStream_t st);

enum FusedOp { F_APPLY = 0, F_APPLY_T = 1, F_SYM = 2, F_MAHAL = 3 };

struct FusedFwdArgs {
    const void *X;
    int64_t ldx;
    const void *Xb;
    int64_t ldb;
    void *Y;  // output vectors, or distances for MAHAL
    int64_t ldy;
    const void *ut;
    const void *tau;
    const int *lead;   // first nonzero entry of each compute-type reflector
    const void *lam;
    const void *din;   // n diagonal entries applied to the input, or null
    const void *dout;  // n diagonal entries applied to the output, or null
    int n, h, npad, hc;
    int64_t N;
    int vec_ok;  // 16-byte accesses are legal for every data operand
    int skip_zeros;  // run the kernels that skip each reflector's leading zero chunks
    void *dots;      // MAHAL, nullable: the h dot products u_k^T s_{k-1} of each pair, rows of h padded to 16 bytes
};

hipError_t launch_fused_fwd(const FusedPlan &p, FusedOp op, const FusedFwdArgs &a,
                            hipStream_t st);
// ndiag: how many n-vectors of diagonal entries the kernel stages beside the
// spectrum (0, 1 or 2)
bool fused_plan(hh_dtype t, int64_t n, int64_t h, int64_t N, FusedPlan *p, int ndiag = 0);
// For the distance kernel with its record of dot products: fewer reflectors
// per LDS staging where the record's staging would not fit beside them.
void fused_plan_fit_record(FusedPlan *p);

}  // namespace hh

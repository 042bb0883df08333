// All-pairs distances and k nearest neighbours in the learned metric (paper
// Sec. IV-C: a new point is transformed, x <- L x with L = sqrt(Lambda) U,
// before k-NN runs on the transformed vectors; here L = diag(sqrt(lam)) Q^T,
// the transform hh_forward_signed computes).  On transformed queries a_i and
// database vectors b_j (FP32, n <= 224):
//   d_ij = ||a_i - b_j||^2 = ||a_i||^2 + ||b_j||^2 - 2 a_i^T b_j,
// the products a_i^T b_j on the matrix cores (v_mfma_f32_16x16x4_f32, full
// FP32), then for every query the k smallest d_ij and their database indices.
//
// A workgroup (4 waves) owns 64 queries, staged once in LDS, and streams the
// database through LDS in tiles of 64 vectors; each wave forms a 32 x 32 block
// of the 64 x 64 product tile (four 16 x 16 MFMA blocks, K = 4 per step).  The
// distance tile goes through LDS, where one thread per query keeps its k best
// in ascending order (a candidate enters only when strictly below the current
// k-th, so among equal distances the earlier database index stays).  The
// expanded form loses accuracy through cancellation when d_ij is small next
// to ||a||^2 + ||b||^2, so the k survivors' distances are recomputed from the
// differences and re-sorted before they are written.
#include <cmath>

#include "hh_internal.h"

namespace hh {
namespace {

constexpr int kQB = 64;       // queries per workgroup
constexpr int kDB = 64;       // database vectors per tile
constexpr int kKT = 256;      // threads
constexpr int kMaxK = 32;
constexpr int kMaxNk = 224;  // keeps the LDS tiles within 160 KB at k = 32

typedef float f32x4 __attribute__((ext_vector_type(4)));

// LDS: queries [kQB][np+1], database tile [kDB][np+1], distance tile
// [kQB][kDB+1], query norms, tile norms, the k best per query (dist, index).
__host__ __device__ inline size_t knn_lds(int np, int k) {
    return ((size_t)kQB * (np + 1) + (size_t)kDB * (np + 1) + (size_t)kQB * (kDB + 1) + kQB + kDB) * 4 +
           (size_t)kQB * k * 8;
}

__global__ __launch_bounds__(kKT) void k_knn(const float *__restrict__ Zq, int64_t ldq, int64_t Nq,
                                            const float *__restrict__ Zd, int64_t ldd, int64_t Nd,
                                            int n, int np, int k, float *__restrict__ dist,
                                            int64_t *__restrict__ idx) {
    extern __shared__ __align__(16) float sm[];
    const int sq = np + 1;
    float *sQ = sm;                              // [kQB][sq]
    float *sD = sQ + kQB * sq;                   // [kDB][sq]
    float *sT = sD + kDB * sq;                   // [kQB][kDB+1]
    float *sQn = sT + kQB * (kDB + 1);           // [kQB]
    float *sDn = sQn + kQB;                      // [kDB]
    float *sBd = sDn + kDB;                      // [kQB][k] best distances
    int *sBi = reinterpret_cast<int *>(sBd + kQB * k);  // [kQB][k] database indices

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * kQB;
    // queries into LDS (zero rows past Nq and columns past n)
    for (int e = tid; e < kQB * np; e += kKT) {
        const int r = e / np, c = e % np;
        sQ[r * sq + c] = (q0 + r < Nq && c < n) ? Zq[(q0 + r) * ldq + c] : 0.f;
    }
    __syncthreads();
    if (tid < kQB) {
        float s = 0.f;
        for (int c = 0; c < n; ++c) s = fmaf(sQ[tid * sq + c], sQ[tid * sq + c], s);
        sQn[tid] = s;
        for (int j = 0; j < k; ++j) {
            sBd[tid * k + j] = INFINITY;
            sBi[tid * k + j] = -1;
        }
    }
    float kth = INFINITY;  // current k-th best of query tid (tid < kQB)
    // wave w: rows 32 (w / 2) .. +31, columns 32 (w % 2) .. +31 of the tile
    const int rb = 32 * (wv >> 1), cbk = 32 * (wv & 1);
    const int r16 = lane & 15, kk = lane >> 4;
    const int64_t ntiles = (Nd + kDB - 1) / kDB;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t j0 = t * kDB;
        __syncthreads();  // previous tile's sD / sT readers are done
        for (int e = tid; e < kDB * np; e += kKT) {
            const int r = e / np, c = e % np;
            sD[r * sq + c] = (j0 + r < Nd && c < n) ? Zd[(j0 + r) * ldd + c] : 0.f;
        }
        __syncthreads();
        if (tid < kDB) {
            float s = 0.f;
            for (int c = 0; c < n; ++c) s = fmaf(sD[tid * sq + c], sD[tid * sq + c], s);
            sDn[tid] = s;
        }
        f32x4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int c0 = 0; c0 < np; c0 += 4) {
            float av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = sQ[(rb + 16 * a + r16) * sq + c0 + kk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = sD[(cbk + 16 * b + r16) * sq + c0 + kk];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();  // sDn ready
        // distance tile: acc[a][b][i] is the product of query rb + 16 a + 4 kk + i
        // and database vector cbk + 16 b + r16
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int qr = rb + 16 * a + 4 * kk + i, dc = cbk + 16 * b + r16;
                    const float d = sQn[qr] + sDn[dc] - 2.f * acc[a][b][i];
                    sT[qr * (kDB + 1) + dc] = j0 + dc < Nd ? fmaxf(d, 0.f) : INFINITY;
                }
        __syncthreads();
        if (tid < kQB) {
            float *bd = sBd + tid * k;
            int *bi = sBi + tid * k;
            for (int c = 0; c < kDB; ++c) {
                const float d = sT[tid * (kDB + 1) + c];
                if (d < kth) {  // insert, keeping ascending order
                    int p = k - 1;
                    while (p > 0 && bd[p - 1] > d) {
                        bd[p] = bd[p - 1];
                        bi[p] = bi[p - 1];
                        --p;
                    }
                    bd[p] = d;
                    bi[p] = (int)(j0 + c);
                    kth = bd[k - 1];
                }
            }
        }
    }
    __syncthreads();
    // exact distances of the survivors from the differences, re-sorted
    if (tid < kQB && q0 + tid < Nq) {
        float *bd = sBd + tid * k;
        int *bi = sBi + tid * k;
        for (int j = 0; j < k; ++j) {
            if (bi[j] < 0) continue;
            const float *b = Zd + (int64_t)bi[j] * ldd;
            float s = 0.f;
            for (int c = 0; c < n; ++c) {
                const float r = sQ[tid * sq + c] - b[c];
                s = fmaf(r, r, s);
            }
            bd[j] = s;
        }
        for (int j = 1; j < k; ++j) {  // insertion sort by (distance, index)
            const float d = bd[j];
            const int x = bi[j];
            int p = j;
            while (p > 0 && (bd[p - 1] > d || (bd[p - 1] == d && (unsigned)bi[p - 1] > (unsigned)x))) {
                bd[p] = bd[p - 1];
                bi[p] = bi[p - 1];
                --p;
            }
            bd[p] = d;
            bi[p] = x;
        }
        for (int j = 0; j < k; ++j) {
            dist[(q0 + tid) * k + j] = bd[j];
            idx[(q0 + tid) * k + j] = bi[j];
        }
    }
}

}  // namespace
}  // namespace hh

using namespace hh;

extern "C" {

hh_status hh_knn(int64_t n, int64_t Nq, int64_t Nd, int64_t k, const float *Zq, int64_t ldq,
                 const float *Zd, int64_t ldd, float *dist, int64_t *idx, hipStream_t st) {
    if (n < 1 || Nq < 0 || Nd < 0 || k < 1)
        return set_error(HH_ERR_INVALID_ARG, "need n >= 1, Nq >= 0, Nd >= 0, k >= 1");
    if (n > kMaxNk || k > kMaxK)
        return set_error(HH_ERR_UNSUPPORTED, "k-NN supports n <= %d and k <= %d", kMaxNk, kMaxK);
    if (Nd > ((int64_t)1 << 31) - 1) return set_error(HH_ERR_UNSUPPORTED, "Nd must be < 2^31");
    if (k > Nd) return set_error(HH_ERR_INVALID_ARG, "k = %lld exceeds Nd = %lld", (long long)k, (long long)Nd);
    if (ldq < n || ldd < n) return set_error(HH_ERR_INVALID_ARG, "leading dimensions must be >= n");
    if (Nq == 0) return HH_OK;
    if (!Zq || !Zd || !dist || !idx) return set_error(HH_ERR_INVALID_ARG, "pointers must not be null");
    const int np = (int)((n + 3) / 4 * 4);
    const size_t lds = knn_lds(np, (int)k);
    const int64_t blocks = (Nq + kQB - 1) / kQB;
    if (blocks > ((int64_t)1 << 31) - 1) return set_error(HH_ERR_UNSUPPORTED, "too many queries");
    hipLaunchKernelGGL(k_knn, dim3((unsigned)blocks), dim3(kKT), lds, st, Zq, ldq, Nq, Zd, ldd, Nd,
                       (int)n, np, (int)k, dist, idx);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HH_OK : set_error(HH_ERR_HIP, "k-NN launch: %s", hipGetErrorString(e));
}

}  // extern "C"

// All-pairs distances and k nearest neighbours in the learned metric (paper
// Sec. IV-C: a new point is transformed, x <- L x with L = sqrt(Lambda) U,
// before k-NN runs on the transformed vectors; here L = diag(sqrt(lam)) Q^T,
// the transform hh_forward_signed computes).  On transformed queries a_i and
// database vectors b_j (FP32, n <= 224):
//   d_ij = ||a_i - b_j||^2 = ||a_i||^2 + ||b_j||^2 - 2 a_i^T b_j,
// the products a_i^T b_j on the matrix cores (v_mfma_f32_16x16x4_f32, full
// FP32), then for every query the k smallest d_ij and their database indices.
//
// A first kernel forms every ||a_i||^2 and ||b_j||^2 (one thread per vector,
// FP32 FMAs in coordinate order).  A workgroup (4 waves) owns 64 queries,
// staged once in LDS, and streams one split of the database through LDS in
// tiles of 64 vectors (the splits give the chip several workgroups per
// compute unit);
// each wave forms a 32 x 32
// block of the 64 x 64 product tile (four 16 x 16 MFMA blocks, K = 4 per
// step).  Each lane screens its distances in registers against each query's
// current k-th distance; only the candidates below it go to LDS, flagged in a
// per-query survivor mask, and one thread per query inserts them in database
// order into its sorted k best (a candidate enters only when strictly below
// the k-th, so among equal distances the earlier index stays).  A second
// kernel merges the splits' lists per query by (distance, index).  The
// expanded form loses accuracy through cancellation when d_ij is small next to
// ||a||^2 + ||b||^2, so the k survivors' distances are recomputed from the
// differences and re-sorted before they are written.
#include <algorithm>
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

// Up to this padded length the queries' MFMA operands are held in registers
// after the start, and the distance tile reuses the queries' LDS space.
constexpr int kQRegNp = 48;

// LDS: queries [kQB][np+1], database tile [kDB][np+1], distance tile
// [kQB][kDB+1] (over the queries when np <= kQRegNp), query norms, tile
// norms, the k best per query (dist, index), the current k-th distance per
// query and the survivor masks.
__host__ __device__ inline size_t knn_lds(int np, int k) {
    const size_t q = (size_t)kQB * (np + 1), tt = (size_t)kQB * (kDB + 1);
    const size_t qt = np <= kQRegNp ? (q > tt ? q : tt) : q + tt;
    return (qt + (size_t)kDB * (np + 1) + kQB + kDB) * 4 + (size_t)kQB * k * 8 + (size_t)kQB * 4 +
           (size_t)kQB * 4 * 4;
}

// Squared norms of the N vectors of Z (FP32 FMAs in coordinate order).
__global__ __launch_bounds__(256) void k_knn_norms(const float *__restrict__ Z, int64_t ld, int64_t N, int n,
                                                  float *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const float *z = Z + j * ld;
    float s = 0.f;
    for (int c = 0; c < n; ++c) s = fmaf(z[c], z[c], s);
    out[j] = s;
}

// Split s of the database (tiles [t0, t1)) against 64 queries: the k best by
// the expanded form, into part_d / part_i (row (s * Nq + q) * k).  Thread t
// fetches row t / 4 of a database tile, columns t % 4 + 4 i (i < np / 4 <=
// PF), into registers; the next tile's fetch is issued as soon as the current
// tile is in LDS, so it is in flight during the products, the screening and
// the insertions.
template <int PF>
__global__ __launch_bounds__(kKT) void k_knn(const float *__restrict__ Zq, int64_t ldq, int64_t Nq,
                                            const float *__restrict__ Zd, int64_t ldd, int64_t Nd,
                                            const float *__restrict__ qnorm, const float *__restrict__ dnorm,
                                            int n, int np, int k, int64_t tiles_per_split,
                                            float *__restrict__ part_d, int *__restrict__ part_i) {
    extern __shared__ __align__(16) float sm[];
    const int sq = np + 1;
    constexpr bool kQReg = 4 * PF <= kQRegNp;  // queries' operands in registers
    const int qsz = kQB * sq, tsz = kQB * (kDB + 1);
    float *sQ = sm;                                               // [kQB][sq]
    float *sD = sQ + (kQReg ? (qsz > tsz ? qsz : tsz) : qsz + tsz);  // [kDB][sq]
    float *sT = kQReg ? sQ : sQ + qsz;                            // [kQB][kDB+1]
    float *sQn = sD + kDB * sq;                                   // [kQB]
    float *sDn = sQn + kQB;                      // [kDB]
    float *sBd = sDn + kDB;                      // [kQB][k] best distances
    int *sBi = reinterpret_cast<int *>(sBd + kQB * k);  // [kQB][k] database indices
    float *sKth = reinterpret_cast<float *>(sBi + kQB * k);  // [kQB]
    unsigned *sMask = reinterpret_cast<unsigned *>(sKth + kQB);  // [kQB][2] survivor bits by column

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * kQB;
    const int split = blockIdx.y;
    // queries into LDS (zero rows past Nq and columns past n)
    for (int e = tid; e < kQB * np; e += kKT) {
        const int r = e / np, c = e % np;
        sQ[r * sq + c] = (q0 + r < Nq && c < n) ? Zq[(q0 + r) * ldq + c] : 0.f;
    }
    __syncthreads();
    if (tid < kQB) {
        sQn[tid] = q0 + tid < Nq ? qnorm[q0 + tid] : 0.f;
        for (int j = 0; j < k; ++j) {
            sBd[tid * k + j] = INFINITY;
            sBi[tid * k + j] = -1;
        }
        sKth[tid] = INFINITY;
        sMask[tid * 2] = 0u;
        sMask[tid * 2 + 1] = 0u;
    }
    __syncthreads();
    // wave w: rows 32 (w / 2) .. +31, columns 32 (w % 2) .. +31 of the tile
    const int rb = 32 * (wv >> 1), cbk = 32 * (wv & 1);
    const int r16 = lane & 15, kk = lane >> 4;
    float qn[2][4];  // norms of this lane's 8 query rows
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) qn[a][i] = sQn[rb + 16 * a + 4 * kk + i];
    // for short vectors the queries' MFMA operands stay in registers (sQ is
    // then overwritten by the distance tile, after the first tile's barriers)
    float qa[2][kQReg ? PF : 1];
    if constexpr (kQReg) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int ic = 0; ic < PF; ++ic)
                qa[a][ic] = 4 * ic < np ? sQ[(rb + 16 * a + r16) * sq + 4 * ic + kk] : 0.f;
    }
    const int64_t ntiles = (Nd + kDB - 1) / kDB;
    const int64_t t0 = split * tiles_per_split;
    const int64_t t1 = t0 + tiles_per_split < ntiles ? t0 + tiles_per_split : ntiles;
    const int lr = tid >> 2, lc = tid & 3, npf = np >> 2;
    float pf[PF], pfn = 0.f;
    auto fetch = [&](int64_t j0) {
        const int64_t j = j0 + lr;
        const float *src = Zd + (j < Nd ? j : 0) * ldd;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int c = lc + 4 * i;
            pf[i] = (i < npf && j < Nd && c < n) ? src[c] : 0.f;
        }
        if (tid < kDB) pfn = j0 + tid < Nd ? dnorm[j0 + tid] : 0.f;
    };
    if (t0 < t1) fetch(t0 * kDB);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t j0 = t * kDB;
        __syncthreads();  // previous tile's sD / sT / sMask readers are done
#pragma unroll
        for (int i = 0; i < PF; ++i)
            if (i < npf) sD[lr * sq + lc + 4 * i] = pf[i];
        if (tid < kDB) sDn[tid] = pfn;
        if (t + 1 < t1) fetch(j0 + kDB);
        __syncthreads();
        f32x4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ic = 0; ic < PF; ++ic) {
            if (4 * ic < np) {
                const int c0 = 4 * ic;
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = kQReg ? qa[a][ic] : sQ[(rb + 16 * a + r16) * sq + c0 + kk];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = sD[(cbk + 16 * b + r16) * sq + c0 + kk];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
        }
        // acc[a][b][i] is the product of query rb + 16 a + 4 kk + i and database
        // vector cbk + 16 b + r16: each lane screens its 16 distances against
        // the queries' k-th distance (as it stood before this tile) and writes
        // only the candidates below it to the distance tile, flagging each in
        // its query's 64-bit survivor mask
        {
            float dnv[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) dnv[b] = sDn[cbk + 16 * b + r16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int qr = rb + 16 * a + 4 * kk + i;
                    const float kt = sKth[qr];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int dc = cbk + 16 * b + r16;
                        const float d = fmaxf(qn[a][i] + dnv[b] - 2.f * acc[a][b][i], 0.f);
                        if (j0 + dc < Nd && d < kt) {
                            sT[qr * (kDB + 1) + dc] = d;
                            atomicOr(&sMask[qr * 2 + (dc >> 5)], 1u << (dc & 31));
                        }
                    }
                }
        }
        __syncthreads();
        if (tid < kQB) {  // the owner inserts the survivors in database order
            float *bd = sBd + tid * k;
            int *bi = sBi + tid * k;
            float kth = sKth[tid];
            for (int part = 0; part < 2; ++part) {
                unsigned m = sMask[tid * 2 + part];
                sMask[tid * 2 + part] = 0u;
                while (m) {
                    const int c = 32 * part + __builtin_ctz(m);
                    m &= m - 1;
                    const float d = sT[tid * (kDB + 1) + c];
                    if (!(d < kth)) continue;
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
            sKth[tid] = kth;
        }
    }
    __syncthreads();
    if (tid < kQB && q0 + tid < Nq) {
        const int64_t row = ((int64_t)split * Nq + q0 + tid) * k;
        for (int j = 0; j < k; ++j) {
            part_d[row + j] = sBd[tid * k + j];
            part_i[row + j] = sBi[tid * k + j];
        }
    }
}

// 16 lanes per query: every lane merges the S split lists (each ascending,
// ties by index) by (distance, index) alike; the k survivors' distances are
// recomputed from the differences, each lane summing coordinates r, r + 16,
// ... in order and the 16 partial sums added by a fixed xor tree; then every
// lane re-sorts and each lane writes the entries j with j % 16 = r.
__global__ __launch_bounds__(256) void k_knn_merge(const float *__restrict__ Zq, int64_t ldq,
                                                  int64_t Nq, const float *__restrict__ Zd,
                                                  int64_t ldd, int n, int k, int S,
                                                  const float *__restrict__ part_d,
                                                  const int *__restrict__ part_i,
                                                  float *__restrict__ dist, int64_t *__restrict__ idx) {
    const int64_t q = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
    const int r = threadIdx.x & 15;
    if (q >= Nq) return;  // the whole 16-lane group
    float bd[kMaxK];
    int bi[kMaxK];
    int pos[16];
    for (int s = 0; s < S; ++s) pos[s] = 0;
    for (int j = 0; j < k; ++j) {
        int best = -1;
        float bdv = INFINITY;
        int biv = 0x7fffffff;
        for (int s = 0; s < S; ++s) {
            if (pos[s] >= k) continue;
            const int64_t row = ((int64_t)s * Nq + q) * k + pos[s];
            const int x = part_i[row];
            if (x < 0) continue;
            const float d = part_d[row];
            if (d < bdv || (d == bdv && x < biv)) {
                bdv = d;
                biv = x;
                best = s;
            }
        }
        bd[j] = bdv;
        bi[j] = best < 0 ? -1 : biv;
        if (best >= 0) ++pos[best];
    }
    const float *a = Zq + q * ldq;
    for (int j = 0; j < k; ++j) {
        if (bi[j] < 0) continue;
        const float *b = Zd + (int64_t)bi[j] * ldd;
        float s = 0.f;
        for (int c = r; c < n; c += 16) {
            const float df = a[c] - b[c];
            s = fmaf(df, df, s);
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
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
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        if (j < k && (j & 15) == r) {
            dist[q * k + j] = bd[j];
            idx[q * k + j] = bi[j];
        }
    }
}

// Database splits S: the workgroups (query blocks x S) run in rounds of
// `cap` (LDS-limited workgroups per compute unit, at most 4, times the units),
// each taking time in proportion to its tiles, so S minimises rounds x tiles
// per split (fewer splits on ties; at most 16, at least 4 tiles per split).
int knn_splits(int64_t Nq, int64_t Nd, int n, int k) {
    const int64_t qb = (Nq + kQB - 1) / kQB, ntiles = (Nd + kDB - 1) / kDB;
    const int np = (n + 3) / 4 * 4;
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(4, (160 * 1024) / (int64_t)knn_lds(np, k)));
    const int64_t cap = per_cu * device_cu_count();
    const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(16, ntiles / 4));
    int64_t best = 1, bestc = -1;
    for (int64_t sp = 1; sp <= smax; ++sp) {
        const int64_t c = (qb * sp + cap - 1) / cap * ((ntiles + sp - 1) / sp);
        if (bestc < 0 || c < bestc) {
            bestc = c;
            best = sp;
        }
    }
    return (int)best;
}

// per-split lists (distances, indices), then the query and database norms
size_t knn_ws_bytes(int64_t Nq, int64_t Nd, int64_t k, int S) {
    return align256((size_t)S * Nq * k * 4) * 2 + align256((size_t)Nq * 4) + align256((size_t)Nd * 4);
}

}  // namespace
}  // namespace hh

using namespace hh;

extern "C" {

static hh_status knn_check(int64_t n, int64_t Nq, int64_t Nd, int64_t k) {
    if (n < 1 || Nq < 0 || Nd < 0 || k < 1)
        return set_error(HH_ERR_INVALID_ARG, "need n >= 1, Nq >= 0, Nd >= 0, k >= 1");
    if (n > kMaxNk || k > kMaxK)
        return set_error(HH_ERR_UNSUPPORTED, "k-NN supports n <= %d and k <= %d", kMaxNk, kMaxK);
    if (Nd > ((int64_t)1 << 31) - 1 || Nq > ((int64_t)1 << 36))
        return set_error(HH_ERR_UNSUPPORTED, "Nd must be < 2^31");
    if (k > Nd) return set_error(HH_ERR_INVALID_ARG, "k = %lld exceeds Nd = %lld", (long long)k, (long long)Nd);
    return HH_OK;
}

hh_status hh_knn_workspace_size(int64_t n, int64_t Nq, int64_t Nd, int64_t k, size_t *bytes) {
    if (!bytes) return set_error(HH_ERR_INVALID_ARG, "bytes must not be null");
    const hh_status s = knn_check(n, Nq, Nd, k);
    if (s != HH_OK) return s;
    *bytes = Nq == 0 ? 0 : knn_ws_bytes(Nq, Nd, k, knn_splits(Nq, Nd, (int)n, (int)k));
    return HH_OK;
}

hh_status hh_knn(int64_t n, int64_t Nq, int64_t Nd, int64_t k, const float *Zq, int64_t ldq,
                 const float *Zd, int64_t ldd, float *dist, int64_t *idx, void *ws, size_t ws_bytes,
                 hipStream_t st) {
    const hh_status s = knn_check(n, Nq, Nd, k);
    if (s != HH_OK) return s;
    if (ldq < n || ldd < n) return set_error(HH_ERR_INVALID_ARG, "leading dimensions must be >= n");
    if (Nq == 0) return HH_OK;
    if (!Zq || !Zd || !dist || !idx || !ws) return set_error(HH_ERR_INVALID_ARG, "pointers must not be null");
    const int S = knn_splits(Nq, Nd, (int)n, (int)k);
    const size_t need = knn_ws_bytes(Nq, Nd, k, S);
    if (ws_bytes < need) return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
    const int np = (int)((n + 3) / 4 * 4);
    const size_t lds = knn_lds(np, (int)k);
    const int64_t qblocks = (Nq + kQB - 1) / kQB;
    if (qblocks > ((int64_t)1 << 31) - 1 || (Nq + 15) / 16 > ((int64_t)1 << 31) - 1)
        return set_error(HH_ERR_UNSUPPORTED, "too many queries");
    const int64_t ntiles = (Nd + kDB - 1) / kDB;
    const int64_t tps = (ntiles + S - 1) / S;
    char *w = static_cast<char *>(ws);
    const size_t lb = align256((size_t)S * Nq * k * 4);
    float *pd = reinterpret_cast<float *>(w);
    int *pi = reinterpret_cast<int *>(w + lb);
    float *qn = reinterpret_cast<float *>(w + 2 * lb);
    float *dn = reinterpret_cast<float *>(w + 2 * lb + align256((size_t)Nq * 4));
    hipLaunchKernelGGL(k_knn_norms, dim3((unsigned)((Nq + 255) / 256)), dim3(256), 0, st, Zq, ldq, Nq, (int)n, qn);
    if (Nd > 0)
        hipLaunchKernelGGL(k_knn_norms, dim3((unsigned)((Nd + 255) / 256)), dim3(256), 0, st, Zd, ldd, Nd, (int)n,
                           dn);
    {
        const dim3 grid((unsigned)qblocks, (unsigned)S);
        if (np <= kQRegNp)
            hipLaunchKernelGGL(k_knn<kQRegNp / 4>, grid, dim3(kKT), lds, st, Zq, ldq, Nq, Zd, ldd, Nd, qn, dn, (int)n, np,
                               (int)k, tps, pd, pi);
        else if (np <= 112)
            hipLaunchKernelGGL(k_knn<28>, grid, dim3(kKT), lds, st, Zq, ldq, Nq, Zd, ldd, Nd, qn, dn, (int)n, np,
                               (int)k, tps, pd, pi);
        else
            hipLaunchKernelGGL(k_knn<kMaxNk / 4>, grid, dim3(kKT), lds, st, Zq, ldq, Nq, Zd, ldd, Nd, qn, dn,
                               (int)n, np, (int)k, tps, pd, pi);
    }
    hipLaunchKernelGGL(k_knn_merge, dim3((unsigned)((Nq * 16 + 255) / 256)), dim3(256), 0, st, Zq, ldq, Nq, Zd,
                       ldd, (int)n, (int)k, S, pd, pi, dist, idx);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HH_OK : set_error(HH_ERR_HIP, "k-NN launch: %s", hipGetErrorString(e));
}

}  // extern "C"

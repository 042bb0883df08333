// Compact-WY path on the matrix cores (BF16 or FP16 inputs, FP32 accumulation).
//
// The product of reflectors H_k = I - tau_k y_k y_k^T (tau_k = 2/||y_k||^2)
// in the order of the paper's eq. 1 / eq. theU2, Q = H_1 ... H_h, equals
// I - Y T Y^T with Y = [y_1 .. y_h] and T upper triangular,
// T^{-1} = diag(||y_k||^2 / 2) + striu(Y^T Y)
// (compact WY form: Bischof & Van Loan 1987, Schreiber & Van Loan 1989; this
// T^{-1} identity is Puglisi 1992 / Joffrain et al. 2006).  Q^T = I - Y T^T Y^T.
// The paper itself applies reflectors one at a time (Sec. II-A); the blocked
// form performs the same 4nh operations per vector as two skinny products
// that map onto MFMA.
//
// Setup (FP64 on the GPU): y_k = u_k/||u_k|| rounded to the 16-bit type; the
// Gram matrix and T are formed from the ROUNDED y_k, so I - Y T Y^T is exactly
// the product of the reflectors of the vectors actually used (orthogonal up to
// the rounding of the products, not of the reflector vectors).  A zero column
// gives y_k = 0 and a diagonal entry 1/2 in T^{-1}, which leaves H_k = I.
// h is padded to HP (64 or 128) with such zero reflectors.
//
// Main kernel, one pass over X: a block of 8 waves owns NB = 16*CB vectors;
// wave w owns rows [w*32P, (w+1)*32P) of them and keeps that slice in
// registers between its single HBM read and single HBM write.
//   GEMM1  W_w = Y_w^T X_w   (per wave, MFMA 16x16x32, K = its rows)
//   sum over waves in LDS, W' = T W (or T^T W) in FP32, split W' = hi + lo
//   GEMM2  Y_w = X_w - Y_w (W'_hi + W'_lo)   (MFMA, K = HP)
// Register layout: lane l (c = l%16, g = l/16) holds, for row group p and
// column block cb, the 8 consecutive rows 32p + 8g .. 32p + 8g + 7 of column
// 16cb + c.  These 8 values are the B operand of GEMM1 (its K positions are
// rows 32p + 8g + j, matched by the A operand read from column-major Y), and
// GEMM2's M rows are permuted (row r of M-block m is 32p + 8(r/4) + 4m + r%4)
// so that its accumulators land on exactly the same 8 rows: one 16-byte load
// and one 16-byte store per (p, cb) and lane.
#include <algorithm>
#include <type_traits>

#include "hh_wy.h"

namespace hh {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 8;
constexpr int kThreadsWY = kWaves * kWave;

// 16-bit element types used on the matrix cores.
struct BF16 {
    typedef __bf16 elem;
    typedef bf16x8 vec8;
    static __device__ __forceinline__ f32x4 mfma(vec8 a, vec8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
struct F16 {
    typedef _Float16 elem;
    typedef f16x8 vec8;
    static __device__ __forceinline__ f32x4 mfma(vec8 a, vec8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

enum WyOp { W_APPLY = 0, W_APPLY_T = 1, W_SYM = 2 };

// ---------------------------------------------------------------------------
// Setup kernels (FP64).
template <typename E>
__global__ __launch_bounds__(256) void k_wy_norm(const float *__restrict__ U, int64_t ldu, int n,
                                                int h, int npad, int hp,
                                                typename E::elem *__restrict__ Yc,
                                                typename E::elem *__restrict__ Yr,
                                                double *__restrict__ nrm2,
                                                double *__restrict__ nrm_raw,
                                                double *__restrict__ uh64) {
    using el = typename E::elem;
    __shared__ double red[256];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    double s = 0.0;
    if (k < h)
        for (int i = t; i < n; i += 256) {
            const double v = (double)U[(int64_t)k * ldu + i];
            s += v * v;
        }
    red[t] = s;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if (t < q) red[t] += red[t + q];
        __syncthreads();
    }
    const double r = sqrt(red[0]);
    __syncthreads();
    double s2 = 0.0;
    for (int i = t; i < npad; i += 256) {
        double v = 0.0;
        if (k < h && i < n && r > 0.0) v = (double)U[(int64_t)k * ldu + i] / r;
        const el y = (el)v;
        Yc[(int64_t)k * npad + i] = y;
        Yr[(int64_t)i * hp + k] = y;
        if (uh64 && k < h && i < n) uh64[(int64_t)k * n + i] = v;
        const double yd = (double)y;
        s2 += yd * yd;
    }
    red[t] = s2;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if (t < q) red[t] += red[t + q];
        __syncthreads();
    }
    if (t == 0) {
        nrm2[k] = red[0];
        if (nrm_raw) nrm_raw[k] = (k < h) ? r : 0.0;
    }
}

// G[a][b] = y_a . y_b for a < b, FP64 (products of 16-bit values are exact).
template <typename E>
__global__ __launch_bounds__(256) void k_wy_gram(const typename E::elem *__restrict__ Yc,
                                                int npad, int hp, double *__restrict__ G) {
    __shared__ double red[256];
    const int a = blockIdx.y, b = blockIdx.x;
    if (b <= a) return;
    const int t = threadIdx.x;
    const typename E::elem *ya = Yc + (int64_t)a * npad;
    const typename E::elem *yb = Yc + (int64_t)b * npad;
    double s = 0.0;
    for (int i = t; i < npad; i += 256) s += (double)ya[i] * (double)yb[i];
    red[t] = s;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if (t < q) red[t] += red[t + q];
        __syncthreads();
    }
    if (t == 0) G[a * hp + b] = red[0];
}

// T = (diag(||y_k||^2/2) + striu(G))^{-1}, upper triangular, by column-wise
// back substitution in FP64 (thread j owns column j).  Tm = T as FP32,
// row-major; Tw = T in FP64 (kept for the backward pass).
__global__ __launch_bounds__(256) void k_wy_tmat(const double *__restrict__ G,
                                                const double *__restrict__ nrm2, int hp,
                                                double *__restrict__ Tw, float *__restrict__ Tm) {
    const int j = threadIdx.x;
    if (j >= hp) return;
    auto dg = [&](int i) { return nrm2[i] > 0.0 ? 0.5 * nrm2[i] : 0.5; };
    for (int i = j + 1; i < hp; ++i) Tw[i * hp + j] = 0.0;
    Tw[j * hp + j] = 1.0 / dg(j);
    for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s += G[i * hp + k] * Tw[k * hp + j];
        Tw[i * hp + j] = -s / dg(i);
    }
    for (int i = 0; i < hp; ++i) Tm[i * hp + j] = (float)Tw[i * hp + j];
}

// ---------------------------------------------------------------------------
// Main kernel.
struct WyArgs {
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    const void *Yc;   // HP x npad, column-major reflectors (GEMM1 A operand)
    const void *Yr;   // npad x HP, row-major reflectors (GEMM2 A operand)
    const float *Tm;  // HP x HP row-major
    const float *lam; // npad (SYM)
    int n, npad;
    int64_t N;
};

// Raw buffer accesses: the base address lives in a scalar descriptor, the
// lane part of the offset in one VGPR and the row-group part in an SGPR, so
// the unrolled loops need no per-access 64-bit addresses.  Reads past
// num_records return zero and writes past it are dropped.
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename V>
__device__ __forceinline__ V bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <typename V>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, V v, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, v), r, voff, soff, 0);
}

template <typename E, int P, int CB, int HP, int OP>
__global__ __launch_bounds__(kThreadsWY) void k_wy_fwd(WyArgs a) {
    using el = typename E::elem;
    using v8 = typename E::vec8;
    constexpr int NB = 16 * CB;   // vectors per tile
    constexpr int HB = HP / 16;   // 16-row blocks of h (GEMM1 M)
    constexpr int KS = HP / 32;   // K steps of GEMM2
    constexpr int SLICE = 32 * P; // rows per wave
    extern __shared__ __align__(16) unsigned char smem[];
    float *sP = reinterpret_cast<float *>(smem);                  // [kWaves][HP][NB]
    float *sT = sP + kWaves * HP * NB;                            // [HP][HP]
    el *sB = reinterpret_cast<el *>(sT + HP * HP);                // [2][CB][16][HP]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int c = lane & 15;
    const int g = lane >> 4;
    const int row0 = w * SLICE;
    const int n = a.n, npad = a.npad;
    const __amdgpu_buffer_rsrc_t rYc = make_rsrc(a.Yc, (uint32_t)HP * npad * 2);
    const __amdgpu_buffer_rsrc_t rYr = make_rsrc(a.Yr, (uint32_t)HP * npad * 2);
    const el *X = static_cast<const el *>(a.X);
    el *Yo = static_cast<el *>(a.Y);

    for (int i = tid; i < HP * HP; i += kThreadsWY) sT[i] = a.Tm[i];
    __syncthreads();

    // lane parts of the buffer offsets (bytes)
    const int vo_yc = ((c * npad) + row0 + 8 * g) * 2;             // + hb*16*npad*2
    const int rsub = 8 * (c >> 2) + (c & 3);                       // GEMM2 A-operand row
    const int vo_yr = ((row0 + rsub) * HP + 8 * g) * 2;            // + (4m*HP + 32ks)*2

    // One application of Q or Q^T to the register tile xr.  The correction
    // C = Y_slice W' of row group p (rows 32p + 8g + 4m + i, m = 0, 1) is
    // handed to consume(p, cc) as soon as it is formed.
    auto wy_pass = [&](v8(&xr)[P][CB], bool trans, auto &&consume) {
        // GEMM1: per-wave partial W = Y_slice^T X_slice.
        f32x4 acc[HB][CB];
#pragma unroll
        for (int hb = 0; hb < HB; ++hb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[hb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < P; ++p) {
            v8 av[HB];
#pragma unroll
            for (int hb = 0; hb < HB; ++hb)
                av[hb] = bload<v8>(rYc, vo_yc + hb * 16 * npad * 2, 64 * p);
#pragma unroll
            for (int hb = 0; hb < HB; ++hb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[hb][cb] = E::mfma(av[hb], xr[p][cb], acc[hb][cb]);
        }
        // partials to LDS: element (h, col) of wave w
#pragma unroll
        for (int hb = 0; hb < HB; ++hb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    sP[(w * HP + hb * 16 + 4 * g + i) * NB + cb * 16 + c] = acc[hb][cb][i];
        __syncthreads();
        // sum over waves (into wave 0's slot; each element has one owner)
        for (int e = tid; e < HP * NB; e += kThreadsWY) {
            float s = sP[e];
#pragma unroll
            for (int v = 1; v < kWaves; ++v) s += sP[v * HP * NB + e];
            sP[e] = s;
        }
        __syncthreads();
        // W' = T W  (or T^T W), split into 16-bit hi + lo, stored as the GEMM2
        // B operand: sB[hl][cb][c][h]
        {
            constexpr int TPR = NB / 4;                 // threads per row of W'
            constexpr int RPP = kThreadsWY / TPR;       // rows per pass
            const int c4 = (tid % TPR) * 4;
            for (int i = tid / TPR; i < HP; i += RPP) {
                f32x4 s = {0.f, 0.f, 0.f, 0.f};
                const int kb = trans ? 0 : i;
                const int ke = trans ? i + 1 : HP;
                for (int k = kb; k < ke; ++k) {
                    const float t = trans ? sT[k * HP + i] : sT[i * HP + k];
                    const f32x4 wv = *reinterpret_cast<const f32x4 *>(sP + k * NB + c4);
                    s += t * wv;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = c4 + q;
                    const el hi = (el)s[q];
                    const el lo = (el)(s[q] - (float)hi);
                    sB[((0 * CB + col / 16) * 16 + col % 16) * HP + i] = hi;
                    sB[((1 * CB + col / 16) * 16 + col % 16) * HP + i] = lo;
                }
            }
        }
        __syncthreads();
        v8 bfr[2][KS][CB];
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    bfr[hl][ks][cb] = *reinterpret_cast<const v8 *>(
                        sB + ((hl * CB + cb) * 16 + c) * HP + ks * 32 + 8 * g);
        // GEMM2: correction C = Y_slice W' for every (p, m, cb)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            v8 av[2][KS];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    av[m][ks] = bload<v8>(rYr, vo_yr + (4 * m * HP + 32 * ks) * 2, 64 * HP * p);
            f32x4 outc[2][CB];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    f32x4 cc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        cc = E::mfma(av[m][ks], bfr[0][ks][cb], cc);
                        cc = E::mfma(av[m][ks], bfr[1][ks][cb], cc);
                    }
                    outc[m][cb] = cc;
                }
            consume(p, outc);
        }
    };

    const int64_t ntiles = (a.N + NB - 1) / NB;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t col0 = tile * NB;
        const int64_t ncols = a.N - col0 < NB ? a.N - col0 : NB;
        const __amdgpu_buffer_rsrc_t rX =
            make_rsrc(X + col0 * a.ldx, (uint32_t)(((ncols - 1) * a.ldx + n) * 2));
        const __amdgpu_buffer_rsrc_t rY =
            make_rsrc(Yo + col0 * a.ldy, (uint32_t)(((ncols - 1) * a.ldy + n) * 2));
        int vo_x[CB], vo_y[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            vo_x[cb] = (int)(((16 * cb + c) * a.ldx + row0 + 8 * g) * 2);
            vo_y[cb] = (int)(((16 * cb + c) * a.ldy + row0 + 8 * g) * 2);
        }
        v8 xr[P][CB];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                v8 v = bload<v8>(rX, vo_x[cb], 64 * p);
                if (row0 + 32 * p + 8 * g >= n) v = v8{};
                xr[p][cb] = v;
            }
        // y = x - C, rounded to the 16-bit type and stored
        auto store_out = [&](int p, const f32x4(&cc)[2][CB]) {
            const bool rok = row0 + 32 * p + 8 * g < n;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                v8 y;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    y[j] = (el)((float)xr[p][cb][j] - cc[0][cb][j]);
                    y[j + 4] = (el)((float)xr[p][cb][j + 4] - cc[1][cb][j]);
                }
                if (rok) bstore<v8>(rY, y, vo_y[cb], 64 * p);
            }
        };
        if constexpr (OP == W_SYM) {
            // z = lam .* (x - C), rounded back into the register tile
            const __amdgpu_buffer_rsrc_t rL = make_rsrc(a.lam, (uint32_t)npad * 4);
            const int vo_l = (row0 + 8 * g) * 4;
            wy_pass(xr, true, [&](int p, const f32x4(&cc)[2][CB]) {
                const f32x4 l0 = bload<f32x4>(rL, vo_l, 128 * p);
                const f32x4 l1 = bload<f32x4>(rL, vo_l + 16, 128 * p);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    v8 z;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        z[j] = (el)(((float)xr[p][cb][j] - cc[0][cb][j]) * l0[j]);
                        z[j + 4] = (el)(((float)xr[p][cb][j + 4] - cc[1][cb][j]) * l1[j]);
                    }
                    xr[p][cb] = z;
                }
            });
            wy_pass(xr, false, store_out);
        } else {
            wy_pass(xr, OP == W_APPLY_T, store_out);
        }
    }
}

// ---------------------------------------------------------------------------
// Host side.
struct WyShape {
    int hp, p, cb, npad;
};

bool wy_shape(int64_t n, int64_t h, WyShape *s) {
    if (h > 128 || n > 8192) return false;
    s->hp = h <= 64 ? 64 : 128;
    s->p = n <= 1024 ? 4 : (n <= 4096 ? 16 : 32);
    s->cb = (s->p == 32 || s->hp == 128) ? 1 : 2;
    s->npad = 256 * s->p;
    return true;
}

size_t wy_lds_bytes(const WyShape &s) {
    const int nb = 16 * s.cb;
    return (size_t)kWaves * s.hp * nb * 4 + (size_t)s.hp * s.hp * 4 + 2 * (size_t)nb * s.hp * 2;
}

struct WyWs {
    size_t yc, yr, nrm2, nrmraw, gram, tw, tm, lam, uh64, total;
};

WyWs wy_ws(const WyShape &s, int64_t n, bool with_lam, bool bwd) {
    WyWs w{};
    size_t off = 0;
    const size_t hp = s.hp, np = s.npad;
    w.yc = off;     off += align256(hp * np * 2);
    w.yr = off;     off += align256(hp * np * 2);
    w.nrm2 = off;   off += align256(hp * 8);
    w.nrmraw = off; off += align256(hp * 8);
    w.gram = off;   off += align256(hp * hp * 8);
    w.tw = off;     off += align256(hp * hp * 8);
    w.tm = off;     off += align256(hp * hp * 4);
    w.lam = off;    off += with_lam ? align256(np * 4) : 0;
    w.uh64 = off;   off += bwd ? align256(hp * (size_t)n * 8) : 0;
    w.total = off;
    return w;
}

__global__ void k_fill_lam(const float *__restrict__ lam, int n, int npad, float *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < npad) out[i] = i < n ? lam[i] : 0.f;
}

__global__ void k_zero_f64(double *p, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < cnt) p[i] = 0.0;
}

template <typename E>
hipError_t wy_setup(const WyShape &s, const float *U, int64_t ldu, int64_t n, int64_t h, char *ws,
                    const WyWs &w, bool want_uh, hipStream_t st) {
    using el = typename E::elem;
    const int hp = s.hp;
    hipLaunchKernelGGL((k_wy_norm<E>), dim3(hp), dim3(256), 0, st, U, ldu, (int)n, (int)h, s.npad,
                       hp, reinterpret_cast<el *>(ws + w.yc), reinterpret_cast<el *>(ws + w.yr),
                       reinterpret_cast<double *>(ws + w.nrm2),
                       reinterpret_cast<double *>(ws + w.nrmraw),
                       want_uh ? reinterpret_cast<double *>(ws + w.uh64) : nullptr);
    hipLaunchKernelGGL(k_zero_f64, dim3((hp * hp + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<double *>(ws + w.gram), (int64_t)hp * hp);
    hipLaunchKernelGGL((k_wy_gram<E>), dim3(hp, hp), dim3(256), 0, st,
                       reinterpret_cast<const el *>(ws + w.yc), s.npad, hp,
                       reinterpret_cast<double *>(ws + w.gram));
    hipLaunchKernelGGL(k_wy_tmat, dim3(1), dim3(256), 0, st,
                       reinterpret_cast<const double *>(ws + w.gram),
                       reinterpret_cast<const double *>(ws + w.nrm2), hp,
                       reinterpret_cast<double *>(ws + w.tw), reinterpret_cast<float *>(ws + w.tm));
    return hipGetLastError();
}

template <typename E, int P, int CB, int HP>
hipError_t launch_main(WyOp op, const WyArgs &a, size_t lds, int grid, hipStream_t st) {
    switch (op) {
    case W_APPLY:
        hipLaunchKernelGGL((k_wy_fwd<E, P, CB, HP, W_APPLY>), dim3(grid), dim3(kThreadsWY), lds, st, a);
        break;
    case W_APPLY_T:
        hipLaunchKernelGGL((k_wy_fwd<E, P, CB, HP, W_APPLY_T>), dim3(grid), dim3(kThreadsWY), lds, st, a);
        break;
    case W_SYM:
        hipLaunchKernelGGL((k_wy_fwd<E, P, CB, HP, W_SYM>), dim3(grid), dim3(kThreadsWY), lds, st, a);
        break;
    }
    return hipGetLastError();
}

template <typename E>
hipError_t dispatch_main(const WyShape &s, WyOp op, const WyArgs &a, hipStream_t st) {
    const size_t lds = wy_lds_bytes(s);
    const int nb = 16 * s.cb;
    const int64_t tiles = (a.N + nb - 1) / nb;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, device_cu_count()));
    if (s.hp == 64) {
        if (s.p == 4) return launch_main<E, 4, 2, 64>(op, a, lds, grid, st);
        if (s.p == 16) return launch_main<E, 16, 2, 64>(op, a, lds, grid, st);
        return launch_main<E, 32, 1, 64>(op, a, lds, grid, st);
    }
    if (s.p == 4) return launch_main<E, 4, 1, 128>(op, a, lds, grid, st);
    if (s.p == 16) return launch_main<E, 16, 1, 128>(op, a, lds, grid, st);
    return launch_main<E, 32, 1, 128>(op, a, lds, grid, st);
}

}  // namespace

hh_status wy_workspace_size(hh_op op, const hh_desc *d, size_t *bytes) {
    WyShape s;
    if (!wy_shape(d->n, d->h, &s))
        return set_error(HH_ERR_UNSUPPORTED, "WY path supports n <= 8192 and h <= 128");
    if (op == HH_OP_MAHAL || op >= HH_OP_APPLY_BWD)
        return set_error(HH_ERR_UNSUPPORTED, "WY path provides Q X, Q^T X and Q diag(lam) Q^T X");
    *bytes = wy_ws(s, d->n, op == HH_OP_SYM, false).total;
    return HH_OK;
}

hh_status wy_forward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                     const void *X, int64_t ldx, const void *Xb, int64_t ldb, void *Y,
                     int64_t ldy, void *ws, size_t ws_bytes, hipStream_t st) {
    (void)Xb;
    (void)ldb;
    WyShape s;
    if (!wy_shape(d->n, d->h, &s))
        return set_error(HH_ERR_UNSUPPORTED, "WY path supports n <= 8192 and h <= 128");
    if (op == HH_OP_MAHAL)
        return set_error(HH_ERR_UNSUPPORTED, "WY path provides Q X, Q^T X and Q diag(lam) Q^T X");
    if (d->io_dtype != d->compute_dtype)
        return set_error(HH_ERR_UNSUPPORTED, "WY path reads and writes data in the compute type");
    const int64_t n = d->n, h = d->h, N = d->N;
    if (n % 8 != 0 || ldx % 8 != 0 || ldy % 8 != 0 || ((uintptr_t)X & 15) || ((uintptr_t)Y & 15))
        return set_error(HH_ERR_UNSUPPORTED,
                         "WY path needs n, ldx, ldy multiples of 8 and 16-byte aligned data");
    const WyWs w = wy_ws(s, n, op == HH_OP_SYM, false);
    if (N == 0) return HH_OK;
    if (h > 0 && !U) return set_error(HH_ERR_INVALID_ARG, "U must not be null");
    if (!X || !Y) return set_error(HH_ERR_INVALID_ARG, "X and Y must not be null");
    if (op == HH_OP_SYM && !lam) return set_error(HH_ERR_INVALID_ARG, "lam must not be null");
    if (Y == X && ldy != ldx) return set_error(HH_ERR_INVALID_ARG, "in-place call needs ldy == ldx");
    if (!ws) return set_error(HH_ERR_INVALID_ARG, "ws must not be null");
    if (ws_bytes < w.total)
        return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, ws_bytes);
    char *base = static_cast<char *>(ws);
    const bool bf = d->compute_dtype == HH_BF16;
    hipError_t e = bf ? wy_setup<BF16>(s, static_cast<const float *>(U), ldu, n, h, base, w, false, st)
                      : wy_setup<F16>(s, static_cast<const float *>(U), ldu, n, h, base, w, false, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY setup launch: %s", hipGetErrorString(e));
    if (op == HH_OP_SYM) {
        hipLaunchKernelGGL(k_fill_lam, dim3((s.npad + 255) / 256), dim3(256), 0, st,
                           static_cast<const float *>(lam), (int)n, s.npad,
                           reinterpret_cast<float *>(base + w.lam));
    }
    WyArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.Yc = base + w.yc;
    a.Yr = base + w.yr;
    a.Tm = reinterpret_cast<const float *>(base + w.tm);
    a.lam = reinterpret_cast<const float *>(base + w.lam);
    a.n = (int)n;
    a.npad = s.npad;
    a.N = N;
    const WyOp wop = op == HH_OP_APPLY ? W_APPLY : op == HH_OP_APPLY_T ? W_APPLY_T : W_SYM;
    e = bf ? dispatch_main<BF16>(s, wop, a, st) : dispatch_main<F16>(s, wop, a, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY kernel launch: %s", hipGetErrorString(e));
    return HH_OK;
}

hh_status wy_backward(hh_op, const hh_desc *, const void *, int64_t, const void *, const void *,
                      int64_t, const void *, int64_t, const void *, int64_t, void *, void *,
                      int64_t, void *, int64_t, void *, void *, size_t, hipStream_t) {
    return set_error(HH_ERR_UNSUPPORTED, "WY backward not built yet");
}

}  // namespace hh

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

#include "hh_wy_common.h"

namespace hh {
namespace {

constexpr int kWaves = 8;
constexpr int kThreadsWY = kWaves * kWave;
#ifndef WY_DEPTH
#define WY_DEPTH 3  // row groups of reflector operands fetched ahead of use
#endif


// ---------------------------------------------------------------------------
// Setup kernels (FP64).
// One block of kNormThreads per reflector k: u_k / ||u_k|| in FP64, rounded to
// the 16-bit type and written to the three fragment-ordered copies, with
// ||y_k||^2 of the rounded vector.  Sums: wave shuffles, then the wave
// partials in a fixed order.
constexpr int kNormThreads = 256;

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double block_sum_f64(double v, double *red) {
    constexpr int NW = kNormThreads / kWave;
    v = wave_sum_f64(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    __syncthreads();
    return s;
}

template <typename E>
__global__ __launch_bounds__(kNormThreads) void k_wy_norm(const float *__restrict__ U, int64_t ldu, int n,
                                                         int h, int npad, int hp,
                                                         typename E::elem *__restrict__ Yc,
                                                         typename E::elem *__restrict__ Yr,
                                                         typename E::elem *__restrict__ Ycs,
                                                         double *__restrict__ nrm2,
                                                         double *__restrict__ nrm_raw,
                                                         double *__restrict__ uh64) {
    using el = typename E::elem;
    __shared__ double red[kNormThreads / kWave];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    double s = 0.0;
    if (k < h)
        for (int i = t; i < n; i += kNormThreads) {
            const double v = (double)U[(int64_t)k * ldu + i];
            s += v * v;
        }
    const double r = sqrt(block_sum_f64(s, red));
    double s2 = 0.0;
    for (int i = t; i < npad; i += kNormThreads) {
        double v = 0.0;
        if (k < h && i < n && r > 0.0) v = (double)U[(int64_t)k * ldu + i] / r;
        const el y = (el)v;
        Yc[yc_index(k, i, npad)] = y;
        Yr[yr_index(k, i, hp)] = y;
        Ycs[ycs_index(k, i, hp)] = y;
        if (uh64 && k < h && i < n) uh64[(int64_t)k * n + i] = v;
        const double yd = (double)y;
        s2 += yd * yd;
    }
    s2 = block_sum_f64(s2, red);
    if (t == 0) {
        nrm2[k] = s2;
        if (nrm_raw) nrm_raw[k] = (k < h) ? r : 0.0;
    }
}

// Partial Gram matrices of the rounded reflectors in FP64 (a product of two
// 16-bit values is exact): Gp[s][a][b] = sum over the rows of segment s of
// y_a y_b, for the 16 x 16 tiles (ta, tb), ta <= tb, one block per (tile
// pair, segment).  Each step stages the fragments (ta, q) and (tb, q) of the
// fragment-ordered copy (32 rows each) in LDS.  With lam, the same pass also
// forms Mp[s][a][b] = sum of y_a lam_r y_b (exact in FP64 too: 11 + 11 + 24
// significant bits), the matrix Y^T diag(lam) Y of the symmetric form.
template <typename E>
__global__ __launch_bounds__(256) void k_wy_gram(const typename E::elem *__restrict__ Yc, int npad,
                                                int hp, const float *__restrict__ lam,
                                                double *__restrict__ Gp, double *__restrict__ Mp) {
    using v8 = typename E::vec8;
    __shared__ double ya[32][17], yb[32][17], lr[32];
    const int nhb = hp >> 4;
    int pr = blockIdx.x, ta = 0;
    while (pr >= nhb - ta) {
        pr -= nhb - ta;
        ++ta;
    }
    const int tb = ta + pr;
    const int nq = npad >> 5, qs = nq / kGramSeg, seg = blockIdx.y;
    const int t = threadIdx.x, i = t >> 4, j = t & 15;
    double acc = 0.0, accm = 0.0;
    for (int q = seg * qs; q < (seg + 1) * qs; ++q) {
        __syncthreads();
        if (t < 128) {
            const int which = t >> 6, ln = t & 63;
            const int hb = which ? tb : ta;
            const v8 v = *reinterpret_cast<const v8 *>(Yc + ((size_t)(hb * nq + q) * 64 + ln) * 8);
            double(*dst)[17] = which ? yb : ya;
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[8 * (ln >> 4) + e][ln & 15] = (double)v[e];
        } else if (lam && t < 160) {
            lr[t - 128] = (double)lam[32 * q + t - 128];
        }
        __syncthreads();
        if (lam) {
#pragma unroll 8
            for (int r = 0; r < 32; ++r) {
                const double p = ya[r][i] * yb[r][j];
                acc += p;
                accm += p * lr[r];
            }
        } else {
#pragma unroll 8
            for (int r = 0; r < 32; ++r) acc += ya[r][i] * yb[r][j];
        }
    }
    const size_t o = ((size_t)seg * hp + 16 * ta + i) * hp + 16 * tb + j;
    Gp[o] = acc;
    if (lam) Mp[o] = accm;
}

// T = (diag(||y_k||^2/2) + striu(G))^{-1}, upper triangular, FP64, by blocked
// inversion in LDS: the 16 x 16 diagonal blocks are inverted by back
// substitution (one column per thread), then neighbouring inverted blocks of
// [A B; 0 C] are merged, the off-diagonal block becoming -A^{-1} (B C^{-1}),
// doubling the block size at each level (each thread forms a 2 x 2 piece;
// every element is accumulated in the same order whatever the thread count).
// Outputs: Tw = T in FP64 (zero below the diagonal); Tf = T (tr = 0) and T^T (tr = 1) as 16-bit MFMA A-operand
// fragments split into hi + lo parts (hi = T rounded, lo = the rest rounded)
// for the streaming kernel's T product: fragment (tr, hl, ib, kb), lane (c, g),
// element j holds T'[sigma_row(ib, c)][32 kb + 8 g + j].
constexpr int kTmatThreads = 1024;

template <int HP, typename E>
__global__ __launch_bounds__(kTmatThreads) void k_wy_tmat(const double *__restrict__ G,
                                                         const double *__restrict__ nrm2,
                                                         double *__restrict__ Tw,
                                                         typename E::elem *__restrict__ Tf) {
    using el = typename E::elem;
    constexpr int LD = HP + 1, NT = kTmatThreads;
    extern __shared__ double M[];
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < (HP * HP + NT - 1) / NT; ++r) {
        const int idx = t + r * NT;
        if (idx < HP * HP) {
            const int i = idx / HP, k = idx % HP;
            const double g = G[idx];
            const double d = nrm2[i];
            M[i * LD + k] = k > i ? g : k < i ? 0.0 : (d > 0.0 ? 0.5 * d : 0.5);
        }
    }
    __syncthreads();
    {
        const bool act = t < HP;  // HP / 16 blocks x 16 columns
        const int o = 16 * (t >> 4), jc = t & 15;
        double x[16];
        if (act) {
#pragma unroll
            for (int i = 15; i >= 0; --i) {
                double s = (i == jc) ? 1.0 : 0.0;
#pragma unroll
                for (int k = i + 1; k < 16; ++k) s -= M[(o + i) * LD + o + k] * x[k];
                x[i] = (i > jc) ? 0.0 : s / M[(o + i) * LD + o + i];
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < 16; ++i) M[(o + i) * LD + o + jc] = x[i];
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 16; s < HP; s *= 2) {
        const int th = s / 2;  // 2 x 2 pieces per row of an s x s block
        const bool act = t < (HP / (2 * s)) * th * th;
        const int pidx = t / (th * th), rr = t % (th * th);
        const int i0 = 2 * s * pidx, a0 = i0 + 2 * (rr / th), b0 = i0 + s + 2 * (rr % th);
        double acc[2][2];
        for (int step = 0; step < 2; ++step) {
            if (act) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 2; ++r) acc[q][r] = 0.0;
                // step 0: B C^{-1} (C^{-1} at rows/cols i0+s..); step 1: A^{-1} X (X in B's place)
                const int ka = step == 0 ? i0 + s : i0;
#pragma unroll 8
                for (int c = 0; c < s; ++c) {
                    double av[2], bv[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        av[q] = M[(a0 + q) * LD + ka + c];
                        bv[q] = M[(ka + c) * LD + b0 + q];
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int r = 0; r < 2; ++r) acc[q][r] += av[q] * bv[r];
                }
            }
            __syncthreads();
            if (act) {
                const double sg = step == 0 ? 1.0 : -1.0;
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 2; ++r) M[(a0 + q) * LD + b0 + r] = sg * acc[q][r];
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int r = 0; r < (HP * HP + NT - 1) / NT; ++r) {
        const int idx = t + r * NT;
        if (idx < HP * HP) {
            const int i = idx / HP, k = idx % HP;
            const double v = (k >= i) ? M[i * LD + k] : 0.0;
            Tw[idx] = v;
        }
    }
    // fragments (the lower triangle of M is zero)
    constexpr int HB = HP / 16, KS = HP / 32, NF = 4 * HB * KS * 64;
    for (int id = t; id < NF; id += NT) {
        const int lane = id & 63, f = id >> 6;
        const int kb = f % KS, ib = (f / KS) % HB, hl = (f / (KS * HB)) & 1, tr = f / (2 * KS * HB);
        const int c = lane & 15, g = lane >> 4;
        const int row = sigma_row(ib, c);
        typename E::vec8 fr;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int col = 32 * kb + 8 * g + j;
            const double v = tr ? M[col * LD + row] : M[row * LD + col];
            // through FP32: hi may differ from T's direct 16-bit rounding in a
            // tie, and lo = T - hi (formed in FP64) absorbs that
            const el hi = (el)(float)v;
            fr[j] = hl ? (el)(float)(v - (double)hi) : hi;
        }
        *reinterpret_cast<typename E::vec8 *>(Tf + (size_t)id * 8) = fr;
    }
}

// Y^T diag(lam) Y (symmetric; the Gram pass fills only the tiles ta <= tb)
// as 16-bit MFMA A-operand fragments split into hi + lo parts, laid out as
// the tr = 0 half of k_wy_tfrag's output: fragment (hl, ib, kb), lane (c, g),
// element j holds M[sigma_row(ib, c)][32 kb + 8 g + j].
template <typename E>
__global__ __launch_bounds__(256) void k_wy_mfrag(const double *__restrict__ Ms, int hp,
                                                 typename E::elem *__restrict__ Mf) {
    using el = typename E::elem;
    const int HB = hp >> 4, KS = hp >> 5;
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= 2 * HB * KS * 64) return;
    const int lane = id & 63, f = id >> 6;
    const int kb = f % KS, ib = (f / KS) % HB, hl = f / (KS * HB);
    const int c = lane & 15, g = lane >> 4;
    const int r = sigma_row(ib, c);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int col = 32 * kb + 8 * g + j;
        const double m = (r >> 4) <= (col >> 4) ? Ms[r * hp + col] : Ms[col * hp + r];
        const el hi = (el)m;
        Mf[(size_t)id * 8 + j] = hl ? (el)(m - (double)hi) : hi;
    }
}

// ---------------------------------------------------------------------------
// Main kernel.

template <typename E, int P, int CB, int HP, int OP, int MINB>
__global__ __launch_bounds__(kThreadsWY, 2 * MINB) void k_wy_fwd(WyArgs a) {
    using el = typename E::elem;
    using v8 = typename E::vec8;
    constexpr int NB = 16 * CB;   // vectors per tile
    constexpr int HB = HP / 16;   // 16-row blocks of h (GEMM1 M)
    constexpr int KS = HP / 32;   // K steps of GEMM2
    constexpr int SLICE = 32 * P; // rows per wave
    extern __shared__ __align__(16) unsigned char smem[];
    // LDS row strides are padded so that the lanes of one access fall in
    // different banks.
    constexpr int NBP = NB + 4;   // partial sums row stride
    constexpr int HBP = HP + 8;   // W' fragment row stride (keeps 16-byte alignment)
    float *sP = reinterpret_cast<float *>(smem);                  // [kWaves][HP][NBP]
    el *sB = reinterpret_cast<el *>(sP + kWaves * HP * NBP);      // [2][CB][16][HBP]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int c = lane & 15;
    const int g = lane >> 4;
    const int row0 = w * SLICE;
    const int n = a.n, npad = a.npad;
    const __amdgpu_buffer_rsrc_t rYc = make_rsrc(a.Yc, (uint32_t)HP * npad * 2);
    const __amdgpu_buffer_rsrc_t rYr = make_rsrc(a.Yr, (uint32_t)HP * npad * 2);
    const __amdgpu_buffer_rsrc_t rTf = make_rsrc(a.Tf, (uint32_t)(8 * HP * HP));
    const el *X = static_cast<const el *>(a.X);
    el *Yo = static_cast<el *>(a.Y);


    // lane parts of the buffer offsets (bytes) into the fragment-ordered
    // reflector copies; the (hb, p, m, ks) parts are uniform
    const int nq = npad >> 5;
    const int vo_yc = ((row0 >> 5) * 64 + lane) * 16;              // + (hb*nq + p) KB
    const int vo_yr = ((row0 >> 5) * 2 * KS * 64 + lane) * 16;     // + ((2p + m) KS + ks) KB

    // One application of Q or Q^T to the register tile xr.  The correction
    // C = Y_slice W' of row group p (rows 32p + 8g + 4m + i, m = 0, 1) is
    // handed to consume(p, cc) as soon as it is formed.
    auto wy_pass = [&](v8(&xr)[P][CB], bool trans, int pass, int64_t col0, bool gemm2,
                       auto &&consume) {
        // GEMM1: per-wave partial W = Y_slice^T X_slice.
        f32x4 acc[HB][CB];
#pragma unroll
        for (int hb = 0; hb < HB; ++hb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[hb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        // A operands are fetched two row groups ahead of their use
        constexpr int DW1 = HB >= 8 ? 1 : WY_DEPTH;  // fewer stages for wide operands
        constexpr int D1 = P < DW1 ? P : DW1;
        v8 abuf[D1][HB];
#pragma unroll
        for (int q = 0; q < D1; ++q)
#pragma unroll
            for (int hb = 0; hb < HB; ++hb)
                abuf[q][hb] = bload<v8>(rYc, vo_yc, (hb * nq + q) * 1024);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            v8 av[HB];
#pragma unroll
            for (int hb = 0; hb < HB; ++hb) av[hb] = abuf[p % D1][hb];
            if (p + D1 < P) {
#pragma unroll
                for (int hb = 0; hb < HB; ++hb)
                    abuf[p % D1][hb] = bload<v8>(rYc, vo_yc, (hb * nq + p + D1) * 1024);
            }
#pragma unroll
            for (int hb = 0; hb < HB; ++hb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[hb][cb] = E::mfma(av[hb], xr[p][cb], acc[hb][cb]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // The T product runs on the matrix cores: wave w < HB * CB forms the
        // 16-row block ib of W' for the 16 vectors of column block cb, from T
        // (or T^T) as 16-bit hi + lo fragments (rows permuted by sigma_row)
        // and W as hi + lo parts (three products, lo * lo dropped).  Its T
        // fragments are fetched now (from L2; no HBM access is outstanding) so
        // that they arrive while the partial sums are formed.
        constexpr int NPAIR = HB * CB;
        const bool tw = w < NPAIR;
        const int ibw = w % HB, cbw = w / HB;
        const int trn = trans ? 1 : 0;
        v8 th[KS], tl[KS];
        if (tw) {
#pragma unroll
            for (int kb = 0; kb < KS; ++kb) {
                th[kb] = bload<v8>(rTf, lane * 16, (((trn * 2 + 0) * HB + ibw) * KS + kb) * 1024);
                tl[kb] = bload<v8>(rTf, lane * 16, (((trn * 2 + 1) * HB + ibw) * KS + kb) * 1024);
            }
        }
        // partials to LDS: element (h, col) of wave w
#pragma unroll
        for (int hb = 0; hb < HB; ++hb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    sP[(w * HP + hb * 16 + 4 * g + i) * NBP + cb * 16 + c] = acc[hb][cb][i];
        __syncthreads();
        // sum over waves (into wave 0's slot; each element has one owner)
        for (int e = tid; e < HP * NB; e += kThreadsWY) {
            const int ep = (e / NB) * NBP + e % NB;
            float s = sP[ep];
#pragma unroll
            for (int v = 1; v < kWaves; ++v) s += sP[v * HP * NBP + ep];
            sP[ep] = s;
        }
        __syncthreads();
        // W' = T W  (or T^T W), split into 16-bit hi + lo, stored as the GEMM2
        // B operand: sB[hl][cb][c][h]
        if (tw) {
            f32x4 zz = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KS; ++kb) {
                v8 wh, wl;  // B operand: W[32 kb + 8 g + j][16 cb + c]
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float v = sP[(32 * kb + 8 * g + j) * NBP + 16 * cbw + c];
                    const el hi = (el)v;
                    wh[j] = hi;
                    wl[j] = (el)(v - (float)hi);
                }
                zz = E::mfma(th[kb], wh, zz);
                zz = E::mfma(th[kb], wl, zz);
                zz = E::mfma(tl[kb], wh, zz);
            }
            // zz[i] is W'[sigma_row(ib, 4 g + i)][16 cb + c]: four consecutive rows
            typedef el el4 __attribute__((ext_vector_type(4)));
            const int r0 = sigma_row(ibw, 4 * g);
            el4 h4, l4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const el hi = (el)zz[i];
                h4[i] = hi;
                l4[i] = (el)(zz[i] - (float)hi);
            }
            *reinterpret_cast<el4 *>(sB + ((0 * CB + cbw) * 16 + c) * HBP + r0) = h4;
            *reinterpret_cast<el4 *>(sB + ((1 * CB + cbw) * 16 + c) * HBP + r0) = l4;
            if (a.coef) {  // coefficients for the backward pass, 16-bit
                const int64_t col = col0 + 16 * cbw + c;
                if (col < a.N) {
                    el *cp = static_cast<el *>(a.coef) + (int64_t)(pass * HP + r0) * a.ldc + col;
#pragma unroll
                    for (int i = 0; i < 4; ++i) cp[(int64_t)i * a.ldc] = (el)zz[i];
                }
            }
        }
        __syncthreads();
        if (!gemm2) return;
        // W' fragments (GEMM2 B operand) are re-read from LDS at each use
        auto bfrag = [&](int hl, int ks, int cb) {
            return *reinterpret_cast<const v8 *>(sB + ((hl * CB + cb) * 16 + c) * HBP + ks * 32 + 8 * g);
        };
        // GEMM2: correction C = Y_slice W' for every (p, m, cb)
        constexpr int DW2 = KS >= 4 ? 1 : WY_DEPTH;
        constexpr int D2 = P < DW2 ? P : DW2;
        v8 bbuf[D2][2][KS];
#pragma unroll
        for (int q = 0; q < D2; ++q)
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    bbuf[q][m][ks] = bload<v8>(rYr, vo_yr, ((2 * q + m) * KS + ks) * 1024);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            v8 av[2][KS];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) av[m][ks] = bbuf[p % D2][m][ks];
            if (p + D2 < P) {
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks)
                        bbuf[p % D2][m][ks] =
                            bload<v8>(rYr, vo_yr, ((2 * (p + D2) + m) * KS + ks) * 1024);
            }
            f32x4 outc[2][CB];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    f32x4 cc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        cc = E::mfma(av[m][ks], bfrag(0, ks, cb), cc);
                        cc = E::mfma(av[m][ks], bfrag(1, ks, cb), cc);
                    }
                    outc[m][cb] = cc;
                }
            consume(p, outc);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    const int64_t ntiles = (a.N + NB - 1) / NB;
    auto tile_rsrc = [&](int64_t tile, const el *base, int64_t ld) {
        const int64_t col0 = tile * NB;
        const int64_t ncols = a.N - col0 < NB ? a.N - col0 : NB;
        return make_rsrc(base + col0 * ld, (uint32_t)(((ncols - 1) * ld + n) * 2));
    };
    int vo_x[CB], vo_y[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        vo_x[cb] = (int)(((16 * cb + c) * a.ldx + row0 + 8 * g) * 2);
        vo_y[cb] = (int)(((16 * cb + c) * a.ldy + row0 + 8 * g) * 2);
    }
    // X tile p-group load; rows at or past n read as zero
    auto load_x = [&](__amdgpu_buffer_rsrc_t rX, int p, int cb) {
        v8 v = bload<v8>(rX, vo_x[cb], 64 * p);
        if (row0 + 32 * p + 8 * g >= n) v = v8{};
        return v;
    };
    v8 xr[P][CB];
    // Every block alternates a compute phase (no HBM access) with an HBM
    // phase (the tile's stores, then the next tile's loads).  Started together,
    // the blocks stay in step, so HBM idles during the compute phases and is
    // oversubscribed during the HBM phases.  With many tiles per block, the
    // blocks of each XCD (dispatched round-robin over the 8 XCDs) start at 16
    // staggered times, spread over about two tile periods, so that the HBM
    // phases of different compute units overlap other units' products.
    {
        const int64_t per_block = ntiles / gridDim.x;
        const int units = per_block < 4 ? 0 : (int)std::min<int64_t>(30, per_block - 2);
        const int ph = (blockIdx.x >> 3) & 15;
        for (int i = 0; i < ph * units / 15; ++i) __builtin_amdgcn_s_sleep(127);
    }
    if ((int64_t)blockIdx.x < ntiles) {
        const __amdgpu_buffer_rsrc_t rX0 = tile_rsrc(blockIdx.x, X, a.ldx);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) xr[p][cb] = load_x(rX0, p, cb);
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t col0 = tile * NB;
        const int64_t next = tile + gridDim.x;
        const bool has_next = next < ntiles;
        const __amdgpu_buffer_rsrc_t rY = tile_rsrc(tile, Yo, a.ldy);
        const __amdgpu_buffer_rsrc_t rXn = tile_rsrc(has_next ? next : tile, X, a.ldx);
        // y = x - C, rounded to the 16-bit type, written back into the
        // register tile.  No HBM access happens inside the GEMM loops: vmcnt
        // retires in issue order, so a store or HBM load issued there would
        // make every later L2 operand fetch wait for an HBM round trip.
        auto keep_out = [&](int p, const f32x4(&cc)[2][CB]) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                v8 y;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    y[j] = (el)((float)xr[p][cb][j] - cc[0][cb][j]);
                    y[j + 4] = (el)((float)xr[p][cb][j + 4] - cc[1][cb][j]);
                }
                pin(y);
                xr[p][cb] = y;
            }
        };
        if constexpr (OP == W_SYM) {
            // z = lam .* (x - C), rounded back into the register tile
            const __amdgpu_buffer_rsrc_t rL = make_rsrc(a.lam, (uint32_t)npad * 4);
            const int vo_l = (row0 + 8 * g) * 4;
            wy_pass(xr, true, 0, col0, true, [&](int p, const f32x4(&cc)[2][CB]) {
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
                    pin(z);
                    xr[p][cb] = z;
                }
            });
            wy_pass(xr, false, 1, col0, a.store != 0, keep_out);
        } else {
            wy_pass(xr, OP == W_APPLY_T, 0, col0, a.store != 0, keep_out);
        }
        // stores of this tile, then the next tile's loads into the same registers
        if (a.store) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    if (row0 + 32 * p + 8 * g < n) bstore<v8>(rY, xr[p][cb], vo_y[cb], 64 * p);
                }
        }
        if (has_next) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) xr[p][cb] = load_x(rXn, p, cb);
        }
    }
}

// ---------------------------------------------------------------------------
// Host side.
size_t wy_lds_bytes(const WyShape &s) {
    const size_t nb = 16 * s.cb, hp = s.hp;
    return kWaves * hp * (nb + 4) * 4 + 2 * nb * (hp + 8) * 2;
}

__global__ void k_fill_lam(const float *__restrict__ lam, int n, int npad, float *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < npad) out[i] = i < n ? lam[i] : 0.f;
}

template <typename E>
hipError_t wy_setup(const WyShape &s, const float *U, int64_t ldu, int64_t n, int64_t h,
                    const float *lam, bool want_m, char *ws, const WyWs &w, bool want_uh,
                    hipStream_t st) {
    using el = typename E::elem;
    const int hp = s.hp;
    const bool m = lam && want_m;
    if (lam)
        hipLaunchKernelGGL(k_fill_lam, dim3((s.npad + 255) / 256), dim3(256), 0, st, lam, (int)n, s.npad,
                           reinterpret_cast<float *>(ws + w.lam));
    hipLaunchKernelGGL((k_wy_norm<E>), dim3(hp), dim3(kNormThreads), 0, st, U, ldu, (int)n, (int)h, s.npad,
                       hp, reinterpret_cast<el *>(ws + w.yc), reinterpret_cast<el *>(ws + w.yr),
                       reinterpret_cast<el *>(ws + w.ycs),
                       reinterpret_cast<double *>(ws + w.nrm2),
                       reinterpret_cast<double *>(ws + w.nrmraw),
                       want_uh ? reinterpret_cast<double *>(ws + w.uh64) : nullptr);
    const int nhb = hp / 16;
    const size_t hh = (size_t)hp * hp;
    double *gp = reinterpret_cast<double *>(ws + w.gram);
    hipLaunchKernelGGL((k_wy_gram<E>), dim3(nhb * (nhb + 1) / 2, kGramSeg), dim3(256), 0, st,
                       reinterpret_cast<const el *>(ws + w.yc), s.npad, hp,
                       m ? reinterpret_cast<const float *>(ws + w.lam) : nullptr, gp,
                       m ? gp + kGramSeg * hh : nullptr);
    hipLaunchKernelGGL((k_sum_parts<double>), dim3(hp * hp / 32, m ? 2 : 1), dim3(256), 0, st, gp, kGramSeg,
                       hh, hp * hp, reinterpret_cast<double *>(ws + w.gsum));
    {
        const double *gs = reinterpret_cast<const double *>(ws + w.gsum);
        const double *n2 = reinterpret_cast<const double *>(ws + w.nrm2);
        double *tw = reinterpret_cast<double *>(ws + w.tw);
        el *tf = reinterpret_cast<el *>(ws + w.tf);
        const size_t lds = (size_t)hp * (hp + 1) * 8;
        if (hp == 64)
            hipLaunchKernelGGL((k_wy_tmat<64, E>), dim3(1), dim3(kTmatThreads), lds, st, gs, n2, tw, tf);
        else
            hipLaunchKernelGGL((k_wy_tmat<128, E>), dim3(1), dim3(kTmatThreads), lds, st, gs, n2, tw, tf);
    }
    const int nfrag = 4 * (hp / 16) * (hp / 32) * 64;
    if (m)
        hipLaunchKernelGGL((k_wy_mfrag<E>), dim3((nfrag / 2 + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<const double *>(ws + w.gsum) + hh, hp,
                           reinterpret_cast<el *>(ws + w.mf));
    return hipGetLastError();
}

template <typename E, int P, int CB, int HP, int MINB = 1>
hipError_t launch_main(WyOp op, const WyArgs &a, size_t lds, int grid, hipStream_t st) {
    grid *= MINB;
    switch (op) {
    case W_APPLY:
        hipLaunchKernelGGL((k_wy_fwd<E, P, CB, HP, W_APPLY, MINB>), dim3(grid), dim3(kThreadsWY), lds, st, a);
        break;
    case W_APPLY_T:
        hipLaunchKernelGGL((k_wy_fwd<E, P, CB, HP, W_APPLY_T, MINB>), dim3(grid), dim3(kThreadsWY), lds, st, a);
        break;
    case W_SYM:
        hipLaunchKernelGGL((k_wy_fwd<E, P, CB, HP, W_SYM, MINB>), dim3(grid), dim3(kThreadsWY), lds, st, a);
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

hipError_t wy_setup_any(bool bf, const WyShape &s, const float *U, int64_t ldu, int64_t n,
                        int64_t h, const float *lam, bool want_m, char *ws, const WyWs &w,
                        bool want_uh, hipStream_t st) {
    return bf ? wy_setup<BF16>(s, U, ldu, n, h, lam, want_m, ws, w, want_uh, st)
              : wy_setup<F16>(s, U, ldu, n, h, lam, want_m, ws, w, want_uh, st);
}

// Which main kernel runs: 0 = register-resident tile, 1 = streaming, 2 = by shape.
#ifndef HH_WY_STREAM_POLICY
#define HH_WY_STREAM_POLICY 2
#endif

// The register-resident kernel reads X once and writes it once but streams
// the whole reflector matrix from L2 for every 16-32 vectors; the streaming
// kernel amortises that stream over 128 vectors at the price of one extra
// read of X per phase.  Measured on MI355X (bf16 / fp16): at n hp = 2^18
// (n = 4096, h = 64) Q X takes 1.43 ms resident vs 1.64 ms streaming for
// 2^18 vectors; at n hp = 2^20 (n = 8192, h = 128) Q diag(lam) Q^T X takes
// 1.66 ms vs 1.19 ms for 2^16 vectors.  A pass that only emits the
// backward's coefficients reads X once in either kernel, and streams faster.
bool wy_stream_selected(const WyShape &s, const WyArgs &a) {
    // 32-bit buffer offsets: a tile of 256 vectors and the coefficient rows
    const int64_t lim = (int64_t)1 << 31;
    if (256 * std::max(a.ldx, a.ldy) * 2 >= lim) return false;
    if (a.coef && 4 * (int64_t)s.hp * a.ldc >= lim) return false;
    if (HH_WY_STREAM_POLICY == 0) return false;
    if (HH_WY_STREAM_POLICY == 1) return true;
    return (int64_t)a.n * s.hp >= (int64_t)1 << 19 || !a.store;
}

hipError_t wy_main_any(bool bf, const WyShape &s, WyOp op, const WyArgs &a, hipStream_t st) {
    if (a.N == 0) return hipSuccess;
    if (wy_stream_selected(s, a)) return wy_stream_any(bf, s, op, a, st);
    return bf ? dispatch_main<BF16>(s, op, a, st) : dispatch_main<F16>(s, op, a, st);
}

hh_status wy_workspace_size16(hh_op op, const hh_desc *d, size_t *bytes) {
    WyShape s;
    if (!wy_shape(d->n, d->h, &s))
        return set_error(HH_ERR_UNSUPPORTED, "WY path supports n <= 8192 and h <= 128");
    if (op == HH_OP_MAHAL || op == HH_OP_MAHAL_BWD)
        return set_error(HH_ERR_UNSUPPORTED, "WY path provides Q X, Q^T X and Q diag(lam) Q^T X");
    if (op >= HH_OP_APPLY_BWD) {
        *bytes = wy_bwd_ws_bytes(op, s, d->n, d->N);
        return HH_OK;
    }
    *bytes = wy_ws(s, d->n, op == HH_OP_SYM, false).total;
    return HH_OK;
}

hh_status wy_saved_size(hh_op op, const hh_desc *d, size_t *bytes) {
    WyShape s;
    if (!wy_shape(d->n, d->h, &s))
        return set_error(HH_ERR_UNSUPPORTED, "WY path supports n <= 8192 and h <= 128");
    if (op != HH_OP_APPLY && op != HH_OP_APPLY_T && op != HH_OP_SYM)
        return set_error(HH_ERR_UNSUPPORTED, "a coefficient record exists for Q X, Q^T X and Q diag(lam) Q^T X");
    *bytes = wy_record(s, d->n, d->N, op == HH_OP_SYM).total;
    return HH_OK;
}

hh_status wy_forward16(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                     const void *X, int64_t ldx, const void *Xb, int64_t ldb, void *Y,
                     int64_t ldy, void *saved, size_t saved_bytes, void *ws, size_t ws_bytes,
                     hipStream_t st) {
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
    const bool sym = op == HH_OP_SYM;
    const WyRecord rec = wy_record(s, n, N, sym);
    if (saved) {
        if (saved_bytes < rec.total)
            return set_error(HH_ERR_INVALID_ARG, "saved record needs %zu bytes, got %zu", rec.total, saved_bytes);
        if (((uintptr_t)saved & 15) != 0)
            return set_error(HH_ERR_INVALID_ARG, "saved record must be 16-byte aligned");
    }
    // Without a record N = 0 is a no-op; with one, the setup is still
    // recorded for the backward.
    if (N == 0 && !saved) return HH_OK;
    if (h > 0 && !U) return set_error(HH_ERR_INVALID_ARG, "U must not be null");
    if (N > 0 && (!X || !Y)) return set_error(HH_ERR_INVALID_ARG, "X and Y must not be null");
    if (sym && !lam) return set_error(HH_ERR_INVALID_ARG, "lam must not be null");
    if (N > 0 && Y == X && ldy != ldx) return set_error(HH_ERR_INVALID_ARG, "in-place call needs ldy == ldx");
    // The setup goes to the record when there is one (the workspace is then
    // not touched), else to the workspace.
    const WyWs w = wy_ws(s, n, sym, saved != nullptr);
    if (!saved) {
        if (!ws) return set_error(HH_ERR_INVALID_ARG, "ws must not be null");
        const size_t need = w.total;
        if (ws_bytes < need)
            return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
    }
    char *base = saved ? static_cast<char *>(saved) + rec.setup : static_cast<char *>(ws);
    if (saved) {  // the record's coefficient columns past N are zero
        const hipError_t ez = wy_zero_pad(saved, rec.m, N, rec.ldc, st);
        if (ez != hipSuccess) return set_error(HH_ERR_HIP, "WY zero fill: %s", hipGetErrorString(ez));
    }
    const bool bf = d->compute_dtype == HH_BF16;
    WyArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.Yc = base + w.yc;
    a.Yr = base + w.yr;
    a.Ycs = base + w.ycs;
    a.Tf = base + w.tf;
    a.Mf = base + w.mf;
    a.lam = reinterpret_cast<const float *>(base + w.lam);
    a.store = 1;
    a.coef = saved;
    a.ldc = rec.ldc;
    a.n = (int)n;
    a.npad = s.npad;
    a.N = N;
    // A record serves any backward pass, so it holds Y^T diag(lam) Y (used by
    // the streaming kernel) and the FP64 reflectors whenever they may be needed.
    hipError_t e = wy_setup_any(bf, s, static_cast<const float *>(U), ldu, n, h,
                                sym ? static_cast<const float *>(lam) : nullptr,
                                sym && (saved || wy_stream_selected(s, a)), base, w, saved != nullptr, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY setup launch: %s", hipGetErrorString(e));
    if (N == 0) return HH_OK;
    const WyOp wop = op == HH_OP_APPLY ? W_APPLY : op == HH_OP_APPLY_T ? W_APPLY_T : W_SYM;
    e = wy_main_any(bf, s, wop, a, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY kernel launch: %s", hipGetErrorString(e));
    return HH_OK;
}

}  // namespace hh

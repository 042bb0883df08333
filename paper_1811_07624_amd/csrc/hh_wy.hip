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
// One block of kNormThreads per reflector k, u_k held in registers (n <=
// npad <= kNormThreads * kNormPer = 8192, the compact-WY limit; all loads of
// a thread issued together): u_k / ||u_k|| in FP64, rounded to the 16-bit
// type and written to the three fragment-ordered copies, with ||y_k||^2 of
// the rounded vector.  Sums: wave shuffles, then the wave partials in a
// fixed order.
constexpr int kNormThreads = 1024, kNormPer = 8;

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
    const bool live = k < h;
    float u[kNormPer];
#pragma unroll
    for (int m = 0; m < kNormPer; ++m) {
        const int i = t + kNormThreads * m;
        u[m] = (live && i < n) ? U[(int64_t)k * ldu + i] : 0.f;
    }
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kNormPer; ++m) s += (double)u[m] * (double)u[m];
    const double r = sqrt(block_sum_f64(s, red));
    double s2 = 0.0;
#pragma unroll
    for (int m = 0; m < kNormPer; ++m) {
        const int i = t + kNormThreads * m;
        if (i < npad) {
            const double v = (live && i < n && r > 0.0) ? (double)u[m] / r : 0.0;
            const el y = (el)v;
            Yc[yc_index(k, i, npad)] = y;
            Yr[yr_index(k, i, hp)] = y;
            Ycs[ycs_index(k, i, hp)] = y;
            if (uh64 && live && i < n) uh64[(int64_t)k * n + i] = v;
            const double yd = (double)y;
            s2 += yd * yd;
        }
    }
    s2 = block_sum_f64(s2, red);
    if (t == 0) {
        nrm2[k] = s2;
        if (nrm_raw) nrm_raw[k] = live ? r : 0.0;
    }
}

// Partial Gram matrices of the rounded reflectors in FP64 on the matrix
// cores: Gp[s][a][b] = sum over the rows of segment s of y_a y_b, for the
// 16 x 16 tiles (ta, tb), ta <= tb, one wave per (tile pair, segment).  A
// product of two 16-bit values is exact in FP64; with lam, a second set of
// waves (blockIdx.z = 1) forms Mp[s][a][b] = sum of y_a lam_r y_b, the matrix
// Y^T diag(lam) Y of the symmetric form, where lam_r y_b (24 + 11 significant
// bits) and its product with y_a are exact too.  The FP64 MFMA (16 x 16 x 4)
// takes, from lane l = m + 16 k, A[m][k] and B[k][m], and returns
// D[4 v + l / 16][l % 16] in element v of lane l.
// Lane (c, g) of a fragment of the fragment-ordered copy holds the rows
// 32q + 8g + j of reflector 16hb + c, so for each j it supplies A[c][g] from
// tile ta and B[g][c] from tile tb, the same row behind K index g in both.
// The chunks of 32 rows are fetched kGramGroup at a time, the next group's
// loads in flight while the current one is multiplied.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kGramGroup = 4;

template <typename E>
__global__ __launch_bounds__(kWave) void k_wy_gram(const typename E::elem *__restrict__ Yc, int npad,
                                                  int hp, const float *__restrict__ lam,
                                                  double *__restrict__ Gp, double *__restrict__ Mp) {
    using v8 = typename E::vec8;
    constexpr int QG = kGramGroup;
    const int nhb = hp >> 4;
    int pr = blockIdx.x, ta = 0;
    while (pr >= nhb - ta) {
        pr -= nhb - ta;
        ++ta;
    }
    const int tb = ta + pr;
    const int nq = npad >> 5, qs = nq / kGramSeg, q0 = blockIdx.y * qs, seg = blockIdx.y;
    const int l = threadIdx.x, g = l >> 4;
    const bool wl = blockIdx.z == 1;  // z = 0: G; z = 1 (with lam only): M
    v8 ca[QG], cb[QG], na[QG], nb[QG];
    f32x4 cl[QG][2], nl[QG][2];
    auto fetch = [&](int grp, v8(&A)[QG], v8(&B)[QG], f32x4(&L)[QG][2]) {
#pragma unroll
        for (int u = 0; u < QG; ++u) {
            const int qq = grp * QG + u;
            if (qq < qs) {
                const int q = q0 + qq;
                A[u] = *reinterpret_cast<const v8 *>(Yc + ((size_t)(ta * nq + q) * 64 + l) * 8);
                B[u] = *reinterpret_cast<const v8 *>(Yc + ((size_t)(tb * nq + q) * 64 + l) * 8);
                if (wl) {
                    L[u][0] = *reinterpret_cast<const f32x4 *>(lam + 32 * q + 8 * g);
                    L[u][1] = *reinterpret_cast<const f32x4 *>(lam + 32 * q + 8 * g + 4);
                }
            }
        }
    };
    // two independent MFMA chains (j even, j odd)
    f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    const int ngrp = (qs + QG - 1) / QG;
    fetch(0, ca, cb, cl);
    for (int grp = 0; grp < ngrp; ++grp) {
        if (grp + 1 < ngrp) fetch(grp + 1, na, nb, nl);
#pragma unroll
        for (int u = 0; u < QG; ++u) {
            if (grp * QG + u < qs) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const double a = (double)ca[u][j];
                    double bv = (double)cb[u][j];
                    if (wl) bv *= (double)cl[u][j >> 2][j & 3];
                    if (j & 1)
                        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc1, 0, 0, 0);
                    else
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc0, 0, 0, 0);
                }
            }
        }
        if (grp + 1 < ngrp) {
#pragma unroll
            for (int u = 0; u < QG; ++u) {
                ca[u] = na[u];
                cb[u] = nb[u];
                cl[u][0] = nl[u][0];
                cl[u][1] = nl[u][1];
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t o = ((size_t)seg * hp + 16 * ta + 4 * v + g) * hp + 16 * tb + (l & 15);
        (wl ? Mp : Gp)[o] = acc0[v] + acc1[v];
    }
}

// T = (diag(||y_k||^2/2) + striu(G))^{-1}, upper triangular, FP64, one column
// per wave by back substitution, the columns of a block being 8 neighbours
// (block b: columns 8b .. 8b+7).  With d_k the diagonal, column j solves
// M x = e_j from the bottom: x_i is final once the rows below it are done, and
// each x_i is then removed from the rows above (column-oriented form).  The
// rows are kept scaled by 1/d_k, w_k = r_k / d_k, so x_i = w_i directly and a
// step is one read of lane i and one FMA per row: w_k -= (G_ki / d_k) x_i.
// The scaled coefficients G_ki / d_k (k < i, zero for k >= i) sit in LDS row
// by row, row i holding column i of M, so the 64 lanes of a wave read one row
// contiguously.  Steps run from i = j down to 0; lane k (and k + 64) holds
// rows k (and k + 64).
// Outputs: Tw = T in FP64 (zero below the diagonal); Tf = T (tr = 0) and T^T
// (tr = 1) as 16-bit MFMA A-operand fragments split into hi + lo parts (hi = T
// rounded, lo = the rest rounded) for the streaming kernel's T product:
// fragment (tr, hl, ib, kb), lane (c, g), element j holds
// T'[sigma_row(ib, c)][32 kb + 8 g + j].  Every such 8-element piece lies in
// one block's 8 columns: for tr = 0 it is a row of them (32 kb + 8 g = 8 b),
// for tr = 1 it is 8 rows of the column sigma_row(ib, c).
constexpr int kTmatCols = 8;  // columns (waves) per block
constexpr int kTmatThreads = kTmatCols * kWave;

template <int HP, typename E>
__global__ __launch_bounds__(kTmatThreads) void k_wy_tmat(const double *__restrict__ G,
                                                         const double *__restrict__ nrm2,
                                                         double *__restrict__ Tw,
                                                         typename E::elem *__restrict__ Tf) {
    using el = typename E::elem;
    constexpr int LDN = HP + 1, HB = HP / 16, KS = HP / 32, SL = HP / kWave;
    extern __shared__ double lds_t[];
    double *sInv = lds_t;              // HP: 1 / d_k
    double *sN = lds_t + HP;           // rows 0 .. cmax-1, LDN apart
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int b = blockIdx.x, c0 = kTmatCols * b, cmax = c0 + kTmatCols;
    if (t < HP) {
        const double d = nrm2[t];
        sInv[t] = 1.0 / (d > 0.0 ? 0.5 * d : 0.5);
    }
    __syncthreads();
    // row i of sN = column i of M scaled: sN[i][k] = G[k][i] / d_k for k < i
    // (rows i < cmax; thread t covers i = t % HP of rows k = t / HP + KST r,
    // all its loads issued together)
    {
        constexpr int KST = kTmatThreads / HP, NR = HP / KST;
        const int i = t % HP, k0 = t / HP;
        if (i < cmax) {
            double g[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) g[r] = G[(k0 + KST * r) * HP + i];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int k = k0 + KST * r;
                const double v = g[r] * sInv[k];  // read for every k: no branch
                sN[i * LDN + k] = k < i ? v : 0.0;
            }
        }
    }
    __syncthreads();
    const int j = c0 + wv;
    double w[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) w[s] = (lane + kWave * s == j) ? sInv[j] : 0.0;
    // steps i = j .. 64 read lane i - 64 of w[1] and touch both halves; steps
    // below 64 read w[0] and leave rows >= 64 (all below the step) alone.
    // Each phase starts at the next multiple of PF steps above j (still below
    // cmax, as cmax - 64 s is a multiple of kTmatCols = PF): those extra steps
    // read x = w_i = 0 and change nothing, and the PF-step body needs no
    // branch.  Coefficient rows are read PF steps ahead.
    constexpr int PF = kTmatCols;
#pragma unroll
    for (int s = SL - 1; s >= 0; --s) {
        const int lo = kWave * s;
        if (j < lo) continue;
        const int ihi = lo + PF * ((std::min(j, lo + kWave - 1) - lo + PF) / PF) - 1;
        double buf[PF][SL];
#pragma unroll
        for (int u = 0; u < PF; ++u)
#pragma unroll
            for (int q = 0; q <= s; ++q) buf[u][q] = sN[(ihi - u) * LDN + lane + kWave * q];
        for (int i = ihi; i >= lo; i -= PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int ii = i - u, nx = std::max(ii - PF, 0);
                double cur[SL];
#pragma unroll
                for (int q = 0; q <= s; ++q) {
                    cur[q] = buf[u][q];
                    buf[u][q] = sN[nx * LDN + lane + kWave * q];
                }
                const int src = ii - lo;
                const int xl = __builtin_amdgcn_readlane(__double2loint(w[s]), src);
                const int xh = __builtin_amdgcn_readlane(__double2hiint(w[s]), src);
                const double x = __hiloint2double(xh, xl);
#pragma unroll
                for (int q = 0; q <= s; ++q) w[q] = fma(-cur[q], x, w[q]);
            }
        }
    }
    __syncthreads();  // sN is done with: the 8 columns go to sT
    double *sT = sN;  // sT[c][k] = T[k][c0 + c]
#pragma unroll
    for (int s = 0; s < SL; ++s) sT[wv * HP + lane + kWave * s] = w[s];
    __syncthreads();
    for (int idx = t; idx < HP * kTmatCols; idx += kTmatThreads) {
        const int k = idx / kTmatCols, c = idx % kTmatCols;
        Tw[k * HP + c0 + c] = sT[c * HP + k];
    }
    // 4 HP pieces of 8 elements: tr = 0 (2 HP of them: hl, ib, c) then tr = 1 (hl, e, kb, g)
    for (int p = t; p < 4 * HP; p += kTmatThreads) {
        const int tr = p >= 2 * HP, pp = tr ? p - 2 * HP : p;
        int hl, ib, c, kb, g;
        double v[8];
        if (!tr) {
            hl = pp / HP;
            ib = (pp % HP) / 16;
            c = pp % 16;
            kb = b / 4;
            g = b % 4;
            const int row = sigma_row(ib, c);
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = sT[e * HP + row];
        } else {
            hl = pp / HP;
            const int e = (pp % HP) / (4 * KS), r4 = pp % (4 * KS);
            kb = r4 / 4;
            g = r4 % 4;
            const int row = c0 + e;  // sigma_row(ib, c) = row
            ib = 2 * (row >> 5) + ((row >> 2) & 1);
            c = 4 * ((row >> 3) & 3) + (row & 3);
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = sT[e * HP + 32 * kb + 8 * g + q];
        }
        typename E::vec8 fr;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // through FP32: hi may differ from T's direct 16-bit rounding in a
            // tie, and lo = T - hi (formed in FP64) absorbs that
            const el h16 = (el)(float)v[q];
            fr[q] = hl ? (el)(float)(v[q] - (double)h16) : h16;
        }
        const int f = ((tr * 2 + hl) * HB + ib) * KS + kb;
        *reinterpret_cast<typename E::vec8 *>(Tf + ((size_t)f * 64 + c + 16 * g) * 8) = fr;
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
    if (s.npad > kNormThreads * kNormPer) return hipErrorInvalidValue;  // k_wy_norm holds a row in registers
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
    hipLaunchKernelGGL((k_wy_gram<E>), dim3(nhb * (nhb + 1) / 2, kGramSeg, m ? 2 : 1), dim3(kWave), 0, st,
                       reinterpret_cast<const el *>(ws + w.yc), s.npad, hp,
                       m ? reinterpret_cast<const float *>(ws + w.lam) : nullptr, gp,
                       m ? gp + kGramSeg * hh : nullptr);
    {
        const hipError_t e = launch_sum_parts<double>(gp, kGramSeg, hh, hp * hp, m ? 2 : 1,
                                                      reinterpret_cast<double *>(ws + w.gsum), st);
        if (e != hipSuccess) return e;
    }
    {
        const double *gs = reinterpret_cast<const double *>(ws + w.gsum);
        const double *n2 = reinterpret_cast<const double *>(ws + w.nrm2);
        double *tw = reinterpret_cast<double *>(ws + w.tw);
        el *tf = reinterpret_cast<el *>(ws + w.tf);
        // the last block holds all hp rows of the scaled coefficients
        const size_t lds = ((size_t)hp + (size_t)hp * (hp + 1)) * 8;
        const dim3 grid(hp / kTmatCols);
        if (hp == 64)
            hipLaunchKernelGGL((k_wy_tmat<64, E>), grid, dim3(kTmatThreads), lds, st, gs, n2, tw, tf);
        else
            hipLaunchKernelGGL((k_wy_tmat<128, E>), grid, dim3(kTmatThreads), lds, st, gs, n2, tw, tf);
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

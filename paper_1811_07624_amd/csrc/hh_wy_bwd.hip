// Backward of the compact-WY path (BF16 / FP16 on the matrix cores).
//
// With coefficients scaled by tau (a_k = tau_k y_k^T s_{k-1}, b_k = tau_k y_k^T g_k)
// the chain rule of one reflector chain sums, over the N vectors, to
//   dL/dY = -(G_end A^T + S_0 B^T) + Y C,   C = h x h triangular parts of B A^T
// (the order of the chain decides which triangle; see the combine step).  The
// coefficient matrices are exactly what the WY products compute: for Q X,
// A = T Y^T X and B = T^T Y^T G; for Q^T X the transposes of T swap.  For the
// symmetric form, substituting Q^T G = G - Y B2 and Q^T X = X - Y A1 leaves only
// the inputs X and G in the large products:
//   dL/dY = -diag(lam) (G A1^T + X B2^T) - (G A2^T + X B1^T)
//           + diag(lam) Y (K1 + K1^T) + Y (stril K2 + striu K2^T + striu K3 + stril K3^T)
//   dlam_i = sum_j G_ij X_ij - sum_k Y_ik (G A1^T + X B2^T)_ik + sum_k (Y K1)_ik Y_ik
// with K1 = B2 A1^T, K2 = B1 A1^T, K3 = B2 A2^T (A1 = T^T Y^T X, A2 = T Y^T lam Q^T X,
// B2 = T^T Y^T G, B1 = T Y^T lam Q^T G).
//
// Steps (all on the caller's stream): setup; a WY pass over X that only emits
// A; a WY pass over G that emits B and writes dX (= Q^T G, Q G or S G); one
// rank-N product out = G [A..]^T + X [B..]^T on MFMA with the reduction over
// vectors split across blocks; coefficient Grams on MFMA; then FP64 sums of
// the block partials, the small h x h terms, and the chain rule of the
// normalisation dU = (I - uh uh^T) dL/duh / ||u||.  Partials are summed in a
// fixed order: the result is deterministic for a given device and shape.
#include <algorithm>

#include "hh_wy_common.h"

namespace hh {
namespace {

constexpr int kT = 512;  // threads of the coefficient Gram kernel
#ifndef HH_RANK_ROWS
#define HH_RANK_ROWS 256
#endif
// Rows per block of the rank-N product (32 per wave).  Measured on MI355X:
// 128 or 64 rows (two or four blocks per compute unit) lose more to the
// repeated coefficient reads than they gain in overlap.
constexpr int kRankRows = HH_RANK_ROWS;

struct RankArgs {
    const void *D[2];   // G, X (n x N, 16-bit, column-major)
    int64_t ld[2];
    const void *C[2];   // coefficients for G and for X (m x ldc, 16-bit, row-major in j)
    int64_t ldc;
    float *out;         // [KS][npad][m]
    float *gx;          // nullable: [KS][4][npad]
    int n, npad;
    int64_t N, chunk;
};

// out[s][r][m] = sum over the vectors j of split s of G[r][j] C0[m][j] + X[r][j] C1[m][j].
// Block of NW waves: rows [RB bx, RB bx + RB), RB = 32 NW; wave w owns 32 of
// them, all m columns.
template <typename E, int MB, int NW>
__global__ __launch_bounds__(64 * NW) void k_wy_rank(RankArgs a) {
    using el = typename E::elem;
    using v8 = typename E::vec8;
    constexpr int T = 64 * NW;    // threads
    constexpr int RB = 32 * NW;   // rows per block
    constexpr int M = 16 * MB;
    // LDS row stride of a staged vector slice (elements): 16-byte aligned and
    // 8 banks apart, so the 16 vector slices a transpose read touches spread
    // over the banks
    constexpr int RS = RB + 16;
    constexpr int CSd = 32 + 8;   // LDS row stride of a staged coefficient row
    constexpr int CD = 4;         // 16-byte data chunks per thread per step (8 RB of them)
    constexpr int CC = (2 * M * 4 + T - 1) / T;
    extern __shared__ __align__(16) unsigned char smem[];
    el *sD = reinterpret_cast<el *>(smem);      // [2][32][RS]
    el *sC = sD + 2 * 32 * RS;                  // [2][M][CSd]

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6, c = lane & 15, g = lane >> 4;
    const int rb0 = blockIdx.x * RB;
    const int64_t jb = (int64_t)blockIdx.y * a.chunk;
    const int64_t je = jb + a.chunk < a.N ? jb + a.chunk : a.N;
    const el *D0 = static_cast<const el *>(a.D[0]);
    const el *D1 = static_cast<const el *>(a.D[1]);
    const el *C0 = static_cast<const el *>(a.C[0]);
    const el *C1 = static_cast<const el *>(a.C[1]);

    f32x4 acc[2][MB];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[r][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float gxr[2] = {0.f, 0.f};  // sum_j G X over this lane's 8 vectors, rows 16 rbk + c

    v8 rd[CD], rc[CC];
    auto load_step = [&](int64_t j0) {
#pragma unroll
        for (int t = 0; t < CD; ++t) {
            const int ci = tid + T * t;
            const int src = ci / (4 * RB), cc = ci % (4 * RB), j = cc / (RB / 8), rcn = cc % (RB / 8);
            const int row = rb0 + 8 * rcn;
            const int64_t jj = j0 + j;
            v8 v = {};
            if (jj < je && row < a.n) {
                const el *Dp = src ? D1 : D0;
                v = *reinterpret_cast<const v8 *>(Dp + jj * a.ld[src] + row);
            }
            rd[t] = v;
        }
#pragma unroll
        for (int t = 0; t < CC; ++t) {
            const int ci = tid + T * t;
            v8 v = {};
            if (ci < 2 * M * 4) {
                const int src = ci / (M * 4), cc = ci % (M * 4), mr = cc >> 2, jc = cc & 3;
                if (j0 + 8 * jc < je) {
                    const el *Cp = src ? C1 : C0;
                    v = *reinterpret_cast<const v8 *>(Cp + (int64_t)mr * a.ldc + j0 + 8 * jc);
                }
            }
            rc[t] = v;
        }
    };
    auto store_step = [&]() {
#pragma unroll
        for (int t = 0; t < CD; ++t) {
            const int ci = tid + T * t;
            const int src = ci / (4 * RB), cc = ci % (4 * RB), j = cc / (RB / 8), rcn = cc % (RB / 8);
            *reinterpret_cast<v8 *>(sD + (src * 32 + j) * RS + 8 * rcn) = rd[t];
        }
#pragma unroll
        for (int t = 0; t < CC; ++t) {
            const int ci = tid + T * t;
            if (ci < 2 * M * 4) {
                const int src = ci / (M * 4), cc = ci % (M * 4), mr = cc >> 2, jc = cc & 3;
                *reinterpret_cast<v8 *>(sC + (src * M + mr) * CSd + 8 * jc) = rc[t];
            }
        }
    };

    if (jb < je) load_step(jb);
    for (int64_t j0 = jb; j0 < je; j0 += 32) {
        __syncthreads();
        store_step();
        __syncthreads();
        if (j0 + 32 < je) load_step(j0 + 32);
        // B operand (K = 8 consecutive vectors, N = one row) straight from the
        // vector-major staging by two transpose reads: within each 16-lane
        // group, lane i receives element i % 4 of the 4-element rows addressed
        // by lanes i/4 + 4j, so lane L of group g points at rows 4 (L % 4) ..
        // +3 of vector 8g + L/4 (+4 for the second read), and lane (c, g) gets
        // D[vector 8g + j][row c], j < 8.
        v8 bfr[2][2];
#pragma unroll
        for (int src = 0; src < 2; ++src)
#pragma unroll
            for (int rbk = 0; rbk < 2; ++rbk) {
                const int L = lane & 15;
                const el *p0 = sD + (src * 32 + 8 * g + (L >> 2)) * RS + 32 * w + 16 * rbk + 4 * (L & 3);
                typedef short v4s __attribute__((ext_vector_type(4)));
                typedef __attribute__((address_space(3))) v4s *lds_v4s;
                const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p0));
                const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p0 + 4 * RS));
                bfr[src][rbk] = __builtin_bit_cast(v8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
            }
#pragma unroll
        for (int src = 0; src < 2; ++src) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const v8 afr = *reinterpret_cast<const v8 *>(sC + (src * M + 16 * mb + c) * CSd + 8 * g);
#pragma unroll
                for (int rbk = 0; rbk < 2; ++rbk) acc[rbk][mb] = E::mfma(afr, bfr[src][rbk], acc[rbk][mb]);
            }
        }
        if (a.gx) {
#pragma unroll
            for (int rbk = 0; rbk < 2; ++rbk)
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    gxr[rbk] = __builtin_fmaf((float)bfr[0][rbk][j], (float)bfr[1][rbk][j], gxr[rbk]);
        }
    }
#pragma unroll
    for (int rbk = 0; rbk < 2; ++rbk) {
        const int r = rb0 + 32 * w + 16 * rbk + c;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            *reinterpret_cast<f32x4 *>(a.out + ((size_t)blockIdx.y * a.npad + r) * M + 16 * mb + 4 * g) =
                acc[rbk][mb];
    }
    if (a.gx) {  // partials per vector group g: [KS][4][npad]
#pragma unroll
        for (int rbk = 0; rbk < 2; ++rbk)
            a.gx[((size_t)blockIdx.y * 4 + g) * a.npad + rb0 + 32 * w + 16 * rbk + c] = gxr[rbk];
    }
}

struct GramArgs {
    const void *P[3], *Q[3];  // coefficient rows (HP x ldc, 16-bit)
    int64_t ldc;
    float *out;               // [pairs][KSg][HP][HP]
    int64_t N, chunk;
};

// out[pair][s][k][l] = sum over the vectors j of split s of P[k][j] Q[l][j].
// Each 32-vector step stages the HP x 32 slices of P and Q in LDS once (one
// 16-byte load per thread and matrix, fetched a step ahead into registers),
// and the 8 waves read their MFMA fragments from there (each fragment crosses
// the global read path once per block instead of once per wave): wave w forms
// the NBW = HB*HB/8 output blocks (kb0, lb0 + i), i < NBW, w NBW = kb0 HB + lb0.
template <typename E, int HB>
__global__ __launch_bounds__(kT) void k_wy_cgram(GramArgs a) {
    using el = typename E::elem;
    using v8 = typename E::vec8;
    constexpr int HP = 16 * HB;
    constexpr int NW = kT / 64;
    constexpr int NBW = HB * HB / NW;  // output blocks per wave
    constexpr int RS = 32 + 8;         // LDS row stride (elements): fragment reads spread over the banks
    constexpr int NLD = HP * 4;        // 16-byte pieces per matrix slice
    static_assert(NBW >= 1 && (HB * HB) % NW == 0, "block split");
    __shared__ __align__(16) el sP[2][HP * RS], sQ[2][HP * RS];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6, c = lane & 15, g = lane >> 4;
    const int pair = blockIdx.y;
    const int64_t jb = (int64_t)blockIdx.x * a.chunk;
    const int64_t je = jb + a.chunk < a.N ? jb + a.chunk : a.N;
    const el *Pm = static_cast<const el *>(a.P[pair]);
    const el *Qm = static_cast<const el *>(a.Q[pair]);
    // piece tid of a slice: row tid / 4, columns 8 (tid % 4) .. + 7
    const bool ld = tid < NLD;
    const int lr = tid >> 2, lc = 8 * (tid & 3);
    v8 rp{}, rq{};
    auto fetch = [&](int64_t j0) {  // pad columns past N are zero in the coefficient buffers
        if (ld) {
            rp = *reinterpret_cast<const v8 *>(Pm + (int64_t)lr * a.ldc + j0 + lc);
            rq = *reinterpret_cast<const v8 *>(Qm + (int64_t)lr * a.ldc + j0 + lc);
        }
    };
    f32x4 acc[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kb0 = (w * NBW) / HB, lb0 = (w * NBW) % HB;  // the wave's blocks: (kb0, lb0 + i)
    if (jb < je) fetch(jb);
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += 32) {
        if (ld) {
            *reinterpret_cast<v8 *>(&sP[buf][lr * RS + lc]) = rp;
            *reinterpret_cast<v8 *>(&sQ[buf][lr * RS + lc]) = rq;
        }
        __syncthreads();
        if (j0 + 32 < je) fetch(j0 + 32);
        const v8 afr = *reinterpret_cast<const v8 *>(&sP[buf][(16 * kb0 + c) * RS + 8 * g]);
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const v8 bfr = *reinterpret_cast<const v8 *>(&sQ[buf][(16 * (lb0 + i) + c) * RS + 8 * g]);
            acc[i] = E::mfma(afr, bfr, acc[i]);
        }
        buf ^= 1;
    }
    float *o = a.out + ((size_t)pair * gridDim.x + blockIdx.x) * HP * HP;
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) o[(16 * kb0 + 4 * g + r) * HP + 16 * (lb0 + i) + c] = acc[i][r];
}

// Zero the columns [N, ldc) of an m x ldc coefficient buffer.
template <typename T>
__global__ void k_zero_cols(T *p, int m, int64_t N, int64_t ldc) {
    const int64_t pad = ldc - N;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < (int64_t)m * pad) p[(i / pad) * ldc + N + i % pad] = (T)0;
}

// From the coefficient Grams K[pair] (summed over vector splits in FP64), the
// h x h matrices the combine step needs, stored as M[l][k] at l * hp + k:
//   Ma = K1 + K1^T (symmetric form only), Mb = the order-dependent triangles,
//   Mc = K1 (symmetric form only).
__global__ __launch_bounds__(256) void k_wy_mmat2(const double *__restrict__ Kd, int hp, int kind,
                                                 double *__restrict__ Ma, double *__restrict__ Mb,
                                                 double *__restrict__ Mc) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= hp * hp) return;
    const int l = e / hp, k = e % hp;  // stored M[l][k] at l * hp + k
    auto K = [&](int pr, int i, int j) { return Kd[(size_t)pr * hp * hp + i * hp + j]; };
    double mb = 0.0;
    if (kind == 0) {         // Q X: chain visits k = h..1 -> striu(K) + stril(K^T)
        mb = (l < k ? K(0, l, k) : 0.0) + (l > k ? K(0, k, l) : 0.0);
    } else if (kind == 1) {  // Q^T X: chain visits k = 1..h -> stril(K) + striu(K^T)
        mb = (l > k ? K(0, l, k) : 0.0) + (l < k ? K(0, k, l) : 0.0);
    } else {                 // symmetric form
        mb = (l > k ? K(1, l, k) : 0.0) + (l < k ? K(1, k, l) : 0.0) +
             (l < k ? K(2, l, k) : 0.0) + (l > k ? K(2, k, l) : 0.0);
        Ma[e] = K(0, l, k) + K(0, k, l);
        Mc[e] = K(0, l, k);
    }
    Mb[e] = mb;
}

struct CombineArgs {
    const double *part;  // [npad][m], rank-N product summed over the vector splits
    const double *gx;    // nullable [npad], sum_j G_rj X_rj
    int m;
    const double *uh;    // h x n, FP64 unit reflectors
    const double *Ma, *Mb, *Mc;  // hp x hp, M[l][k] at l * hp + k
    const float *lam;    // padded spectrum (symmetric form)
    double *dV;          // hp x npad
    float *dlam;         // nullable, n
    int n, h, npad, kind;
};

// dV[k][r] = -(rank-N product)[r][k] + sum_l y[r][l] M[l][k] (plus the lam
// terms of the symmetric form).  256 threads for kCombineRows rows (two blocks
// per compute unit at n = 8192): thread k = t % HP owns reflector k for RT
// consecutive rows of its row group t / HP.  The y rows of the block
// sit in LDS; the M matrices pass through LDS LC rows at a time, each element
// serving RT rows.
constexpr int kCombineRows = 16;

template <int HP>
__global__ __launch_bounds__(256, 2) void k_wy_combine(CombineArgs a) {
    constexpr int NG = 256 / HP, R = kCombineRows, RT = R / NG, LC = 8;
    __shared__ double ys[R][HP + 1];
    __shared__ double sm[3][LC][HP];
    const int t = threadIdx.x;
    const int k = t % HP, grp = t / HP;
    const int r0 = blockIdx.x * R;
    const bool sym = a.kind == 2;
    const int nm = sym ? 3 : 1;
    for (int e = t; e < R * HP; e += 256) {
        const int kk = e / R, rr = e % R, r = r0 + rr;
        ys[rr][kk] = (kk < a.h && r < a.n) ? a.uh[(size_t)kk * a.n + r] : 0.0;
    }
    double yb[RT], ya[RT], yc[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) yb[i] = ya[i] = yc[i] = 0.0;
    // the next LC rows of the M matrices are fetched into registers while the
    // current ones are used
    constexpr int PER = LC * HP / 256;
    double pre[3][PER];
    auto fetch = [&](int l0) {
#pragma unroll
        for (int mi = 0; mi < 3; ++mi) {
            if (mi < nm) {
                const double *src = (mi == 0 ? a.Mb : mi == 1 ? a.Ma : a.Mc) + (size_t)l0 * HP;
#pragma unroll
                for (int q = 0; q < PER; ++q) pre[mi][q] = src[q * 256 + t];
            }
        }
    };
    fetch(0);
#pragma unroll 1
    for (int l0 = 0; l0 < HP; l0 += LC) {
        __syncthreads();
#pragma unroll
        for (int mi = 0; mi < 3; ++mi) {
            if (mi < nm) {
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = q * 256 + t;
                    sm[mi][e / HP][e % HP] = pre[mi][q];
                }
            }
        }
        __syncthreads();
        if (l0 + LC < HP) fetch(l0 + LC);
#pragma unroll 2
        for (int ll = 0; ll < LC; ++ll) {
            const double mb = sm[0][ll][k];
            const double ma = sym ? sm[1][ll][k] : 0.0;
            const double mc = sym ? sm[2][ll][k] : 0.0;
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const double y = ys[grp * RT + i][l0 + ll];
                yb[i] += y * mb;
                ya[i] += y * ma;
                yc[i] += y * mc;
            }
        }
    }
    double contrib[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int r = r0 + grp * RT + i;
        const double *row = a.part + (size_t)r * a.m;
        const double o1 = row[k];
        const double o2 = sym ? row[HP + k] : 0.0;
        double dv;
        if (sym) {
            const double lr = (double)a.lam[r];  // padded with zeros past n
            const double yk = ys[grp * RT + i][k];
            dv = -lr * o1 - o2 + lr * ya[i] + yb[i];
            contrib[i] = -yk * o1 + yc[i] * yk;
        } else {
            dv = -o1 + yb[i];
            contrib[i] = 0.0;
        }
        a.dV[(size_t)k * a.npad + r] = dv;
    }
    if (!sym || !a.dlam) return;
    __syncthreads();  // reuse ys for the per-row sums over k
#pragma unroll
    for (int i = 0; i < RT; ++i) ys[grp * RT + i][k] = contrib[i];
    __syncthreads();
    if (t < R) {
        const int r = r0 + t;
        if (r < a.n) {
            double s = 0.0;
            for (int kk = 0; kk < HP; ++kk) s += ys[t][kk];
            a.dlam[r] = (float)((a.gx ? a.gx[r] : 0.0) + s);
        }
    }
}

// dU_k = (I - uh_k uh_k^T) dV_k / ||u_k||, one block per reflector, the row
// held in registers (n <= kFinishThreads * kFinishPer = 8192, the compact-WY
// limit; all loads of a thread issued together); uh_k^T dV_k summed by wave
// shuffles, then the wave partials in a fixed order.
constexpr int kFinishThreads = 1024, kFinishPer = 8;
static_assert(kFinishThreads * kFinishPer >= 8192, "k_wy_finish must cover the compact-WY limit n <= 8192");
__global__ __launch_bounds__(kFinishThreads) void k_wy_finish(const double *__restrict__ dV, int npad, int n,
                                                             const double *__restrict__ uh,
                                                             const double *__restrict__ nrm,
                                                             float *__restrict__ dU, int64_t lddu) {
    constexpr int NW = kFinishThreads / 64;
    __shared__ double red[NW];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    const double *v = dV + (size_t)k * npad;
    const double *u = uh + (size_t)k * n;
    double uu[kFinishPer], vv[kFinishPer];
#pragma unroll
    for (int m = 0; m < kFinishPer; ++m) {
        const int e = t + kFinishThreads * m;
        uu[m] = e < n ? u[e] : 0.0;
        vv[m] = e < n ? v[e] : 0.0;
    }
    double p = 0.0;
#pragma unroll
    for (int m = 0; m < kFinishPer; ++m) p += uu[m] * vv[m];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if ((t & 63) == 0) red[t >> 6] = p;
    __syncthreads();
    p = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) p += red[w];
    const double nk = nrm[k];
#pragma unroll
    for (int m = 0; m < kFinishPer; ++m) {
        const int e = t + kFinishThreads * m;
        if (e < n) dU[e + (int64_t)k * lddu] = nk > 0.0 ? (float)((vv[m] - p * uu[m]) / nk) : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Host side.
struct BwdLayout {
    WyWs base;
    int64_t ldc;
    int m, ks, ksg, npairs;
    int64_t chunk, gchunk;
    size_t cg, cx, part, gx, psum, gxsum, gpart, kd, ma, mb, mc, dv, total;
};

BwdLayout bwd_layout(hh_op op, const WyShape &s, int64_t n, int64_t N) {
    BwdLayout L{};
    const bool sym = op == HH_OP_SYM_BWD;
    L.base = wy_ws(s, n, sym, true);
    L.ldc = wy_ldc(N);
    L.m = sym ? 2 * s.hp : s.hp;
    const int rowblocks = s.npad / kRankRows;
    const int64_t steps = std::max<int64_t>(1, (N + 31) / 32);
    L.ks = (int)std::min<int64_t>(steps, std::max(1, 2 * device_cu_count() / rowblocks));
    L.chunk = (steps + L.ks - 1) / L.ks * 32;
    L.ks = (int)std::max<int64_t>(1, (N + L.chunk - 1) / L.chunk);
    L.npairs = sym ? 3 : 1;
    L.ksg = (int)std::min<int64_t>(steps, 128);
    L.gchunk = (steps + L.ksg - 1) / L.ksg * 32;
    L.ksg = (int)std::max<int64_t>(1, (N + L.gchunk - 1) / L.gchunk);
    const size_t hp = s.hp;
    size_t off = L.base.total;
    L.cg = off;    off += align256((size_t)L.m * L.ldc * 2);
    L.cx = off;    off += align256((size_t)L.m * L.ldc * 2);
    L.part = off;  off += align256((size_t)L.ks * s.npad * L.m * 4);
    L.gx = off;    off += sym ? align256((size_t)L.ks * 4 * s.npad * 4) : 0;
    L.psum = off;  off += align256((size_t)s.npad * L.m * 8);
    L.gxsum = off; off += sym ? align256((size_t)s.npad * 8) : 0;
    L.gpart = off; off += align256((size_t)L.npairs * L.ksg * hp * hp * 4);
    L.kd = off;    off += align256((size_t)L.npairs * hp * hp * 8);
    L.ma = off;    off += align256(hp * hp * 8);
    L.mb = off;    off += align256(hp * hp * 8);
    L.mc = off;    off += align256(hp * hp * 8);
    L.dv = off;    off += align256(hp * (size_t)s.npad * 8);
    L.total = off;
    return L;
}

template <typename E>
hipError_t launch_products(const WyShape &s, const BwdLayout &L, char *ws, const char *cgp,
                           const void *G, int64_t ldg, const void *X, int64_t ldx, int64_t N,
                           int n, bool sym, hipStream_t st) {
    RankArgs ra{};
    ra.D[0] = G;
    ra.ld[0] = ldg;
    ra.D[1] = X;
    ra.ld[1] = ldx;
    ra.C[0] = cgp;
    ra.C[1] = ws + L.cx;
    ra.ldc = L.ldc;
    ra.out = reinterpret_cast<float *>(ws + L.part);
    ra.gx = sym ? reinterpret_cast<float *>(ws + L.gx) : nullptr;
    ra.n = n;
    ra.npad = s.npad;
    ra.N = N;
    ra.chunk = L.chunk;
    const dim3 rgrid(s.npad / kRankRows, L.ks);
    const size_t rlds = (size_t)(2 * 32 * (kRankRows + 16) + 2 * L.m * (32 + 8)) * 2;
    const dim3 rblock(2 * kRankRows);
    switch (L.m) {
    case 64: hipLaunchKernelGGL((k_wy_rank<E, 4, kRankRows / 32>), rgrid, rblock, rlds, st, ra); break;
    case 128: hipLaunchKernelGGL((k_wy_rank<E, 8, kRankRows / 32>), rgrid, rblock, rlds, st, ra); break;
    default: hipLaunchKernelGGL((k_wy_rank<E, 16, kRankRows / 32>), rgrid, rblock, rlds, st, ra); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GramArgs ga{};
    const size_t hpb = (size_t)s.hp * L.ldc * 2;  // bytes of HP coefficient rows
    const char *cg = cgp, *cx = ws + L.cx;
    if (sym) {  // K1 = B2 A1^T, K2 = B1 A1^T, K3 = B2 A2^T
        ga.P[0] = cx; ga.Q[0] = cg;
        ga.P[1] = cx + hpb; ga.Q[1] = cg;
        ga.P[2] = cx; ga.Q[2] = cg + hpb;
    } else {    // K = B A^T
        ga.P[0] = cx; ga.Q[0] = cg;
    }
    ga.ldc = L.ldc;
    ga.out = reinterpret_cast<float *>(ws + L.gpart);
    ga.N = N;
    ga.chunk = L.gchunk;
    const dim3 ggrid(L.ksg, L.npairs);
    if (s.hp == 64) hipLaunchKernelGGL((k_wy_cgram<E, 4>), ggrid, dim3(kT), 0, st, ga);
    else hipLaunchKernelGGL((k_wy_cgram<E, 8>), ggrid, dim3(kT), 0, st, ga);
    return hipGetLastError();
}

}  // namespace

size_t wy_bwd_ws_bytes(hh_op op, const WyShape &s, int64_t n, int64_t N) {
    return bwd_layout(op, s, n, N).total;
}

hipError_t wy_zero_pad(void *rows, int m, int64_t N, int64_t ldc, hipStream_t st) {
    const int64_t padn = (int64_t)m * (ldc - N);
    if (padn <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_zero_cols<unsigned short>), dim3((unsigned)((padn + 255) / 256)), dim3(256), 0,
                       st, static_cast<unsigned short *>(rows), m, N, ldc);
    return hipGetLastError();
}

hh_status wy_backward16(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                      const void *X, int64_t ldx, const void *Xb, int64_t ldb, const void *G,
                      int64_t ldg, void *dX, void *dXb, int64_t lddx, void *dU, int64_t lddu,
                      void *dlam, const void *saved, size_t saved_bytes, void *ws,
                      size_t ws_bytes, hipStream_t st) {
    (void)Xb;
    (void)ldb;
    (void)dXb;
    WyShape s;
    if (!wy_shape(d->n, d->h, &s))
        return set_error(HH_ERR_UNSUPPORTED, "WY path supports n <= 8192 and h <= 128");
    if (op == HH_OP_MAHAL_BWD)
        return set_error(HH_ERR_UNSUPPORTED, "WY path provides Q X, Q^T X and Q diag(lam) Q^T X");
    if (d->io_dtype != d->compute_dtype)
        return set_error(HH_ERR_UNSUPPORTED, "WY path reads and writes data in the compute type");
    const int64_t n = d->n, h = d->h, N = d->N;
    const bool sym = op == HH_OP_SYM_BWD;
    auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    if (n % 8 != 0 || ldx % 8 != 0 || ldg % 8 != 0 || (dX && lddx % 8 != 0) ||
        (N > 0 && (!al16(X) || !al16(G) || (dX && !al16(dX)))))
        return set_error(HH_ERR_UNSUPPORTED,
                         "WY path needs n and leading dimensions multiples of 8 and 16-byte aligned data");
    const BwdLayout L = bwd_layout(op, s, n, N);
    if (h > 0 && !U) return set_error(HH_ERR_INVALID_ARG, "U must not be null");
    if (N > 0 && (!X || !G)) return set_error(HH_ERR_INVALID_ARG, "X and dY must not be null");
    if (sym && !lam) return set_error(HH_ERR_INVALID_ARG, "lam must not be null");
    if (!ws) return set_error(HH_ERR_INVALID_ARG, "ws must not be null");
    if (ws_bytes < L.total)
        return set_error(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", L.total, ws_bytes);
    const WyRecord rec = wy_record(s, n, N, sym);
    if (saved) {
        if (saved_bytes < rec.total)
            return set_error(HH_ERR_INVALID_ARG, "saved record needs %zu bytes, got %zu", rec.total, saved_bytes);
        if (((uintptr_t)saved & 15) != 0)
            return set_error(HH_ERR_INVALID_ARG, "saved record must be 16-byte aligned");
    }
    const bool want_params = dU || (sym && dlam);
    if (!want_params && (!dX || N == 0)) return HH_OK;

    char *base = static_cast<char *>(ws);
    // the forward's setup (normalised reflectors, T, spectrum) from the record,
    // else formed here in the workspace
    char *sb = saved ? const_cast<char *>(static_cast<const char *>(saved)) + rec.setup : base;
    const bool bf = d->compute_dtype == HH_BF16;
    WyArgs a{};
    a.Yc = sb + L.base.yc;
    a.Yr = sb + L.base.yr;
    a.Ycs = sb + L.base.ycs;
    a.Tf = sb + L.base.tf;
    a.Mf = sb + L.base.mf;
    a.lam = reinterpret_cast<const float *>(sb + L.base.lam);
    a.ldc = L.ldc;
    a.n = (int)n;
    a.npad = s.npad;
    a.N = N;
    const WyOp xop = op == HH_OP_APPLY_BWD ? W_APPLY : op == HH_OP_APPLY_T_BWD ? W_APPLY_T : W_SYM;
    const WyOp gop = op == HH_OP_APPLY_BWD ? W_APPLY_T : op == HH_OP_APPLY_T_BWD ? W_APPLY : W_SYM;
    WyArgs ax = a;  // pass over X: coefficients only
    ax.X = X;
    ax.ldx = ldx;
    ax.Y = const_cast<void *>(X);
    ax.ldy = ldx;
    ax.coef = base + L.cg;
    ax.store = 0;
    WyArgs ag = a;  // pass over G: coefficients and dX
    ag.X = G;
    ag.ldx = ldg;
    ag.Y = dX ? dX : const_cast<void *>(G);
    ag.ldy = dX ? lddx : ldg;
    ag.coef = want_params ? base + L.cx : nullptr;
    ag.store = dX ? 1 : 0;
    const bool want_m = sym && ((want_params && wy_stream_selected(s, ax)) || wy_stream_selected(s, ag));
    hipError_t e = hipSuccess;
    if (!saved) {
        e = wy_setup_any(bf, s, static_cast<const float *>(U), ldu, n, h,
                         sym ? static_cast<const float *>(lam) : nullptr, want_m, base, L.base, true, st);
        if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY setup launch: %s", hipGetErrorString(e));
    }
    // coefficient rows of the pass over X: the caller's record of the
    // forward, else formed here by a coefficient-only pass
    const char *cgp = saved ? static_cast<const char *>(saved) : base + L.cg;
    e = wy_zero_pad(base + L.cx, L.m, N, L.ldc, st);
    if (e == hipSuccess && !saved) e = wy_zero_pad(base + L.cg, L.m, N, L.ldc, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY zero fill: %s", hipGetErrorString(e));
    if (want_params && !saved) {
        e = wy_main_any(bf, s, xop, ax, st);
        if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY pass over X: %s", hipGetErrorString(e));
    }
    e = wy_main_any(bf, s, gop, ag, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY pass over dY: %s", hipGetErrorString(e));
    if (!want_params) return HH_OK;
    e = bf ? launch_products<BF16>(s, L, base, cgp, G, ldg, X, ldx, N, (int)n, sym, st)
           : launch_products<F16>(s, L, base, cgp, G, ldg, X, ldx, N, (int)n, sym, st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY product launch: %s", hipGetErrorString(e));
    const int hp = s.hp;
    const int kind = op == HH_OP_APPLY_BWD ? 0 : op == HH_OP_APPLY_T_BWD ? 1 : 2;
    const dim3 mg((hp * hp + 255) / 256);
    e = launch_sum_parts<float>(reinterpret_cast<const float *>(base + L.gpart), L.ksg, (size_t)hp * hp, hp * hp,
                                L.npairs, reinterpret_cast<double *>(base + L.kd), st);
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY partial sums: %s", hipGetErrorString(e));
    hipLaunchKernelGGL(k_wy_mmat2, mg, dim3(256), 0, st, reinterpret_cast<const double *>(base + L.kd), hp,
                       kind, reinterpret_cast<double *>(base + L.ma), reinterpret_cast<double *>(base + L.mb),
                       reinterpret_cast<double *>(base + L.mc));
    {
        const size_t ne = (size_t)s.npad * L.m;
        e = launch_sum_parts<float>(reinterpret_cast<const float *>(base + L.part), L.ks, ne, (int)ne, 1,
                                    reinterpret_cast<double *>(base + L.psum), st);
        if (e == hipSuccess && sym)
            e = launch_sum_parts<float>(reinterpret_cast<const float *>(base + L.gx), 4 * L.ks, (size_t)s.npad,
                                        s.npad, 1, reinterpret_cast<double *>(base + L.gxsum), st);
        if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY partial sums: %s", hipGetErrorString(e));
    }
    CombineArgs ca{};
    ca.part = reinterpret_cast<const double *>(base + L.psum);
    ca.gx = sym ? reinterpret_cast<const double *>(base + L.gxsum) : nullptr;
    ca.m = L.m;
    ca.uh = reinterpret_cast<const double *>(sb + L.base.uh64);
    ca.Ma = reinterpret_cast<const double *>(base + L.ma);
    ca.Mb = reinterpret_cast<const double *>(base + L.mb);
    ca.Mc = reinterpret_cast<const double *>(base + L.mc);
    ca.lam = reinterpret_cast<const float *>(sb + L.base.lam);
    ca.dV = reinterpret_cast<double *>(base + L.dv);
    ca.dlam = sym ? static_cast<float *>(dlam) : nullptr;
    ca.n = (int)n;
    ca.h = (int)h;
    ca.npad = s.npad;
    ca.kind = kind;
    if (hp == 64) hipLaunchKernelGGL(k_wy_combine<64>, dim3(s.npad / kCombineRows), dim3(256), 0, st, ca);
    else hipLaunchKernelGGL(k_wy_combine<128>, dim3(s.npad / kCombineRows), dim3(256), 0, st, ca);
    if (dU && h > 0)
        hipLaunchKernelGGL(k_wy_finish, dim3((unsigned)h), dim3(kFinishThreads), 0, st,
                           reinterpret_cast<const double *>(base + L.dv), s.npad, (int)n,
                           reinterpret_cast<const double *>(sb + L.base.uh64),
                           reinterpret_cast<const double *>(sb + L.base.nrmraw), static_cast<float *>(dU),
                           lddu);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(HH_ERR_HIP, "WY finish launch: %s", hipGetErrorString(e));
    return HH_OK;
}

}  // namespace hh

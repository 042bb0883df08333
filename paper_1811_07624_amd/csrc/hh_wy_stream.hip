// Streaming form of the compact-WY main kernel (BF16 / FP16 on the matrix
// cores, FP32 accumulation) for long vectors and many reflectors.
//
// The register-resident kernel keeps a tile of only 16-32 vectors on chip, so
// every tile re-reads the whole reflector matrix (hp n 16-bit values, twice)
// from L2; at n h = 2^18 or more that operand stream, not HBM, sets the speed.
// Here a block owns a tile of V = 8 * 16 * NCB vectors (wave w owns 16 NCB of
// them) and sweeps the rows of the tile in chunks of 32 QC rows, once per
// phase, re-reading X from HBM instead of holding it:
//   phase 1   W = Y^T X                       (GEMM1, reduction over the rows)
//   T step    Z = T W  (Q X)  or  T^T W  (Q^T X)
//   phase 3   Y_out = X - Y Z                 (GEMM2)
// and for Q diag(lam) Q^T X, with s = lam .* (X - Y Z1) = diag(lam) Q^T X:
//   phase 1   W1 = Y^T X,  V = Y^T (lam .* X)  (both from one read of X)
//   T steps   Z1 = T^T W1,  W2 = V - M Z1 (= Y^T s, M = Y^T diag(lam) Y),
//             Z2 = T W2
//   phase 3   Y_out = s - Y Z2, s formed from X and rounded to 16 bits.
// Forming Y^T s from V and M instead of from s itself saves a full read of X
// (two reads and one write instead of three reads and one write).
// Reflector chunks reach all 8 waves through LDS (two slots), fetched D chunks
// ahead through registers together with each wave's own X chunk; loads are
// issued reflectors first so that waiting for them never waits for the X
// loads of later chunks (vector-memory counters retire in issue order).
//
// Register layouts (lane l: c = l % 16, g = l / 16; MFMA 16x16x32):
//  * X chunk: rows 32q + 8g + j (j < 8) of vector 16cb + c, one 16-byte load;
//    it is GEMM1's B operand and matches GEMM2's accumulator layout (GEMM2's
//    M rows come permuted from the fragment-ordered copy Yr).
//  * GEMM1's M rows are permuted, h = sigma(hb, r) = 32(hb/2) + 8(r/4) +
//    4(hb%2) + r%4, so its accumulators are directly the B operand of the T
//    product (K index 8g + j of block kb is h = 32kb + 8g + j).  The T
//    product's M rows are permuted the same way, so Z lands directly in the
//    B-operand layout of GEMM2.  No LDS round trip or lane exchange is needed.
//  * T and W enter the T product as 16-bit hi + lo parts (three products,
//    lo*lo dropped), Z enters GEMM2 as hi + lo parts: the corrections keep
//    about twice the 16-bit precision, as in the register-resident kernel
//    (except the Y Z1 of the symmetric form's last phase, see gemm2x2).
#include <algorithm>

#include "hh_wy_common.h"

namespace hh {
namespace {

constexpr int kSW = 8;             // waves per block
constexpr int kST = kSW * kWave;   // threads per block

template <bool YC, bool YR, bool LM> struct Parts {
    static constexpr bool ycs = YC, yr = YR, lam = LM;
};

template <typename E, int HP, int NCB, int QC, int D, int OP, int BPC>
__global__ __launch_bounds__(kST, 2 * BPC) void k_wy_stream(WyArgs a) {
    using el = typename E::elem;
    using v8 = typename E::vec8;
    constexpr int HB = HP / 16, KS = HP / 32;
    constexpr int V = kSW * 16 * NCB;          // vectors per tile
    constexpr int RC = 32 * QC;                // rows per chunk
    constexpr int YCS_B = QC * HB * 1024;      // GEMM1 operand bytes per chunk
    constexpr int YR_B = QC * 2 * KS * 1024;   // GEMM2 operand bytes per chunk
    constexpr int LAM_B = RC * 4;
    constexpr int SLOT = YCS_B + YR_B + LAM_B;
    constexpr int NYC = (YCS_B / 16 + kST - 1) / kST;   // 16-byte pieces per thread
    constexpr int NYR = (YR_B / 16 + kST - 1) / kST;
    constexpr int NY = NYC + NYR + 1;
    extern __shared__ __align__(16) unsigned char smem[];  // [2][SLOT]

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6, c = lane & 15, g = lane >> 4;
    const int n = a.n;
    const int nch = (n + RC - 1) / RC;
    const __amdgpu_buffer_rsrc_t rYcs = make_rsrc(a.Ycs, (uint32_t)HP * a.npad * 2);
    const __amdgpu_buffer_rsrc_t rYr = make_rsrc(a.Yr, (uint32_t)HP * a.npad * 2);
    const __amdgpu_buffer_rsrc_t rLam = make_rsrc(a.lam, (uint32_t)a.npad * 4);
    const __amdgpu_buffer_rsrc_t rTf = make_rsrc(a.Tf, (uint32_t)(8 * HP * HP));
    const __amdgpu_buffer_rsrc_t rMf = make_rsrc(a.Mf, OP == W_SYM ? (uint32_t)(4 * HP * HP) : 0u);
    const el *X = static_cast<const el *>(a.X);
    el *Yo = static_cast<el *>(a.Y);
    const int wcol = 16 * NCB * w;  // first vector of this wave within the tile

    int vo_x[NCB], vo_y[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        vo_x[cb] = (int)(((int64_t)(wcol + 16 * cb + c) * a.ldx + 8 * g) * 2);
        vo_y[cb] = (int)(((int64_t)(wcol + 16 * cb + c) * a.ldy + 8 * g) * 2);
    }

    i32x4 ys[D][NY];
    v8 xs[D][QC][NCB];
    __amdgpu_buffer_rsrc_t rX, rCo;

    // Loads of chunk ch into register stage S: reflector parts first, then X.
    // Every thread issues the same loads for every ch (chunks past the end
    // and rows past n read zeros through out-of-range offsets), so the waits
    // the compiler derives are exact: waiting for one chunk's reflector part
    // never waits for a later chunk's X loads.
    constexpr int NPC = YCS_B / 16, NPR = YR_B / 16, NPL = LAM_B / 16;
    const uint32_t yrange = (uint32_t)HP * a.npad * 2;
    auto issue = [&](auto S, auto parts, int ch) {
        using PT = decltype(parts);
        const bool live = ch < nch;
        if constexpr (PT::ycs) {
#pragma unroll
            for (int i = 0; i < NYC; ++i) {
                const int pc = (tid + i * kST) % NPC;
                ys[S][i] = bload<i32x4>(rYcs, pc * 16, live ? ch * YCS_B : (int)yrange);
            }
        }
        if constexpr (PT::yr) {
#pragma unroll
            for (int i = 0; i < NYR; ++i) {
                const int pc = (tid + i * kST) % NPR;
                ys[S][NYC + i] = bload<i32x4>(rYr, pc * 16, live ? ch * YR_B : (int)yrange);
            }
        }
        if constexpr (PT::lam) {
            ys[S][NY - 1] = bload<i32x4>(rLam, (tid % NPL) * 16, live ? ch * LAM_B : a.npad * 4);
        }
#pragma unroll
        for (int qi = 0; qi < QC; ++qi) {
            const int q = ch * QC + qi;
            const bool ok = 32 * q + 8 * g < n;  // also false past the last chunk
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                xs[S][qi][cb] = bload<v8>(rX, ok ? vo_x[cb] + 64 * q : (int)0x80000000, 0);
        }
    };
    // Register stage S (chunk ch) into LDS slot ch & 1.
    auto commit = [&](auto S, auto parts, int ch) {
        using PT = decltype(parts);
        unsigned char *sl = smem + (ch & 1) * SLOT;
        if constexpr (PT::ycs) {
#pragma unroll
            for (int i = 0; i < NYC; ++i) {
                const int pc = tid + i * kST;
                if (NPC % kST == 0 || pc < NPC) *reinterpret_cast<i32x4 *>(sl + pc * 16) = ys[S][i];
            }
        }
        if constexpr (PT::yr) {
#pragma unroll
            for (int i = 0; i < NYR; ++i) {
                const int pc = tid + i * kST;
                if (NPR % kST == 0 || pc < NPR) *reinterpret_cast<i32x4 *>(sl + YCS_B + pc * 16) = ys[S][NYC + i];
            }
        }
        if constexpr (PT::lam) {
            if (tid < NPL) *reinterpret_cast<i32x4 *>(sl + YCS_B + YR_B + tid * 16) = ys[S][NY - 1];
        }
    };
    // One sweep over the rows: body(ch, slot, x registers of the chunk) for
    // ch < nch rounded up to a multiple of D (the extra chunks are all zero
    // and store nothing), so the unrolled loop has no conditional paths.
    const int nchp = (nch + D - 1) / D * D;
    auto sweep = [&](auto parts, auto &&body) {
        static_for<D>([&](auto S) { issue(S, parts, (int)S); });
        commit(std::integral_constant<int, 0>{}, parts, 0);
        __syncthreads();
        for (int ch0 = 0; ch0 < nchp; ch0 += D) {
            static_for<D>([&](auto S) {
                const int ch = ch0 + S;
                body(ch, smem + (ch & 1) * SLOT, xs[S]);
                issue(S, parts, ch + D);
                commit(std::integral_constant<int, (S + 1) % D>{}, parts, ch + 1);
                __syncthreads();
            });
        }
    };
    auto lds_frag = [&](const unsigned char *p) { return *reinterpret_cast<const v8 *>(p + lane * 16); };

    // GEMM2 correction of chunk row block qi: o[cb][m] = Yr(qi, m) (Zh + Zl)
    auto gemm2 = [&](const unsigned char *sl, int qi, const v8(&z)[2][KS][NCB], f32x4(&o)[NCB][2]) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) o[cb][0] = o[cb][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const v8 a0 = lds_frag(sl + YCS_B + ((qi * 2 + 0) * KS + ks) * 1024);
            const v8 a1 = lds_frag(sl + YCS_B + ((qi * 2 + 1) * KS + ks) * 1024);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                o[cb][0] = E::mfma(a0, z[0][ks][cb], o[cb][0]);
                o[cb][0] = E::mfma(a0, z[1][ks][cb], o[cb][0]);
                o[cb][1] = E::mfma(a1, z[0][ks][cb], o[cb][1]);
                o[cb][1] = E::mfma(a1, z[1][ks][cb], o[cb][1]);
            }
        }
    };
    // Both corrections of the symmetric form's last phase from one read of
    // the GEMM2 operand: o[cb][m] = Yr(qi, m) Z1 from Z1's high part only, and
    // o2[cb][m] = Yr(qi, m) Z2 (high and low parts).  The first forms
    // t = x - Y Z1, which is scaled by lam and rounded to 16 bits at once, so
    // Z1's low part changes s by less than that rounding (measured at
    // n = 8192, h = 128: max relative error of Q diag(lam) Q^T X
    // 3.33e-4 -> 3.40e-4 in FP16, 2.67e-3 -> 2.74e-3 in BF16), for a quarter
    // fewer products.
    auto gemm2x2 = [&](const unsigned char *sl, int qi, const v8(&z)[2][KS][NCB], const v8(&z2)[2][KS][NCB],
                       f32x4(&o)[NCB][2], f32x4(&o2)[NCB][2]) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
            o[cb][0] = o[cb][1] = o2[cb][0] = o2[cb][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const v8 a0 = lds_frag(sl + YCS_B + ((qi * 2 + 0) * KS + ks) * 1024);
            const v8 a1 = lds_frag(sl + YCS_B + ((qi * 2 + 1) * KS + ks) * 1024);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                o[cb][0] = E::mfma(a0, z[0][ks][cb], o[cb][0]);
                o[cb][1] = E::mfma(a1, z[0][ks][cb], o[cb][1]);
                o2[cb][0] = E::mfma(a0, z2[0][ks][cb], o2[cb][0]);
                o2[cb][0] = E::mfma(a0, z2[1][ks][cb], o2[cb][0]);
                o2[cb][1] = E::mfma(a1, z2[0][ks][cb], o2[cb][1]);
                o2[cb][1] = E::mfma(a1, z2[1][ks][cb], o2[cb][1]);
            }
        }
    };
    // GEMM1 step of chunk row block qi: acc[hb][cb] += Ycs(qi, hb)^T b[cb]
    auto gemm1 = [&](const unsigned char *sl, int qi, const v8(&b)[NCB], f32x4(&acc)[HB][NCB]) {
#pragma unroll
        for (int hb = 0; hb < HB; ++hb) {
            const v8 av = lds_frag(sl + (qi * HB + hb) * 1024);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[hb][cb] = E::mfma(av, b[cb], acc[hb][cb]);
        }
    };
    // Both GEMM1 products of the symmetric form's phase 1 from one read of
    // each A fragment: acc += Ycs^T b, acc2 += Ycs^T b2.
    auto gemm1x2 = [&](const unsigned char *sl, int qi, const v8(&b)[NCB], const v8(&b2)[NCB],
                       f32x4(&acc)[HB][NCB], f32x4(&acc2)[HB][NCB]) {
#pragma unroll
        for (int hb = 0; hb < HB; ++hb) {
            const v8 av = lds_frag(sl + (qi * HB + hb) * 1024);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                acc[hb][cb] = E::mfma(av, b[cb], acc[hb][cb]);
                acc2[hb][cb] = E::mfma(av, b2[cb], acc2[hb][cb]);
            }
        }
    };
    // lam .* x, 16-bit
    auto lamx = [&](const unsigned char *sl, int qi, const v8 &x) {
        const f32x4 l0 = *reinterpret_cast<const f32x4 *>(sl + YCS_B + YR_B + (qi * 32 + 8 * g) * 4);
        const f32x4 l1 = *reinterpret_cast<const f32x4 *>(sl + YCS_B + YR_B + (qi * 32 + 8 * g + 4) * 4);
        v8 r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            r[j] = (el)((float)x[j] * l0[j]);
            r[j + 4] = (el)((float)x[j + 4] * l1[j]);
        }
        return r;
    };
    // s = lam .* (x - o), 16-bit
    auto scaled = [&](const unsigned char *sl, int qi, const v8 &x, const f32x4(&o)[2]) {
        const f32x4 l0 = *reinterpret_cast<const f32x4 *>(sl + YCS_B + YR_B + (qi * 32 + 8 * g) * 4);
        const f32x4 l1 = *reinterpret_cast<const f32x4 *>(sl + YCS_B + YR_B + (qi * 32 + 8 * g + 4) * 4);
        v8 s;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[j] = (el)(((float)x[j] - o[0][j]) * l0[j]);
            s[j + 4] = (el)(((float)x[j + 4] - o[1][j]) * l1[j]);
        }
        return s;
    };
    // T step: z = T' W (T' = T or T^T) as GEMM2 B operands, hi + lo; the
    // coefficients of pass `pass` are written for the backward when asked.
    auto tstep = [&](const f32x4(&acc)[HB][NCB], int tr, int pass, int64_t col0, v8(&z)[2][KS][NCB]) {
        v8 wf[2][KS][NCB];
#pragma unroll
        for (int kb = 0; kb < KS; ++kb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float v = acc[2 * kb + j / 4][cb][j % 4];
                    const el hi = (el)v;
                    wf[0][kb][cb][j] = hi;
                    wf[1][kb][cb][j] = (el)(v - (float)hi);
                }
#pragma unroll
        for (int ib = 0; ib < HB; ++ib) {
            v8 th[KS], tl[KS];
#pragma unroll
            for (int kb = 0; kb < KS; ++kb) {
                th[kb] = bload<v8>(rTf, lane * 16, (((tr * 2 + 0) * HB + ib) * KS + kb) * 1024);
                tl[kb] = bload<v8>(rTf, lane * 16, (((tr * 2 + 1) * HB + ib) * KS + kb) * 1024);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                f32x4 zz = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KS; ++kb) {
                    zz = E::mfma(th[kb], wf[0][kb][cb], zz);
                    zz = E::mfma(th[kb], wf[1][kb][cb], zz);
                    zz = E::mfma(tl[kb], wf[0][kb][cb], zz);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const el hi = (el)zz[i];
                    z[0][ib / 2][cb][4 * (ib % 2) + i] = hi;
                    z[1][ib / 2][cb][4 * (ib % 2) + i] = (el)(zz[i] - (float)hi);
                }
                if (a.coef) {
                    // row pass*HP + sigma_row(ib, 4g + i): the g part per lane,
                    // the rest uniform (scalar offset)
                    const int64_t col = col0 + wcol + 16 * cb + c;
                    const int vo = col < a.N ? (int)((col - col0 + 8 * g * a.ldc) * 2) : (int)0x80000000;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = pass * HP + 32 * (ib >> 1) + 4 * (ib & 1) + i;
                        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (el)zz[i]),
                                                              rCo, vo, (int)(row * a.ldc * 2), 0);
                    }
                }
            }
            // keeps the T fragment loads of later row blocks from being
            // hoisted here (they would all be live at once)
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // acc -= M Z for the symmetric form (M and Z as hi + lo parts, lo*lo
    // dropped).  Z is in the B-operand layout of GEMM2 (K = h in order) and
    // M's rows are permuted like T's in tstep, so the product lands in
    // GEMM1's accumulator layout.
    auto mstep = [&](const v8(&z)[2][KS][NCB], f32x4(&acc)[HB][NCB]) {
#pragma unroll
        for (int ib = 0; ib < HB; ++ib) {
            v8 mh[KS], ml[KS];
#pragma unroll
            for (int kb = 0; kb < KS; ++kb) {
                mh[kb] = bload<v8>(rMf, lane * 16, ((0 * HB + ib) * KS + kb) * 1024);
                ml[kb] = bload<v8>(rMf, lane * 16, ((1 * HB + ib) * KS + kb) * 1024);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                f32x4 mz = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KS; ++kb) {
                    mz = E::mfma(mh[kb], z[0][kb][cb], mz);
                    mz = E::mfma(mh[kb], z[1][kb][cb], mz);
                    mz = E::mfma(ml[kb], z[0][kb][cb], mz);
                }
                acc[ib][cb] -= mz;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    const int64_t ntiles = (a.N + V - 1) / V;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t col0 = tile * V;
        const int64_t ncols = a.N - col0 < V ? a.N - col0 : V;
        rX = make_rsrc(X + col0 * a.ldx, (uint32_t)(((ncols - 1) * a.ldx + n) * 2));
        // coefficient rows are 2 HP long at most; the range ends with the buffer
        rCo = make_rsrc(static_cast<el *>(a.coef) + col0, (uint32_t)((2 * HP * a.ldc - col0) * 2));
        const __amdgpu_buffer_rsrc_t rYo = make_rsrc(Yo + col0 * a.ldy, (uint32_t)(((ncols - 1) * a.ldy + n) * 2));
        auto store_rows = [&](int q, int cb, const v8 &y) {  // rows past n are dropped
            bstore<v8>(rYo, y, 32 * q + 8 * g < n ? vo_y[cb] + 64 * q : (int)0x80000000, 0);
        };

        constexpr bool SYM = OP == W_SYM;
        f32x4 acc[HB][NCB], acc2[SYM ? HB : 1][NCB];
#pragma unroll
        for (int hb = 0; hb < HB; ++hb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[hb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (SYM) {
#pragma unroll
            for (int hb = 0; hb < HB; ++hb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc2[hb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
            sweep(Parts<true, false, true>{}, [&](int ch, const unsigned char *sl, const v8(&xc)[QC][NCB]) {
#pragma unroll
                for (int qi = 0; qi < QC; ++qi) {
                    v8 lx[NCB];
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) lx[cb] = lamx(sl, qi, xc[qi][cb]);
                    gemm1x2(sl, qi, xc[qi], lx, acc, acc2);
                }
            });
        } else {
            sweep(Parts<true, false, false>{}, [&](int ch, const unsigned char *sl, const v8(&xc)[QC][NCB]) {
#pragma unroll
                for (int qi = 0; qi < QC; ++qi) gemm1(sl, qi, xc[qi], acc);
            });
        }
        v8 z1[2][KS][NCB];
        tstep(acc, OP == W_APPLY ? 0 : 1, 0, col0, z1);

        if constexpr (SYM) {
            mstep(z1, acc2);
            v8 z2[2][KS][NCB];
            tstep(acc2, 0, 1, col0, z2);
            if (a.store) {
                sweep(Parts<false, true, true>{}, [&](int ch, const unsigned char *sl, const v8(&xc)[QC][NCB]) {
#pragma unroll
                    for (int qi = 0; qi < QC; ++qi) {
                        f32x4 o[NCB][2], o2[NCB][2];
                        gemm2x2(sl, qi, z1, z2, o, o2);
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
                            const v8 sv = scaled(sl, qi, xc[qi][cb], o[cb]);
                            v8 y;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                y[j] = (el)((float)sv[j] - o2[cb][0][j]);
                                y[j + 4] = (el)((float)sv[j + 4] - o2[cb][1][j]);
                            }
                            store_rows(ch * QC + qi, cb, y);
                        }
                    }
                });
            }
        } else {
            if (a.store) {
                sweep(Parts<false, true, false>{}, [&](int ch, const unsigned char *sl, const v8(&xc)[QC][NCB]) {
#pragma unroll
                    for (int qi = 0; qi < QC; ++qi) {
                        f32x4 o[NCB][2];
                        gemm2(sl, qi, z1, o);
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
                            v8 y;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                y[j] = (el)((float)xc[qi][cb][j] - o[cb][0][j]);
                                y[j + 4] = (el)((float)xc[qi][cb][j + 4] - o[cb][1][j]);
                            }
                            store_rows(ch * QC + qi, cb, y);
                        }
                    }
                });
            }
        }
    }
}

template <int HP, int QC> constexpr size_t stream_lds() {
    return 2 * (size_t)(QC * (HP / 16) * 1024 + QC * 2 * (HP / 32) * 1024 + 32 * QC * 4);
}

// BPC = blocks per compute unit (1, or 2 when the registers allow it).
template <typename E, int HP, int NCB, int QC, int D, int BPC>
hipError_t launch_stream(WyOp op, const WyArgs &a, hipStream_t st) {
    constexpr int V = kSW * 16 * NCB;
    const int64_t tiles = (a.N + V - 1) / V;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)BPC * device_cu_count())));
    constexpr size_t lds = stream_lds<HP, QC>();
    switch (op) {
    case W_APPLY:
        hipLaunchKernelGGL((k_wy_stream<E, HP, NCB, QC, D, W_APPLY, BPC>), grid, dim3(kST), lds, st, a);
        break;
    case W_APPLY_T:
        hipLaunchKernelGGL((k_wy_stream<E, HP, NCB, QC, D, W_APPLY_T, BPC>), grid, dim3(kST), lds, st, a);
        break;
    case W_SYM:
        hipLaunchKernelGGL((k_wy_stream<E, HP, NCB, QC, D, W_SYM, BPC>), grid, dim3(kST), lds, st, a);
        break;
    }
    return hipGetLastError();
}

// Tile shapes measured best on MI355X: 128 vectors per block and chunks of
// 256 rows for h <= 64; 256 vectors per block and chunks of 64 rows for
// h <= 128 (the symmetric form then spills a few registers and is still 8 %
// faster than with 128 vectors); two chunks in flight.
#ifndef HH_STREAM_NCB64
#define HH_STREAM_NCB64 1
#endif
#ifndef HH_STREAM_NCB128
#define HH_STREAM_NCB128 2
#endif
#ifndef HH_STREAM_QC64
#define HH_STREAM_QC64 8
#endif
#ifndef HH_STREAM_QC128
#define HH_STREAM_QC128 2
#endif
#ifndef HH_STREAM_D
#define HH_STREAM_D 2
#endif
#ifndef HH_STREAM_BPC64
#define HH_STREAM_BPC64 1
#endif
#ifndef HH_STREAM_BPC128
#define HH_STREAM_BPC128 1
#endif

template <typename E>
hipError_t dispatch_stream(const WyShape &s, WyOp op, const WyArgs &a, hipStream_t st) {
    if (s.hp == 64)
        return launch_stream<E, 64, HH_STREAM_NCB64, HH_STREAM_QC64, HH_STREAM_D, HH_STREAM_BPC64>(op, a, st);
    return launch_stream<E, 128, HH_STREAM_NCB128, HH_STREAM_QC128, HH_STREAM_D, HH_STREAM_BPC128>(op, a, st);
}

}  // namespace

hipError_t wy_stream_any(bool bf, const WyShape &s, WyOp op, const WyArgs &a, hipStream_t st) {
    if (a.N == 0) return hipSuccess;
    return bf ? dispatch_stream<BF16>(s, op, a, st) : dispatch_stream<F16>(s, op, a, st);
}

}  // namespace hh

// Fused backward kernels for Q X, Q^T X, Q diag(lam) Q^T X and the
// Mahalanobis distance, in FP32 or FP64.
//
// The paper never differentiates the application of its factorisation; the
// gradients here are the chain rule of the reflector steps it defines
// (Sec. II-A, eq. 2).  For one step s_r = s_{r-1} - tau (u^T s_{r-1}) u with
// upstream g_r = dL/ds_r:
//     dL/ds_{r-1} = g_r - tau (u^T g_r) u          (H is symmetric)
//     dL/du      += -tau [ (u^T s_{r-1}) g_r + (u^T g_r) s_{r-1} ]
// Intermediate vectors are not stored: the forward sweep keeps only the h dot
// products a_r = u^T s_{r-1} (in LDS; for the distance, a record the forward
// wrote can supply them, and the forward sweep is then updates only), and the
// reverse sweep rebuilds
// s_{r-1} = s_r + tau a_r u, which undoes the forward update exactly up to one
// rounding because H is its own inverse.
//
// A wave owns V vectors (64 lanes x NC 16-byte chunks each) and walks their
// chains side by side: the V dot products of a step are independent, which
// hides the latency of their cross-lane reductions.  The h reflectors are
// staged in LDS once per block when they fit with the per-vector state in the
// 64 KB budget (both sweeps walk them many times per vector); otherwise both
// sweeps read them from the workspace through the caches (UL = false).  A lane
// holds at most 16 chunks of a vector, so n <= 4096 in FP32 and 2048 in FP64;
// longer vectors are refused (HH_ERR_UNSUPPORTED).  dL/du for
// HB reflectors at a time stays in registers across all the vectors a block
// processes (shared by the V vectors of a wave); larger h takes several passes.  Each block writes its partial
// sums; a second kernel adds the block partials in a fixed order in FP64
// (deterministic for a given grid), scales by -tau_k and applies the chain
// rule of the normalisation uh = u/||u||: dU = (I - uh uh^T) dL/duh / ||u||.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "hh_bwd.h"

namespace hh {
namespace {

constexpr int kWPB = 4;
constexpr int kThreads = kWPB * kWave;
constexpr size_t kLdsBudget = 64 * 1024;

enum BwdOp { B_APPLY = 0, B_APPLY_T = 1, B_SYM = 2, B_MAHAL = 3 };

template <typename T, int NC> constexpr int hb_for() {
    constexpr int regs_per_elem = sizeof(T) / 4;
    constexpr int E = NC * V16<T>::W;
    constexpr int hb = 128 / (E * regs_per_elem);
    return hb < 1 ? 1 : (hb > 16 ? 16 : hb);
}

#ifndef HH_BWD_SUM4
#define HH_BWD_SUM4 1
#endif

// Sums of four values over the 64 lanes of a wave, for the four chains of a
// step at once.  Two exchange steps inside each quad leave lane l with the
// quad sum of value l % 4 (each step keeps one value and sends the other),
// two row rotations complete the row sums and two lane permutes (LDS
// crossbar, no LDS memory) add the four rows; lane v then holds sum v.
// 17 VALU instructions for four sums instead of 28.
__device__ __forceinline__ void wave_sum4(float (&p)[4]) {
    const int l = __lane_id();
    const bool b0 = l & 1, b1 = l & 2;
    float k1 = b0 ? p[1] : p[0];
    const float s1 = b0 ? p[0] : p[1];
    float k2 = b0 ? p[3] : p[2];
    const float s2 = b0 ? p[2] : p[3];
    k1 += dpp_mov<0xB1>(s1);  // from lane l ^ 1
    k2 += dpp_mov<0xB1>(s2);
    float k = b1 ? k2 : k1;
    const float s = b1 ? k1 : k2;
    k += dpp_mov<0x4E>(s);    // from lane l ^ 2
    k += dpp_mov<0x124>(k);
    k += dpp_mov<0x128>(k);
    k += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((l ^ 16) << 2, __builtin_bit_cast(int, k)));
    k += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((l ^ 32) << 2, __builtin_bit_cast(int, k)));
#pragma unroll
    for (int v = 0; v < 4; ++v) p[v] = read_lane(k, v);
}

template <typename T, int NC, int OP, bool UL, int HB, int V>
__global__ __launch_bounds__(kThreads) void k_fused_bwd(FusedBwdArgs a, int k0, int kcnt,
                                                       int write_dx, int do_lam, int nblocks) {
    using VT = typename V16<T>::type;
    constexpr int W = V16<T>::W;
    constexpr int E = NC * W;
    constexpr int STR = kWave * W;
    extern __shared__ __align__(16) unsigned char smem[];

    const int n = a.n, h = a.h, npad = a.npad;
    const int R = (OP == B_SYM) ? 2 * h : h;
    const int RS = R > 0 ? R : 1;
    // LDS: [reflectors (UL only)] [spectrum] [combine buffer] [saved dots] [tau]
    T *sU = reinterpret_cast<T *>(smem);
    T *sLam = sU + (UL ? (size_t)h * npad : 0);
    T *sComb = sLam + npad;
    T *sAl = sComb + npad;
    T *sTau = sAl + kWPB * V * RS;
    const T *uBase = UL ? sU : static_cast<const T *>(a.ut);

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    {
        if constexpr (UL) {
            const VT *src = static_cast<const VT *>(a.ut);
            VT *dst = reinterpret_cast<VT *>(sU);
            const int total = h * (npad / W);
            for (int i = tid; i < total; i += kThreads) dst[i] = src[i];
        }
        if constexpr (OP == B_SYM || OP == B_MAHAL) {
            const VT *ls = static_cast<const VT *>(a.lam);
            for (int i = tid; i < npad / W; i += kThreads) reinterpret_cast<VT *>(sLam)[i] = ls[i];
        }
        for (int i = tid; i < h; i += kThreads) sTau[i] = static_cast<const T *>(a.tau)[i];
    }
    __syncthreads();
    T *myAl = sAl + wave * V * RS;  // vector v's saved dots at myAl + v * RS

    T acc[HB][E];
    T lacc[E];
#pragma unroll
    for (int b = 0; b < HB; ++b)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[b][e] = (T)0;
#pragma unroll
    for (int e = 0; e < E; ++e) lacc[e] = (T)0;

    auto load_u = [&](int k, VT(&uv)[NC]) {
        const T *u = uBase + (size_t)k * npad + lane * W;
#pragma unroll
        for (int i = 0; i < NC; ++i) uv[i] = *reinterpret_cast<const VT *>(u + i * STR);
    };
    // Lane partial of u^T v: one accumulation chain per vector when the V
    // chains of a step run side by side (no partial sums to merge).
    auto dotp = [&](const VT(&uv)[NC], const T(&v)[E]) {
        T p;
        if constexpr (V > 1) {
            p = uv[0][0] * v[0];
#pragma unroll
            for (int e = 1; e < E; ++e) p = fmat(uv[e / W][e % W], v[e], p);
        } else {
            T part[W];
#pragma unroll
            for (int q = 0; q < W; ++q) part[q] = (T)0;
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int q = 0; q < W; ++q) part[q] = fmat(uv[i][q], v[i * W + q], part[q]);
            p = part[0];
#pragma unroll
            for (int q = 1; q < W; ++q) p += part[q];
        }
        return p;
    };
    // p[v] <- u^T x_v for the V vectors of a step (wave-uniform results)
    auto dots = [&](const VT(&uv)[NC], const T(&x)[V][E], T(&p)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) p[v] = dotp(uv, x[v]);
        if constexpr (V == 4 && std::is_same_v<T, float> && HH_BWD_SUM4) {
            wave_sum4(p);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) p[v] = group_sum<64>(p[v]);
        }
    };
    auto axpy = [&](T coef, const VT(&uv)[NC], T(&v)[E]) {
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int q = 0; q < W; ++q) v[i * W + q] = fmat(coef, uv[i][q], v[i * W + q]);
    };
    // forward sweep over one chain; up: k = r, down: k = h-1-r.  Stores a_r.
    auto fwd_chain = [&](bool up, T(&s)[V][E], int abase) {
#pragma unroll 1
        for (int r = 0; r < h; ++r) {
            const int k = up ? r : h - 1 - r;
            VT uv[NC];
            load_u(k, uv);
            T p[V];
            dots(uv, s, p);
            const T t = sTau[k];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (lane == 0) myAl[v * RS + abase + r] = p[v];
                axpy(-p[v] * t, uv, s[v]);
            }
        }
    };
    // One reverse step for reflector k at chain position r: rebuilds s_{r-1},
    // propagates g and, when ACC, accumulates dL/du into acc[B].
    auto rev_step = [&](auto accb, int k, int r, T(&s)[V][E], T(&g)[V][E], int abase) {
        constexpr int B = decltype(accb)::value;
        VT uv[NC];
        load_u(k, uv);
        T beta[V];
        dots(uv, g, beta);
        const T t = sTau[k];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T p = myAl[v * RS + abase + r];
            axpy(t * p, uv, s[v]);  // s <- s_{r-1}
            if constexpr (B >= 0) {
#pragma unroll
                for (int e = 0; e < E; ++e)
                    acc[B][e] = fmat(p, g[v][e], fmat(beta[v], s[v][e], acc[B][e]));
            }
            axpy(-t * beta[v], uv, g[v]);
        }
    };
    using NoAcc = std::integral_constant<int, -1>;
    // reverse sweep over one chain.  The accumulated window k0 .. k0+kcnt-1 is
    // a contiguous run of steps, walked with compile-time accumulator slots.
    auto rev_chain = [&](bool up, T(&s)[V][E], T(&g)[V][E], int abase) {
        const int kw = k0 + kcnt;
        if (up) {  // reverse visits k = h-1 .. 0, position r = k
#pragma unroll 1
            for (int k = h - 1; k >= kw; --k) rev_step(NoAcc{}, k, k, s, g, abase);
            static_for<HB>([&](auto bb) {
                constexpr int b = HB - 1 - decltype(bb)::value;
                if (b < kcnt) rev_step(std::integral_constant<int, b>{}, k0 + b, k0 + b, s, g, abase);
            });
#pragma unroll 1
            for (int k = k0 - 1; k >= 0; --k) rev_step(NoAcc{}, k, k, s, g, abase);
        } else {   // reverse visits k = 0 .. h-1, position r = h-1-k
#pragma unroll 1
            for (int k = 0; k < k0; ++k) rev_step(NoAcc{}, k, h - 1 - k, s, g, abase);
            static_for<HB>([&](auto bb) {
                constexpr int b = decltype(bb)::value;
                if (b < kcnt) rev_step(std::integral_constant<int, b>{}, k0 + b, h - 1 - k0 - b, s, g, abase);
            });
#pragma unroll 1
            for (int k = kw; k < h; ++k) rev_step(NoAcc{}, k, h - 1 - k, s, g, abase);
        }
    };
    auto load_vec = [&](T(&x)[E], const T *base, int64_t ld, int64_t j, bool valid) {
        if (a.vec_ok) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const int e0 = i * STR + lane * W;
                VT v = {};
                if (valid && e0 < n) v = *reinterpret_cast<const VT *>(base + j * ld + e0);
#pragma unroll
                for (int q = 0; q < W; ++q) x[i * W + q] = v[q];
            }
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const int e = i * STR + lane * W + q;
                    x[i * W + q] = (valid && e < n) ? base[j * ld + e] : (T)0;
                }
        }
    };
    auto store_vec = [&](const T(&x)[E], T sign, T *base, int64_t ld, int64_t j) {
        if (a.vec_ok) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const int e0 = i * STR + lane * W;
                if (e0 < n) {
                    VT v;
#pragma unroll
                    for (int q = 0; q < W; ++q) v[q] = sign * x[i * W + q];
                    *reinterpret_cast<VT *>(base + j * ld + e0) = v;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const int e = i * STR + lane * W + q;
                    if (e < n) base[j * ld + e] = sign * x[i * W + q];
                }
        }
    };
    auto lam_chunk = [&](int i) { return *reinterpret_cast<const VT *>(sLam + i * STR + lane * W); };
    // x <- diag(d) x for the caller's n diagonal entries (read through the
    // caches; entries past n are zero in x already)
    auto scale = [&](T(&x)[E], const void *dv) {
        const T *d = static_cast<const T *>(dv);
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int e = i * STR + lane * W + q;
                x[i * W + q] *= (e < n) ? d[e] : (T)0;
            }
    };

    const int64_t vpb = (int64_t)kWPB * V;
    for (int64_t b0 = (int64_t)blockIdx.x * vpb; b0 < a.N; b0 += (int64_t)gridDim.x * vpb) {
        const int64_t j0 = b0 + (int64_t)wave * V;
        T s[V][E], g[V][E];
#pragma unroll
        for (int v = 0; v < V; ++v) load_vec(s[v], static_cast<const T *>(a.X), a.ldx, j0 + v, j0 + v < a.N);
        if constexpr (OP == B_MAHAL) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                load_vec(g[v], static_cast<const T *>(a.Xb), a.ldb, j0 + v, j0 + v < a.N);
#pragma unroll
                for (int e = 0; e < E; ++e) s[v][e] -= g[v][e];
            }
        }
        if (a.din)
#pragma unroll
            for (int v = 0; v < V; ++v) scale(s[v], a.din);
        if constexpr (OP == B_APPLY || OP == B_APPLY_T) {
            constexpr bool up = (OP == B_APPLY_T);
            fwd_chain(up, s, 0);
#pragma unroll
            for (int v = 0; v < V; ++v) load_vec(g[v], static_cast<const T *>(a.G), a.ldg, j0 + v, j0 + v < a.N);
            if (a.dout)
#pragma unroll
                for (int v = 0; v < V; ++v) scale(g[v], a.dout);
            rev_chain(up, s, g, 0);
        } else if constexpr (OP == B_SYM) {
            fwd_chain(true, s, 0);
            T z[V][E];
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const VT l = lam_chunk(i);
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        z[v][i * W + q] = s[v][i * W + q];
                        s[v][i * W + q] *= l[q];
                    }
            }
            fwd_chain(false, s, h);
#pragma unroll
            for (int v = 0; v < V; ++v) load_vec(g[v], static_cast<const T *>(a.G), a.ldg, j0 + v, j0 + v < a.N);
            if (a.dout)
#pragma unroll
                for (int v = 0; v < V; ++v) scale(g[v], a.dout);
            rev_chain(false, s, g, h);  // g = Q^T dY
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const VT l = lam_chunk(i);
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        lacc[i * W + q] = fmat(g[v][i * W + q], z[v][i * W + q], lacc[i * W + q]);
                        g[v][i * W + q] *= l[q];
                        s[v][i * W + q] = z[v][i * W + q];
                    }
            }
            rev_chain(true, s, g, 0);
        } else {  // B_MAHAL
            if (a.dots) {
                // the forward's dot products into the wave's slots, then the
                // forward sweep without dot products or reductions
                const T *dp = static_cast<const T *>(a.dots);
                constexpr int RW = 16 / (int)sizeof(T);
                const int hp = (h + RW - 1) / RW * RW;  // record row length
                for (int l = lane; l < V * h; l += kWave) {
                    const int v = l / h, r = l % h;
                    myAl[v * RS + r] = (j0 + v < a.N) ? dp[(j0 + v) * hp + r] : (T)0;
                }
#pragma unroll 1
                for (int r = 0; r < h; ++r) {
                    VT uv[NC];
                    load_u(r, uv);
                    const T t = sTau[r];
#pragma unroll
                    for (int v = 0; v < V; ++v) axpy(-myAl[v * RS + r] * t, uv, s[v]);
                }
            } else {
                fwd_chain(true, s, 0);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const T w = (j0 + v < a.N) ? static_cast<const T *>(a.G)[j0 + v] : (T)0;
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    const VT l = lam_chunk(i);
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const T z = s[v][i * W + q];
                        lacc[i * W + q] = fmat(w * z, z, lacc[i * W + q]);
                        g[v][i * W + q] = (T)2 * w * l[q] * z;
                    }
                }
            }
            rev_chain(true, s, g, 0);
        }
        if (write_dx) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (a.din) scale(g[v], a.din);
                const int64_t j = j0 + v;
                if (j < a.N) {
                    if (a.dX) store_vec(g[v], (T)1, static_cast<T *>(a.dX), a.lddx, j);
                    if constexpr (OP == B_MAHAL)
                        if (a.dXb) store_vec(g[v], (T)-1, static_cast<T *>(a.dXb), a.lddx, j);
                }
            }
        }
    }

    // Block partials: the waves add into one LDS buffer in a fixed order.
    T *part = static_cast<T *>(a.scratch);
    auto emit = [&](const T(&v)[E], T *dst) {
        for (int w = 0; w < kWPB; ++w) {
            __syncthreads();
            if (wave == w) {
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    VT *c = reinterpret_cast<VT *>(sComb + i * STR + lane * W);
                    VT t = (w == 0) ? VT{} : *c;
#pragma unroll
                    for (int q = 0; q < W; ++q) t[q] += v[i * W + q];
                    *c = t;
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < npad; e += kThreads) dst[e] = sComb[e];
    };
    static_for<HB>([&](auto bb) {
        constexpr int b = decltype(bb)::value;
        if (b < kcnt) emit(acc[b], part + ((size_t)blockIdx.x * h + k0 + b) * npad);
    });
    if (do_lam) emit(lacc, part + (size_t)nblocks * h * npad + (size_t)blockIdx.x * npad);
}

// Fixed-order FP64 sum of the block partials: grid (npad/256, h+1); row h is
// the spectrum gradient, written straight to dlam.
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_reduce(const T *__restrict__ part, int nblocks,
                                                   int n, int h, int npad, int kfirst,
                                                   double *__restrict__ red,
                                                   T *__restrict__ dlam) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int k = kfirst + (int)blockIdx.y;
    if (e >= n) return;
    double s = 0.0;
    if (k < h) {
        for (int b = 0; b < nblocks; ++b) s += (double)part[((size_t)b * h + k) * npad + e];
        red[(size_t)k * npad + e] = s;
    } else if (dlam) {
        const T *lp = part + (size_t)nblocks * h * npad;
        for (int b = 0; b < nblocks; ++b) s += (double)lp[(size_t)b * npad + e];
        dlam[e] = (T)s;
    }
}

// -tau_k and the chain rule of the normalisation, one block per reflector:
// dU_k = (I - uh_k uh_k^T) g_k / ||u_k||, g_k = -tau_k * (summed partials).
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_finish(const double *__restrict__ red, int n,
                                                   int npad, const T *__restrict__ tau,
                                                   const double *__restrict__ uh64,
                                                   const double *__restrict__ nrm64,
                                                   T *__restrict__ dU, int64_t lddu) {
    __shared__ double sred[256];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    const double nrm = nrm64[k];
    const double mt = -(double)tau[k];
    const double *g = red + (size_t)k * npad;
    const double *u = uh64 + (size_t)k * n;
    double p = 0.0;
    for (int e = t; e < n; e += 256) p += u[e] * (mt * g[e]);
    sred[t] = p;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sred[t] += sred[t + s];
        __syncthreads();
    }
    p = sred[0];
    for (int e = t; e < n; e += 256) {
        double v = 0.0;
        if (nrm > 0.0) v = (mt * g[e] - p * u[e]) / nrm;
        dU[e + (int64_t)k * lddu] = (T)v;
    }
}

// Vectors per wave: HH_BWD_VPW when a vector takes at most 8 registers per
// lane, else one.
#ifndef HH_BWD_VPW
#define HH_BWD_VPW 4
#endif
template <typename T, int NC> constexpr int vpw_for() {
    return NC * V16<T>::W * (int)(sizeof(T) / 4) <= 8 ? HH_BWD_VPW : 1;
}
int bwd_vpw(const FusedPlan &p) {
    const int regs = p.s.nc * ((p.t == HH_F64) ? 2 : 4) * ((p.t == HH_F64) ? 2 : 1);
    return regs <= 8 ? HH_BWD_VPW : 1;
}

size_t lds_small(hh_op op, const FusedPlan &p) {
    const size_t es = (p.t == HH_F64) ? 8 : 4;
    const size_t R = (op == HH_OP_SYM_BWD) ? 2 * (size_t)p.h : (size_t)p.h;
    return 2 * (size_t)p.s.npad * es + (size_t)kWPB * bwd_vpw(p) * std::max<size_t>(R, 1) * es +
           std::max<size_t>((size_t)p.h, 1) * es;
}
bool refl_in_lds(hh_op op, const FusedPlan &p) {
    const size_t es = (p.t == HH_F64) ? 8 : 4;
    return lds_small(op, p) + (size_t)p.h * p.s.npad * es <= kLdsBudget;
}
size_t lds_bytes_for(hh_op op, const FusedPlan &p) {
    const size_t es = (p.t == HH_F64) ? 8 : 4;
    return lds_small(op, p) + (refl_in_lds(op, p) ? (size_t)p.h * p.s.npad * es : 0);
}

size_t partial_bytes(const FusedPlan &p, int nb) {
    const size_t es = (p.t == HH_F64) ? 8 : 4;
    return align256((size_t)nb * ((size_t)p.h + 1) * p.s.npad * es);
}

int bwd_blocks(const FusedPlan &p) {
    const int64_t vpb = (int64_t)kWPB * bwd_vpw(p);
    const int64_t need = (p.N + vpb - 1) / vpb;
    const int64_t cap = (int64_t)device_cu_count() * 2;
    return (int)std::max<int64_t>(1, std::min(need, cap));
}

template <typename T, int NC, bool UL, int HB, int V>
hipError_t launch_main(hh_op op, const FusedPlan &p, const FusedBwdArgs &a, dim3 grid,
                       size_t lds, int k0, int kcnt, int wdx, int dl, int nb, hipStream_t st) {
    switch (op) {
    case HH_OP_APPLY_BWD:
        hipLaunchKernelGGL((k_fused_bwd<T, NC, B_APPLY, UL, HB, V>), grid, dim3(kThreads), lds, st, a, k0,
                           kcnt, wdx, dl, nb);
        break;
    case HH_OP_APPLY_T_BWD:
        hipLaunchKernelGGL((k_fused_bwd<T, NC, B_APPLY_T, UL, HB, V>), grid, dim3(kThreads), lds, st, a, k0,
                           kcnt, wdx, dl, nb);
        break;
    case HH_OP_SYM_BWD:
        hipLaunchKernelGGL((k_fused_bwd<T, NC, B_SYM, UL, HB, V>), grid, dim3(kThreads), lds, st, a, k0,
                           kcnt, wdx, dl, nb);
        break;
    default:
        hipLaunchKernelGGL((k_fused_bwd<T, NC, B_MAHAL, UL, HB, V>), grid, dim3(kThreads), lds, st, a, k0,
                           kcnt, wdx, dl, nb);
        break;
    }
    return hipGetLastError();
}

// ULO: only the form with the reflectors in LDS is instantiated (h <= 10,
// whose reflectors always fit).
template <typename T, int NC, int HB, bool ULO = false>
hipError_t run_bwd_hb(hh_op op, const FusedPlan &p, const FusedBwdArgs &a, hipStream_t st) {
    constexpr int V = vpw_for<T, NC>();
    const int nb = bwd_blocks(p);
    const size_t lds = lds_bytes_for(op, p);
    const dim3 grid(nb);
    const int h = (int)p.h;
    const bool ul = refl_in_lds(op, p);
    auto go = [&](int k0, int cnt, int wdx, int dl) {
        if constexpr (ULO) return launch_main<T, NC, true, HB, V>(op, p, a, grid, lds, k0, cnt, wdx, dl, nb, st);
        else
            return ul ? launch_main<T, NC, true, HB, V>(op, p, a, grid, lds, k0, cnt, wdx, dl, nb, st)
                      : launch_main<T, NC, false, HB, V>(op, p, a, grid, lds, k0, cnt, wdx, dl, nb, st);
    };
    if (!a.dU || h == 0) {
        hipError_t e = go(0, 0, 1, 1);
        if (e != hipSuccess) return e;
    } else {
        for (int k0 = 0; k0 < h; k0 += HB) {
            const int cnt = std::min(HB, h - k0);
            hipError_t e = go(k0, cnt, k0 + HB >= h, k0 == 0);
            if (e != hipSuccess) return e;
        }
    }
    const bool has_lam = (op == HH_OP_SYM_BWD || op == HH_OP_MAHAL_BWD) && a.dlam;
    const bool has_u = a.dU && h > 0;
    if (has_u || has_lam) {
        double *red = reinterpret_cast<double *>(static_cast<char *>(a.scratch) +
                                                 partial_bytes(p, nb));
        const dim3 rgrid((a.n + 255) / 256, has_u ? h + 1 : 1);
        // with no dU wanted the single grid row handles the spectrum (k = h)
        hipLaunchKernelGGL((k_bwd_reduce<T>), rgrid, dim3(256), 0, st,
                           static_cast<const T *>(a.scratch), nb, a.n, h, a.npad,
                           has_u ? 0 : h, red, has_lam ? static_cast<T *>(a.dlam) : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (has_u) {
        double *red = reinterpret_cast<double *>(static_cast<char *>(a.scratch) +
                                                 partial_bytes(p, nb));
        hipLaunchKernelGGL((k_bwd_finish<T>), dim3(h), dim3(256), 0, st, red, a.n, a.npad,
                           static_cast<const T *>(a.tau), a.uh64, a.nrm64,
                           static_cast<T *>(a.dU), a.lddu);
        return hipGetLastError();
    }
    return hipSuccess;
}

// Accumulator window: 10 slots when h <= 10 (the reflectors then always fit
// in LDS) and the registers allow 16, else what the registers allow.
template <typename T, int NC>
hipError_t run_bwd(hh_op op, const FusedPlan &p, const FusedBwdArgs &a, hipStream_t st) {
    constexpr int HBM = hb_for<T, NC>();
    if constexpr (HBM >= 16) {
        if (p.h <= 10 && refl_in_lds(op, p)) return run_bwd_hb<T, NC, 10, true>(op, p, a, st);
        return run_bwd_hb<T, NC, 16>(op, p, a, st);
    } else {
        return run_bwd_hb<T, NC, HBM>(op, p, a, st);
    }
}

template <typename T>
hipError_t dispatch_nc(hh_op op, const FusedPlan &p, const FusedBwdArgs &a, hipStream_t st) {
    switch (p.s.nc) {
    case 1: return run_bwd<T, 1>(op, p, a, st);
    case 2: return run_bwd<T, 2>(op, p, a, st);
    case 4: return run_bwd<T, 4>(op, p, a, st);
    case 8: return run_bwd<T, 8>(op, p, a, st);
    case 16: return run_bwd<T, 16>(op, p, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool fused_bwd_plan(hh_dtype t, int64_t n, int64_t h, int64_t N, FusedPlan *p) {
    const int W = (t == HH_F64) ? 2 : 4;
    int nc = 1;
    while ((int64_t)nc * 64 * W < n) nc <<= 1;
    if (nc > 16) return false;
    p->t = t;
    p->n = n;
    p->h = h;
    p->N = N;
    p->s.lpv = 64;
    p->s.nc = nc;
    p->s.npad = nc * 64 * W;
    p->hc = (int)h;
    p->lds_bytes = 0;
    return true;
}

bool fused_bwd_supported(hh_op op, const FusedPlan &p) {
    return p.s.lpv == 64 && p.s.nc <= 16 && lds_bytes_for(op, p) <= kLdsBudget;
}

size_t fused_bwd_ws_bytes(hh_op op, const FusedPlan &p) {
    (void)op;
    return partial_bytes(p, bwd_blocks(p)) + align256(((size_t)p.h + 1) * p.s.npad * 8);
}

hipError_t launch_fused_bwd(const FusedPlan &p, hh_op op, const FusedBwdArgs &a,
                            hipStream_t st) {
    if (p.t == HH_F32) return dispatch_nc<float>(op, p, a, st);
    return dispatch_nc<double>(op, p, a, st);
}

}  // namespace hh

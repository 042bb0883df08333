// Fused sequential-reflector kernels (forward): Q X, Q^T X, Q diag(lam) Q^T X
// and the Mahalanobis distance, in FP32 or FP64.
//
// Each vector is applied the reflectors one after another (paper Sec. II-A:
// a dot product and an update per reflector, 4n operations; Sec. III-A:
// (8h+1)n for the symmetric form).  The vector never leaves the registers
// between its single HBM read and its single HBM write.
//
// Mapping: a group of LPV lanes (16 or 64) owns VPL vectors; lane c holds
// NC 16-byte chunks of each at element offsets i*LPV*W + c*W (W = 4 floats or
// 2 doubles), so every load and store instruction moves LPV*16 contiguous
// bytes per vector.  A dot product is a per-lane partial sum followed by a
// DPP reduction across the LPV lanes (no LDS round trip).  Reflectors (and the
// spectrum) are staged in LDS, all at once when they fit, otherwise in chunks
// of hc reflectors that every wave of the block walks through in lockstep;
// each chunk of a reflector read from LDS serves the VPL vectors of the group.
// A reflector whose first nonzero entry lies past whole chunks (reflectors of
// a Householder QR have k - 1 leading zeros, the remark after Result 3) skips
// those chunks in its dot product and update: 4(n - k + 1) operations instead
// of 4n, with the same result (the skipped terms are exact zeros).  The
// distance kernel can also write each pair's h dot products (a record the
// backward reads instead of forming them again).
#include <algorithm>
#include <type_traits>

#include "hh_internal.h"

namespace hh {
namespace {

constexpr size_t kLdsBudget = 64 * 1024;       // several blocks per compute unit
constexpr size_t kLdsBudgetWide = 144 * 1024;  // one 8-wave block per compute unit

template <typename T, int LPV, int NC, int OP, int VPL, int WPB, bool SKIP>
__global__ __launch_bounds__(WPB * kWave) void k_fused_fwd(FusedFwdArgs a) {
    using VT = typename V16<T>::type;
    constexpr int W = V16<T>::W;
    constexpr int E = NC * W;      // elements per lane and vector
    constexpr int VPW = kWave / LPV;
    constexpr int STR = LPV * W;   // element stride between a lane's chunks
    constexpr int kThreads = WPB * kWave;
    extern __shared__ __align__(16) unsigned char smem[];

    const int n = a.n, h = a.h, npad = a.npad, hc = a.hc;
    T *sU = reinterpret_cast<T *>(smem);
    T *sLam = sU + (size_t)hc * npad;
    T *sDin = sLam + npad;                         // diagonal on the input (if given)
    T *sDout = sDin + (a.din ? npad : 0);          // diagonal on the output (if given)
    T *sTau = sDout + (a.dout ? npad : 0);         // tau of the reflectors of the current chunk
    int *sLead = reinterpret_cast<int *>(sTau + hc);  // leading zero chunks (SKIP)
    const T *gU = static_cast<const T *>(a.ut);
    const T *gTau = static_cast<const T *>(a.tau);

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int c = lane % LPV;
    const int row = lane / LPV;

    if constexpr (OP == F_SYM || OP == F_MAHAL) {
        const VT *src = static_cast<const VT *>(a.lam);
        for (int i = tid; i < npad / W; i += kThreads) reinterpret_cast<VT *>(sLam)[i] = src[i];
    }
    // the caller's diagonals hold n entries (no padding, no alignment assumed)
    auto stage_diag = [&](T *dst, const void *src) {
        const T *d = static_cast<const T *>(src);
        for (int i = tid; i < npad; i += kThreads) dst[i] = i < n ? d[i] : (T)0;
    };
    if (a.din) stage_diag(sDin, a.din);
    if (a.dout) stage_diag(sDout, a.dout);
    __syncthreads();

    const int nchunks = h > 0 ? (h + hc - 1) / hc : 0;
    // copy `total` 16-byte pieces (piece i at offset at(i) in both) from the
    // reflectors in memory to LDS, four loads of a thread in flight before
    // their stores (a chunk is re-staged for every batch of vectors)
    auto stage_pieces = [&](VT *dst, const VT *src, int total, auto at) {
        int i = tid;
        for (; i + 3 * kThreads < total; i += 4 * kThreads) {
            VT v[4];
            int o[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                o[u] = at(i + u * kThreads);
                v[u] = src[o[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[o[u]] = v[u];
        }
        for (; i < total; i += kThreads) {
            const int oi = at(i);
            dst[oi] = src[oi];
        }
    };
    int loaded = -1;      // block-uniform
    int chunk_skip = 0;   // block-uniform: leading zero chunks shared by every reflector of the loaded chunk
    auto load_chunk = [&](int q) {
        if (q == loaded) return;
        __syncthreads();
        const int k0 = q * hc;
        const int cnt = min(hc, h - k0);
        const VT *src = reinterpret_cast<const VT *>(gU + (size_t)k0 * npad);
        VT *dst = reinterpret_cast<VT *>(sU);
        if constexpr (SKIP) {
            // the fewest leading zero chunks over the chunk's reflectors
            // (QR reflectors: k - 1 leading zeros, so this changes slowly);
            // those chunks are neither staged nor read
            if (tid == 0) sLead[0] = NC;
            __syncthreads();
            int mn = NC;
            for (int i = tid; i < cnt; i += kThreads) {
                sTau[i] = gTau[k0 + i];
                mn = min(mn, a.lead[k0 + i] / STR);
            }
            if (mn < NC) atomicMin(&sLead[0], mn);
            __syncthreads();
            // in steps of G chunks, at most eight loop variants (run_chunk)
            constexpr int NV = NC < 8 ? NC : 8;
            constexpr int G = NC / NV;
            chunk_skip = min(sLead[0] / G, NV - 1) * G;
            const int off = chunk_skip * (STR / W);  // skipped 16-byte pieces per reflector
            const int per = npad / W - off;
            stage_pieces(dst, src, cnt * per, [&](int i) {
                const int r = i / per;
                return r * (npad / W) + off + (i - r * per);
            });
            __syncthreads();
        } else {
            stage_pieces(dst, src, cnt * (npad / W), [](int i) { return i; });
            for (int i = tid; i < cnt; i += kThreads) sTau[i] = gTau[k0 + i];
            __syncthreads();
        }
        loaded = q;
    };
    if (nchunks == 1) load_chunk(0);
    // Record of the distance's dot products: row j (hp = h rounded up to 16
    // bytes, the padding zero) holds pair j's.  Each wave stages its vectors'
    // dot products of the current reflector chunk in LDS (rows of hcp values),
    // then writes them with consecutive lanes: whole padded rows at once when
    // one chunk holds all h reflectors, so that the rows of a batch step cover
    // whole cache lines (partial-line writes are costly).
    constexpr int RW = 16 / (int)sizeof(T);
    const int hp = (h + RW - 1) / RW * RW, hcp = (hc + RW - 1) / RW * RW;
    constexpr int NVW = VPW * VPL;  // vectors of a wave
    // (an offset from smem, 16-byte aligned: arithmetic on the LDS base keeps
    // the accesses ds_read / ds_write instead of generic flat ones)
    const int dots_off = ((int)(reinterpret_cast<unsigned char *>(sLead + hc) - smem) + 15) & ~15;
    T *sDots = reinterpret_cast<T *>(smem + dots_off);
    if constexpr (OP == F_MAHAL)
        if (a.dots)  // the padding slots stay zero
            for (int i = lane; i < NVW * hcp; i += kWave) sDots[wave * NVW * hcp + i] = (T)0;
    int64_t jwave = 0;  // first vector of the wave in the current batch step
    // rows jw .. jw + NVW - 1, reflectors kb .. ke - 1 of the record
    auto flush_dots = [&](int64_t jw, int kb, int ke) {
        const int cnt = ke - kb;
        T *dst = static_cast<T *>(a.dots);
        if (cnt == h && jw + NVW <= a.N) {  // whole padded rows: a straight copy
            for (int l = lane; l < NVW * hp; l += kWave) dst[jw * hp + l] = sDots[wave * NVW * hp + l];
            return;
        }
        const int wid = ke == h ? hp - kb : cnt;  // the last chunk also writes the row's padding
        for (int l = lane; l < NVW * wid; l += kWave) {
            const int vi = l / wid, kk = l % wid;
            const int64_t j = jw + vi;
            if (j < a.N) dst[j * hp + kb + kk] = kk < cnt ? sDots[(wave * NVW + vi) * hcp + kk] : (T)0;
        }
    };
    // With all h reflectors in one chunk, a batch step's dot products wait in
    // LDS and are written after the next step's loads are issued (vector-memory
    // counters retire in issue order: stores issued before those loads would
    // hold up the wait for them); else each chunk's are written at once.
    int64_t jprev = -1;

    // One reflection of the lane's slices of its VPL vectors by reflector k,
    // over chunks S .. NC-1 (S = 0: the whole vector).
    auto reflect_from = [&](auto S0, int k, T(&x)[VPL][E]) {
        constexpr int S = decltype(S0)::value;
        const T *u = sU + (size_t)(k - loaded * hc) * npad + c * W;
        VT uv[NC];
#pragma unroll
        for (int i = S; i < NC; ++i) uv[i] = *reinterpret_cast<const VT *>(u + i * STR);
        const T tk = sTau[k - loaded * hc];
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            T part[W];
#pragma unroll
            for (int q = 0; q < W; ++q) part[q] = (T)0;
#pragma unroll
            for (int i = S; i < NC; ++i)
#pragma unroll
                for (int q = 0; q < W; ++q) part[q] = fmat(uv[i][q], x[v][i * W + q], part[q]);
            T p = part[0];
#pragma unroll
            for (int q = 1; q < W; ++q) p += part[q];
            p = group_sum<LPV>(p);
            if constexpr (OP == F_MAHAL)
                if (a.dots && c == 0) sDots[((wave * VPW + row) * VPL + v) * hcp + (k - loaded * hc)] = p;
            const T coef = -p * tk;
#pragma unroll
            for (int i = S; i < NC; ++i)
#pragma unroll
                for (int q = 0; q < W; ++q) x[v][i * W + q] = fmat(coef, uv[i][q], x[v][i * W + q]);
        }
    };
    // The reflectors of a chunk that all start past chunk S of every lane's
    // slice (S = chunk_skip, a multiple of G): one scalar dispatch per LDS
    // chunk to the loop that leaves out chunks 0 .. S-1 (at most eight
    // variants).
    auto run_chunk = [&](int kb, int ke, int step, T(&x)[VPL][E]) {
        auto loop = [&](auto S0) {
#pragma unroll 1
            for (int k = kb; k != ke; k += step) reflect_from(S0, k, x);
        };
        if constexpr (SKIP) {
            constexpr int NV = NC < 8 ? NC : 8;
            constexpr int G = NC / NV;
            const int sv = __builtin_amdgcn_readfirstlane(chunk_skip) / G;
            static_for<NV>([&](auto cc) {
                if (sv == decltype(cc)::value) loop(std::integral_constant<int, decltype(cc)::value * G>{});
            });
        } else {
            loop(std::integral_constant<int, 0>{});
        }
    };
    // x <- diag(d) x on the lane's slices (d staged in LDS like the spectrum)
    auto scale = [&](T(&x)[VPL][E], const T *sd) {
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            VT l = *reinterpret_cast<const VT *>(sd + i * STR + c * W);
#pragma unroll
            for (int v = 0; v < VPL; ++v)
#pragma unroll
                for (int q = 0; q < W; ++q) x[v][i * W + q] *= l[q];
        }
    };
    auto run_up = [&](T(&x)[VPL][E]) {  // k = 0 .. h-1  (Q^T: H_1 first)
#pragma unroll 1
        for (int q = 0; q < nchunks; ++q) {
            load_chunk(q);
            const int kend = min(h, (q + 1) * hc);
            run_chunk(q * hc, kend, 1, x);
            if constexpr (OP == F_MAHAL)
                if (a.dots && nchunks > 1) flush_dots(jwave, q * hc, kend);
        }
    };
    auto run_down = [&](T(&x)[VPL][E]) {  // k = h-1 .. 0  (Q: H_h first)
#pragma unroll 1
        for (int q = nchunks - 1; q >= 0; --q) {
            load_chunk(q);
            const int kend = min(h, (q + 1) * hc);
            run_chunk(kend - 1, q * hc - 1, -1, x);
        }
    };
    auto load_vec = [&](T(&x)[E], const T *base, int64_t ld, int64_t j, bool valid) {
        if (a.vec_ok) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const int e0 = i * STR + c * W;
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
                    const int e = i * STR + c * W + q;
                    x[i * W + q] = (valid && e < n) ? base[j * ld + e] : (T)0;
                }
        }
    };
    auto store_vec = [&](const T(&x)[E], T *base, int64_t ld, int64_t j, bool valid) {
        if (!valid) return;
        if (a.vec_ok) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const int e0 = i * STR + c * W;
                if (e0 < n) {
                    VT v;
#pragma unroll
                    for (int q = 0; q < W; ++q) v[q] = x[i * W + q];
                    *reinterpret_cast<VT *>(base + j * ld + e0) = v;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const int e = i * STR + c * W + q;
                    if (e < n) base[j * ld + e] = x[i * W + q];
                }
        }
    };

    const int64_t vpb = (int64_t)WPB * VPW * VPL;
    const int64_t gstride = (int64_t)gridDim.x * vpb;
    const int64_t joff = (int64_t)(wave * VPW + row) * VPL;
    for (int64_t b0 = (int64_t)blockIdx.x * vpb; b0 < a.N; b0 += gstride) {
        const int64_t j0 = b0 + joff;
        jwave = b0 + (int64_t)wave * VPW * VPL;
        T x[VPL][E];
#pragma unroll
        for (int v = 0; v < VPL; ++v) load_vec(x[v], static_cast<const T *>(a.X), a.ldx, j0 + v, j0 + v < a.N);
        if constexpr (OP == F_MAHAL && VPL == 1) {
            T xb[E];
            load_vec(xb, static_cast<const T *>(a.Xb), a.ldb, j0, j0 < a.N);
            if (a.dots && nchunks == 1 && jprev >= 0) flush_dots(jprev, 0, h);  // behind this step's loads
#pragma unroll
            for (int e = 0; e < E; ++e) x[0][e] -= xb[e];
        } else if constexpr (OP == F_MAHAL) {
            if (a.dots && nchunks == 1 && jprev >= 0) flush_dots(jprev, 0, h);
            // x - xb one 16-byte chunk at a time (keeps the second input's
            // registers to one chunk when a lane holds two vectors)
            const T *Xb = static_cast<const T *>(a.Xb);
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const int64_t j = j0 + v;
                const bool valid = j < a.N;
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    const int e0 = i * STR + c * W;
                    if (a.vec_ok) {
                        VT b = {};
                        if (valid && e0 < n) b = *reinterpret_cast<const VT *>(Xb + j * a.ldb + e0);
#pragma unroll
                        for (int q = 0; q < W; ++q) x[v][i * W + q] -= b[q];
                    } else {
#pragma unroll
                        for (int q = 0; q < W; ++q)
                            if (valid && e0 + q < n) x[v][i * W + q] -= Xb[j * a.ldb + e0 + q];
                    }
                }
            }
        }
        if (a.din) scale(x, sDin);
        if constexpr (OP == F_APPLY) run_down(x);
        if constexpr (OP == F_APPLY_T || OP == F_SYM || OP == F_MAHAL) run_up(x);
        if constexpr (OP == F_MAHAL)
            if (a.dots && nchunks == 1) jprev = jwave;
        if constexpr (OP == F_SYM) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                VT l = *reinterpret_cast<const VT *>(sLam + i * STR + c * W);
#pragma unroll
                for (int v = 0; v < VPL; ++v)
#pragma unroll
                    for (int q = 0; q < W; ++q) x[v][i * W + q] *= l[q];
            }
            run_down(x);
        }
        if constexpr (OP != F_MAHAL)
            if (a.dout) scale(x, sDout);
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const int64_t j = j0 + v;
            const bool valid = j < a.N;
            if constexpr (OP == F_MAHAL) {
                T part = (T)0;
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    VT l = *reinterpret_cast<const VT *>(sLam + i * STR + c * W);
#pragma unroll
                    for (int q = 0; q < W; ++q) part = fmat(l[q] * x[v][i * W + q], x[v][i * W + q], part);
                }
                part = group_sum<LPV>(part);
                if (valid && c == 0) static_cast<T *>(a.Y)[j] = part;
            } else {
                store_vec(x[v], static_cast<T *>(a.Y), a.ldy, j, valid);
            }
        }
    }
    if constexpr (OP == F_MAHAL)
        if (a.dots && nchunks == 1 && jprev >= 0) flush_dots(jprev, 0, h);
}

template <typename T, int LPV, int NC, int VPL, int WPB, bool SKIP>
hipError_t launch_op_s(FusedOp op, const FusedPlan &p, const FusedFwdArgs &a, dim3 grid,
                       hipStream_t st) {
    const dim3 block(WPB * kWave);
    switch (op) {
    case F_APPLY:
        hipLaunchKernelGGL((k_fused_fwd<T, LPV, NC, F_APPLY, VPL, WPB, SKIP>), grid, block, p.lds_bytes, st, a);
        break;
    case F_APPLY_T:
        hipLaunchKernelGGL((k_fused_fwd<T, LPV, NC, F_APPLY_T, VPL, WPB, SKIP>), grid, block, p.lds_bytes, st, a);
        break;
    case F_SYM:
        hipLaunchKernelGGL((k_fused_fwd<T, LPV, NC, F_SYM, VPL, WPB, SKIP>), grid, block, p.lds_bytes, st, a);
        break;
    case F_MAHAL: {
        // the dot-product staging of the record: hc values per vector of the block, 16-byte aligned
        constexpr size_t es = sizeof(T);
        const size_t rw = 16 / es, hcp = (p.hc + rw - 1) / rw * rw;
        const size_t stage = a.dots ? 16 + (size_t)WPB * (kWave / LPV) * VPL * hcp * es : 0;
        hipLaunchKernelGGL((k_fused_fwd<T, LPV, NC, F_MAHAL, VPL, WPB, SKIP>), grid, block, p.lds_bytes + stage, st,
                           a);
        break;
    }
    }
    return hipGetLastError();
}

// skip: the kernels that leave out each reflector's leading zero chunks
// (HH_ALGO_FUSED_QR); the others treat every reflector as dense.
template <typename T, int LPV, int NC, int VPL = 1, int WPB = 4>
hipError_t launch_op(FusedOp op, const FusedPlan &p, const FusedFwdArgs &a, dim3 grid,
                     hipStream_t st) {
    return a.skip_zeros ? launch_op_s<T, LPV, NC, VPL, WPB, true>(op, p, a, grid, st)
                        : launch_op_s<T, LPV, NC, VPL, WPB, false>(op, p, a, grid, st);
}

template <typename T>
hipError_t dispatch(FusedOp op, const FusedPlan &p, const FusedFwdArgs &a, dim3 grid,
                    hipStream_t st) {
    const int lpv = p.s.lpv, nc = p.s.nc;
    if (lpv == 16) {
        switch (nc) {
        case 1: return launch_op<T, 16, 1>(op, p, a, grid, st);
        case 2: return launch_op<T, 16, 2>(op, p, a, grid, st);
        case 4: return launch_op<T, 16, 4>(op, p, a, grid, st);
        case 8:
            if constexpr (std::is_same_v<T, float>)
                if (p.s.vpl == 2) return launch_op<T, 16, 8, 2, 8>(op, p, a, grid, st);
            return launch_op<T, 16, 8>(op, p, a, grid, st);
        case 16:
            if constexpr (std::is_same_v<T, float>)
                if (p.s.vpl == 2) return launch_op<T, 16, 16, 2, 4>(op, p, a, grid, st);
            return launch_op<T, 16, 16>(op, p, a, grid, st);
        }
    } else if (lpv == 64) {
        switch (nc) {
        case 8: return launch_op<T, 64, 8, 2, 8>(op, p, a, grid, st);
        case 16: return launch_op<T, 64, 16, 2, 8>(op, p, a, grid, st);
        case 32: return launch_op<T, 64, 32>(op, p, a, grid, st);
        }
    }
    return hipErrorInvalidValue;
}

int next_pow2(int64_t v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

bool fused_shape(hh_dtype t, int64_t n, FusedShape *s) {
    const int W = (t == HH_F64) ? 2 : 4;
    s->vpl = 1;
    s->wpb = 4;
    if (t == HH_F32 && n > 16 * W * 8 && n <= 16 * W * 16) {
        // 512 < n <= 1024: each 16-lane row holds two vectors, so each
        // reflector chunk read from LDS serves two vectors and a dot product
        // needs only the four DPP steps of one row (this size is bound by
        // VALU issue, and the 32-lane layout spent a further four
        // instructions per reduction)
        s->lpv = 16;
        s->nc = 16;
        s->vpl = 2;
    } else if (n <= 16 * W * 16) {
        s->lpv = 16;
        s->nc = next_pow2((n + 16 * W - 1) / (16 * W));
    } else if (n <= 64 * W * 32) {
        s->lpv = 64;
        s->nc = std::max(8, next_pow2((n + 64 * W - 1) / (64 * W)));
        if (s->nc <= 16) {
            // two vectors per wave and 8-wave blocks: each reflector chunk
            // staged in LDS (up to 144 KB, one block per compute unit) serves
            // 16 vectors
            s->vpl = 2;
            s->wpb = 8;
        }
    } else {
        return false;
    }
    s->npad = s->nc * s->lpv * W;
    return true;
}

bool fused_plan(hh_dtype t, int64_t n, int64_t h, int64_t N, FusedPlan *p, int ndiag) {
    p->t = t;
    p->n = n;
    p->h = h;
    p->N = N;
    if (!fused_shape(t, n, &p->s)) return false;
    const size_t es = (t == HH_F64) ? 8 : 4;
    const size_t vec_bytes = (size_t)p->s.npad * es;
    const size_t fixed = vec_bytes * (1 + (size_t)ndiag);  // spectrum and the diagonals
    size_t budget = p->s.wpb == 8 ? kLdsBudgetWide : kLdsBudget;
    // with diagonals, a large n runs with fewer blocks per compute unit
    if (ndiag > 0 && fixed + vec_bytes > budget) budget = kLdsBudgetWide;
    if (fixed + vec_bytes > budget) return false;
    int64_t fit = (int64_t)((budget - fixed) / vec_bytes);
    if (t == HH_F32 && p->s.lpv == 16 && p->s.nc == 8 && p->s.vpl == 1 && h > fit) {
        // more reflectors than one staging (e.g. QR's h = n - 1): every batch
        // of vectors stages them all again, so 8-wave blocks with two vectors
        // per lane group let each staged chunk (144 KB) serve 64 vectors
        // instead of 16 (the distance kernel's record staging is fitted
        // beside it by fused_plan_fit_record)
        p->s.vpl = 2;
        p->s.wpb = 8;
        budget = kLdsBudgetWide;
        fit = (int64_t)((budget - fixed) / vec_bytes);
    }
    p->hc = (int)std::max<int64_t>(1, std::min<int64_t>(h, fit));
    // reflectors, their tau and their leading zero chunk counts
    p->lds_bytes = fixed + (size_t)p->hc * (vec_bytes + es + sizeof(int));
    return true;
}

void fused_plan_fit_record(FusedPlan *p) {
    // the distance kernel's record staging: hc values (padded to 16 bytes)
    // per vector of the block, beside the plan's LDS, within 160 KB
    constexpr size_t kLdsMax = 160 * 1024;
    const size_t es = p->t == HH_F64 ? 8 : 4, rw = 16 / es;
    const size_t vpb = (size_t)p->s.wpb * (kWave / p->s.lpv) * p->s.vpl;
    const size_t per = (size_t)p->s.npad * es + es + sizeof(int);  // one staged reflector
    const size_t fixed = p->lds_bytes - (size_t)p->hc * per;
    while (p->hc > 1) {
        const size_t hcp = ((size_t)p->hc + rw - 1) / rw * rw;
        if (p->lds_bytes + 16 + vpb * hcp * es <= kLdsMax) break;
        --p->hc;
        p->lds_bytes = fixed + (size_t)p->hc * per;
    }
}

hipError_t launch_fused_fwd(const FusedPlan &p, FusedOp op, const FusedFwdArgs &a,
                            hipStream_t st) {
    const int vpb = p.s.wpb * (kWave / p.s.lpv) * p.s.vpl;
    const int64_t need = (p.N + vpb - 1) / vpb;
    // a grid-stride loop over at most 8 blocks per compute unit
    const int64_t cap = (int64_t)device_cu_count() * 8;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min(need, cap)));
    if (p.t == HH_F32) return dispatch<float>(op, p, a, grid, st);
    return dispatch<double>(op, p, a, grid, st);
}

}  // namespace hh

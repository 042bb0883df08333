// Internal declarations shared by the compact-WY translation units.
#pragma once

#include "hh_wy.h"

namespace hh {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));


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
// Fragment-ordered copies of the reflector matrix.  Every operand load of the
// main kernel then reads one contiguous 1 KB block (64 lanes x 16 bytes).
//   Yc (GEMM1 A operand, lane = (c, g)): element (h, row) with
//     h = 16 hb + c, row = 32 q + 8 g + j  at  ((hb * NQ + q) * 64 + 16 g + c) * 8 + j
//   Yr (GEMM2 A operand): element (h, row) with row = 32 q + 8 (c/4) + 4 m + c%4,
//     h = 32 ks + 8 g + j  at  (((q * 2 + m) * KS + ks) * 64 + 16 g + c) * 8 + j
// with NQ = npad / 32 and KS = hp / 32.
__device__ __forceinline__ int64_t yc_index(int h, int row, int npad) {
    const int hb = h >> 4, c = h & 15, q = row >> 5, g = (row >> 3) & 3, j = row & 7;
    return ((int64_t)(hb * (npad >> 5) + q) * 64 + 16 * g + c) * 8 + j;
}
__device__ __forceinline__ int64_t yr_index(int h, int row, int hp) {
    const int q = row >> 5, rr = row & 31;
    const int c = 4 * (rr >> 3) + (rr & 3), m = (rr >> 2) & 1;
    const int ks = h >> 5, g = (h >> 3) & 3, j = h & 7;
    return ((int64_t)((q * 2 + m) * (hp >> 5) + ks) * 64 + 16 * g + c) * 8 + j;
}

// Copy read by the streaming kernel's GEMM1 (chunk-major, permuted h):
// fragment (q, hb) holds, for lane (c, g), the 8 rows 32q + 8g + j of
// reflector h = 32(hb/2) + 8(c/4) + 4(hb%2) + c%4, at
//   ((q * HB + hb) * 64 + 16 g + c) * 8 + j,   HB = hp / 16.
__device__ __forceinline__ int64_t ycs_index(int h, int row, int hp) {
    const int hb = 2 * (h >> 5) + ((h >> 2) & 1), c = 4 * ((h >> 3) & 3) + (h & 3);
    const int q = row >> 5, g = (row >> 3) & 3, j = row & 7;
    return ((int64_t)(q * (hp >> 4) + hb) * 64 + 16 * g + c) * 8 + j;
}
// Row permutation of a 16-row MFMA block b used by the streaming kernel.
__device__ __forceinline__ int sigma_row(int b, int r) {
    return 32 * (b >> 1) + 8 * (r >> 2) + 4 * (b & 1) + (r & 3);
}

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
// Forces v to be materialised here (an empty asm that reads and writes it),
// so the optimiser cannot sink its computation towards a distant use.
template <typename V> __device__ __forceinline__ void pin(V &v) { asm volatile("" : "+v"(v)); }

template <typename V>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, V v, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, v), r, voff, soff, 0);
}

struct WyArgs {
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    const void *Yc;   // HP x npad, column-major reflectors (GEMM1 A operand)
    const void *Yr;   // npad x HP, row-major reflectors (GEMM2 A operand)
    const void *Ycs;  // streaming kernel: GEMM1 operand, chunk-major (ycs_index)
    const void *Tf;   // streaming kernel: T and T^T as 16-bit hi/lo MFMA fragments
    const void *Mf;   // streaming kernel, SYM: Y^T diag(lam) Y as hi/lo fragments
    const float *lam; // npad (SYM)
    void *coef;       // nullable: W' of pass q written to rows [q*HP, (q+1)*HP), ld = ldc
    int64_t ldc;
    int store;        // 0: skip the last product and the stores (coefficients only)
    int n, npad;
    int64_t N;
};

// Tile shape of the main kernel: HP padded reflector count, P row groups of
// 32 per wave (npad = 256 P), CB column blocks of 16 vectors per tile.
struct WyShape {
    int hp, p, cb, npad;
};

inline bool wy_shape(int64_t n, int64_t h, WyShape *s) {
    if (h > 128 || n > 8192) return false;
    s->hp = h <= 64 ? 64 : 128;
    s->p = n <= 1024 ? 4 : (n <= 4096 ? 16 : 32);
    s->cb = (s->p == 32 || s->hp == 128) ? 1 : 2;
    s->npad = 256 * s->p;
    return true;
}

// Row segments of the partial Gram matrices (npad / 32 is a multiple of it).
constexpr int kGramSeg = 16;

// Columns of a 16-bit coefficient row: N rounded up to 32 (at least 32); the
// columns past N are zero.
inline int64_t wy_ldc(int64_t N) { return N <= 32 ? 32 : (N + 31) / 32 * 32; }

// Workspace of the WY path.  With lam (Q diag(lam) Q^T X) the Gram buffers
// hold a second matrix after the first: gram -> [2][kGramSeg][hp][hp]
// partials, gsum -> [2][hp][hp] (Y^T Y, then Y^T diag(lam) Y), and mf holds
// the fragments of the second.
struct WyWs {
    size_t yc, yr, ycs, tf, mf, nrm2, nrmraw, gram, gsum, tw, lam, uh64, total;
};

inline WyWs wy_ws(const WyShape &s, int64_t n, bool with_lam, bool bwd) {
    WyWs w{};
    size_t off = 0;
    const size_t hp = s.hp, np = s.npad;
    w.yc = off;     off += align256(hp * np * 2);
    w.yr = off;     off += align256(hp * np * 2);
    w.ycs = off;    off += align256(hp * np * 2);
    const size_t nm = with_lam ? 2 : 1;
    w.tf = off;     off += align256(4 * hp * hp * 2);
    w.mf = off;     off += with_lam ? align256(2 * hp * hp * 2) : 0;
    w.nrm2 = off;   off += align256(hp * 8);
    w.nrmraw = off; off += align256(hp * 8);
    w.gram = off;   off += align256(nm * kGramSeg * hp * hp * 8);
    w.gsum = off;   off += align256(nm * hp * hp * 8);
    w.tw = off;     off += align256(hp * hp * 8);
    w.lam = off;    off += with_lam ? align256(np * 4) : 0;
    w.uh64 = off;   off += bwd ? align256(hp * (size_t)n * 8) : 0;
    w.total = off;
    return w;
}

// Coefficient record of a forward (hh_forward_save): m = HP (2 HP for the
// symmetric form) 16-bit coefficient rows of ldc = wy_ldc(N) columns, then,
// from a 256-byte aligned offset, the forward's setup laid out as
// wy_ws(s, n, sym, true) (reflector copies, T fragments, the spectrum and the
// FP64 normalised reflectors the backward's chain rule needs).
struct WyRecord {
    int m;
    int64_t ldc;
    size_t setup, total;
};
inline WyRecord wy_record(const WyShape &s, int64_t n, int64_t N, bool sym) {
    WyRecord r{};
    r.m = sym ? 2 * s.hp : s.hp;
    r.ldc = wy_ldc(N);
    r.setup = align256((size_t)r.m * r.ldc * 2);
    r.total = r.setup + wy_ws(s, n, sym, true).total;
    return r;
}

// Launchers defined in hh_wy.hip.
// Setup: normalised reflectors, T; with lam also the padded spectrum and,
// when want_m, the fragments of Y^T diag(lam) Y (streaming symmetric form).
hipError_t wy_setup_any(bool bf, const WyShape &s, const float *U, int64_t ldu, int64_t n,
                        int64_t h, const float *lam, bool want_m, char *ws, const WyWs &w,
                        bool want_uh, hipStream_t st);
// True when wy_main_any runs the streaming kernel for these arguments.
bool wy_stream_selected(const WyShape &s, const WyArgs &a);
hipError_t wy_main_any(bool bf, const WyShape &s, WyOp op, const WyArgs &a, hipStream_t st);

// Defined in hh_wy_stream.hip.
hipError_t wy_stream_any(bool bf, const WyShape &s, WyOp op, const WyArgs &a, hipStream_t st);

// Defined in hh_wy_bwd.hip.
size_t wy_bwd_ws_bytes(hh_op op, const WyShape &s, int64_t n, int64_t N);
// Zeroes columns N .. ldc-1 of m 16-bit coefficient rows (row stride ldc).
hipError_t wy_zero_pad(void *rows, int m, int64_t N, int64_t ldc, hipStream_t st);

}  // namespace hh

// C ABI of libhh.so: argument validation, workspace layout and dispatch.
// Every entry point validates on the host, enqueues on the caller's stream and
// returns; nothing here allocates device memory or synchronises.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "hh_internal.h"
#include "hh_wy.h"
#include "hh_bwd.h"

namespace hh {

static thread_local std::string g_last_error;

hh_status set_error(hh_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}
#define fail set_error

static hh_status hip_fail(hipError_t e, const char *what) {
    return fail(HH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int device_cu_count() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

static size_t dtype_size(hh_dtype t) {
    switch (t) {
    case HH_F64: return 8;
    case HH_F32: return 4;
    case HH_BF16:
    case HH_F16: return 2;
    }
    return 0;
}

// An enum object holding a value outside its enumerators (a caller's bad
// code) must not be read as that enum type: such a load is undefined in C++.
// Codes are read as the int they are stored in and checked before use.
template <typename E> static int raw_code(const E &e) {
    static_assert(sizeof(E) == sizeof(int), "C enums are int-sized");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

static bool valid_dtype(int t) { return t == HH_F64 || t == HH_F32 || t == HH_BF16 || t == HH_F16; }

// True when op is one of the codes in [lo, hi].
static bool op_in(const hh_op &op, int lo, int hi) {
    const int v = raw_code(op);
    return v >= lo && v <= hi;
}

// ---------------------------------------------------------------------------
// Descriptor checks shared by every entry point.
enum class Algo { Fused, WY };

static hh_status check_desc(const hh_desc *d, Algo *algo) {
    if (!d) return fail(HH_ERR_INVALID_ARG, "descriptor is null");
    if (d->n < 1) return fail(HH_ERR_INVALID_ARG, "n = %lld must be >= 1", (long long)d->n);
    if (d->h < 0) return fail(HH_ERR_INVALID_ARG, "h = %lld must be >= 0", (long long)d->h);
    if (d->N < 0) return fail(HH_ERR_INVALID_ARG, "N = %lld must be >= 0", (long long)d->N);
    if (d->n > (int64_t)1 << 30 || d->h > (int64_t)1 << 30)
        return fail(HH_ERR_UNSUPPORTED, "n and h must be < 2^30");
    if (!valid_dtype(raw_code(d->param_dtype)) || !valid_dtype(raw_code(d->io_dtype)) ||
        !valid_dtype(raw_code(d->compute_dtype)))
        return fail(HH_ERR_INVALID_ARG, "unknown dtype code");
    const int ac = raw_code(d->algo);
    if (ac != HH_ALGO_AUTO && ac != HH_ALGO_FUSED && ac != HH_ALGO_WY && ac != HH_ALGO_FUSED_QR)
        return fail(HH_ERR_INVALID_ARG, "unknown algo code");
    hh_algo a = d->algo == HH_ALGO_FUSED_QR ? HH_ALGO_FUSED : d->algo;
    if (a == HH_ALGO_AUTO)
        a = (d->compute_dtype == HH_F64 || d->compute_dtype == HH_F32) ? HH_ALGO_FUSED : HH_ALGO_WY;
    if (a == HH_ALGO_FUSED) {
        if (!(d->compute_dtype == HH_F64 || d->compute_dtype == HH_F32) ||
            d->param_dtype != d->compute_dtype || d->io_dtype != d->compute_dtype)
            return fail(HH_ERR_UNSUPPORTED,
                        "FUSED needs param = io = compute in {F64, F32}");
        *algo = Algo::Fused;
        return HH_OK;
    }
    if (a == HH_ALGO_WY) {
        if (!(d->compute_dtype == HH_BF16 || d->compute_dtype == HH_F16) ||
            d->param_dtype != HH_F32 || (d->io_dtype != d->compute_dtype && d->io_dtype != HH_F32))
            return fail(HH_ERR_UNSUPPORTED,
                        "WY needs compute in {BF16, F16}, param F32 and io = compute or F32");
        *algo = Algo::WY;
        return HH_OK;
    }
    return fail(HH_ERR_INVALID_ARG, "unknown algo code");
}

static hh_status check_ld(const char *name, int64_t ld, int64_t n) {
    if (ld < n) return fail(HH_ERR_INVALID_ARG, "%s = %lld must be >= n = %lld", name, (long long)ld, (long long)n);
    return HH_OK;
}

static hh_status check_ptr(const char *name, const void *p) {
    if (!p) return fail(HH_ERR_INVALID_ARG, "%s must not be null", name);
    return HH_OK;
}

#define HH_TRY(expr)                  \
    do {                              \
        hh_status _s = (expr);        \
        if (_s != HH_OK) return _s;   \
    } while (0)

// ---------------------------------------------------------------------------
// Workspace layout of the fused path.
struct FusedWs {
    size_t ut, tau, lead, lam, uh64, nrm64, bwd, total;
};

static bool is_bwd(hh_op op) { return op >= HH_OP_APPLY_BWD; }
static bool uses_lam(hh_op op) {
    return op == HH_OP_SYM || op == HH_OP_MAHAL || op == HH_OP_SYM_BWD || op == HH_OP_MAHAL_BWD;
}

static FusedWs fused_ws(hh_op op, const FusedPlan &p) {
    const size_t es = dtype_size(p.t);
    const size_t h = (size_t)p.h, npad = (size_t)p.s.npad;
    FusedWs w{};
    size_t off = 0;
    w.ut = off;   off += align256(h * npad * es);
    w.tau = off;  off += align256(std::max<size_t>(h, 1) * es);
    w.lead = off; off += is_bwd(op) ? 0 : align256(std::max<size_t>(h, 1) * 4);
    w.lam = off;  off += uses_lam(op) ? align256(npad * es) : 0;
    w.uh64 = off; off += is_bwd(op) ? align256(h * (size_t)p.n * 8) : 0;
    w.nrm64 = off; off += is_bwd(op) ? align256(std::max<size_t>(h, 1) * 8) : 0;
    w.bwd = off;  off += is_bwd(op) ? fused_bwd_ws_bytes(op, p) : 0;
    w.total = off;
    return w;
}

static hh_status make_fused_plan(const hh_desc *d, FusedPlan *p, int ndiag = 0) {
    if (!fused_plan(d->compute_dtype, d->n, d->h, d->N, p))
        return fail(HH_ERR_UNSUPPORTED,
                    "fused path supports n <= %d for this dtype (n = %lld)",
                    d->compute_dtype == HH_F64 ? 4096 : 8192, (long long)d->n);
    if (ndiag > 0 && !fused_plan(d->compute_dtype, d->n, d->h, d->N, p, ndiag))
        return fail(HH_ERR_UNSUPPORTED,
                    "%d diagonal(s) and the spectrum do not fit in on-chip memory beside a reflector "
                    "(n = %lld)", ndiag, (long long)d->n);
    return HH_OK;
}

static hh_status make_fused_bwd_plan(const hh_desc *d, FusedPlan *p) {
    if (!fused_bwd_plan(d->compute_dtype, d->n, d->h, d->N, p))
        return fail(HH_ERR_UNSUPPORTED,
                    "fused backward supports n <= %d for this dtype (n = %lld)",
                    d->compute_dtype == HH_F64 ? 2048 : 4096, (long long)d->n);
    return HH_OK;
}

static int aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Record of the fused distance: the h dot products of every pair, one row of
// h rounded up to 16 bytes per pair, in the compute type.
static size_t mahal_dots_bytes(const hh_desc *d) {
    const size_t es = dtype_size(d->compute_dtype), rw = 16 / es;
    const size_t hp = ((size_t)d->h + rw - 1) / rw * rw;
    return align256(hp * (size_t)d->N * es);
}

// ---------------------------------------------------------------------------
// Forward entry (all four ops).
static hh_status forward(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                         const void *lam, const void *X, int64_t ldx, const void *Xb,
                         int64_t ldb, void *Y, int64_t ldy, void *ws, size_t ws_bytes,
                         hipStream_t st, void *saved = nullptr, size_t saved_bytes = 0,
                         const void *din = nullptr, const void *dout = nullptr) {
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    const int64_t n = d->n, h = d->h, N = d->N;
    HH_TRY(check_ld("ldu", ldu, h > 0 ? n : 0));
    HH_TRY(check_ld(op == HH_OP_MAHAL ? "lda" : "ldx", ldx, n));
    if (op == HH_OP_MAHAL) HH_TRY(check_ld("ldb", ldb, n));
    else HH_TRY(check_ld("ldy", ldy, n));
    if (op == HH_OP_MAHAL && dout)
        return fail(HH_ERR_INVALID_ARG, "a distance has no output diagonal (d_out must be null)");
    if (algo == Algo::WY) {
        if (din || dout) return fail(HH_ERR_UNSUPPORTED, "diagonals are applied on the fused path only");
        return wy_forward(op, d, U, ldu, lam, X, ldx, Xb, ldb, Y, ldy, saved, saved_bytes, ws,
                          ws_bytes, st);
    }
    if (saved && op != HH_OP_MAHAL)
        return fail(HH_ERR_UNSUPPORTED, "a coefficient record exists on the WY path only");

    FusedPlan p;
    HH_TRY(make_fused_plan(d, &p, (din ? 1 : 0) + (dout ? 1 : 0)));
    if (saved) fused_plan_fit_record(&p);
    const FusedWs w = fused_ws(op, p);
    if (saved && saved_bytes < mahal_dots_bytes(d))
        return fail(HH_ERR_WORKSPACE, "record needs %zu bytes, got %zu", mahal_dots_bytes(d), saved_bytes);
    if (N == 0) return HH_OK;
    if (h > 0) HH_TRY(check_ptr("U", U));
    HH_TRY(check_ptr(op == HH_OP_MAHAL ? "Xa" : "X", X));
    HH_TRY(check_ptr(op == HH_OP_MAHAL ? "dist" : "Y", Y));
    if (op == HH_OP_MAHAL) HH_TRY(check_ptr("Xb", Xb));
    if (uses_lam(op)) HH_TRY(check_ptr("lam", lam));
    if (op != HH_OP_MAHAL && Y == X && ldy != ldx)
        return fail(HH_ERR_INVALID_ARG, "in-place call needs ldy == ldx");
    if (w.total > 0) HH_TRY(check_ptr("ws", ws));
    if (ws_bytes < w.total)
        return fail(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, ws_bytes);

    char *base = static_cast<char *>(ws);
    hipError_t e = launch_setup_fused(p.t, U, ldu, uses_lam(op) ? lam : nullptr, n, h, p.s.npad,
                                      base + w.ut, base + w.tau,
                                      uses_lam(op) ? base + w.lam : nullptr, nullptr, nullptr,
                                      reinterpret_cast<int *>(base + w.lead), st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");

    const size_t es = dtype_size(p.t);
    const int wvec = 16 / (int)es;
    FusedFwdArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.Xb = Xb;
    a.ldb = ldb;
    a.Y = Y;
    a.ldy = ldy;
    a.ut = base + w.ut;
    a.tau = base + w.tau;
    a.lead = reinterpret_cast<const int *>(base + w.lead);
    a.lam = base + w.lam;
    a.din = din;
    a.dout = dout;
    a.n = (int)n;
    a.h = (int)h;
    a.npad = p.s.npad;
    a.hc = p.hc;
    a.N = N;
    bool vec = (n % wvec == 0) && aligned16(X) && (ldx % wvec == 0);
    if (op == HH_OP_MAHAL) vec = vec && aligned16(Xb) && (ldb % wvec == 0);
    else vec = vec && aligned16(Y) && (ldy % wvec == 0);
    a.vec_ok = vec ? 1 : 0;
    a.skip_zeros = d->algo == HH_ALGO_FUSED_QR ? 1 : 0;
    a.dots = saved;
    FusedOp fop = op == HH_OP_APPLY ? F_APPLY : op == HH_OP_APPLY_T ? F_APPLY_T
                : op == HH_OP_SYM ? F_SYM : F_MAHAL;
    e = launch_fused_fwd(p, fop, a, st);
    if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Backward entry (all four ops).
static hh_status backward(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                          const void *lam, const void *X, int64_t ldx, const void *Xb,
                          int64_t ldb, const void *G, int64_t ldg, void *dX, void *dXb,
                          int64_t lddx, void *dU, int64_t lddu, void *dlam, void *ws,
                          size_t ws_bytes, hipStream_t st, const void *saved = nullptr,
                          size_t saved_bytes = 0, const void *din = nullptr,
                          const void *dout = nullptr) {
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    const int64_t n = d->n, h = d->h, N = d->N;
    HH_TRY(check_ld("ldu", ldu, h > 0 ? n : 0));
    HH_TRY(check_ld(op == HH_OP_MAHAL_BWD ? "lda" : "ldx", ldx, n));
    if (op == HH_OP_MAHAL_BWD) HH_TRY(check_ld("ldb", ldb, n));
    else HH_TRY(check_ld("lddy", ldg, n));
    if (dX || dXb) HH_TRY(check_ld("lddx", lddx, n));
    if (dU && h > 0) HH_TRY(check_ld("lddu", lddu, n));
    if (op == HH_OP_MAHAL_BWD && dout)
        return fail(HH_ERR_INVALID_ARG, "a distance has no output diagonal (d_out must be null)");
    if (algo == Algo::WY && (din || dout))
        return fail(HH_ERR_UNSUPPORTED, "diagonals are applied on the fused path only");
    if (algo == Algo::WY)
        return wy_backward(op, d, U, ldu, lam, X, ldx, Xb, ldb, G, ldg, dX, dXb, lddx, dU, lddu,
                           dlam, saved, saved_bytes, ws, ws_bytes, st);
    if (saved && op != HH_OP_MAHAL_BWD)
        return fail(HH_ERR_UNSUPPORTED, "a coefficient record exists on the WY path only");

    FusedPlan p;
    HH_TRY(make_fused_bwd_plan(d, &p));
    if (!fused_bwd_supported(op, p))
        return fail(HH_ERR_UNSUPPORTED,
                    "fused backward's per-vector state does not fit in on-chip memory (n = %lld, h = %lld)",
                    (long long)n, (long long)h);
    if (saved && saved_bytes < mahal_dots_bytes(d))
        return fail(HH_ERR_WORKSPACE, "record needs %zu bytes, got %zu", mahal_dots_bytes(d), saved_bytes);
    const FusedWs w = fused_ws(op, p);
    if (h > 0) HH_TRY(check_ptr("U", U));
    if (N > 0) {
        HH_TRY(check_ptr(op == HH_OP_MAHAL_BWD ? "Xa" : "X", X));
        HH_TRY(check_ptr(op == HH_OP_MAHAL_BWD ? "ddist" : "dY", G));
        if (op == HH_OP_MAHAL_BWD) HH_TRY(check_ptr("Xb", Xb));
    }
    if (uses_lam(op)) HH_TRY(check_ptr("lam", lam));
    if (w.total > 0) HH_TRY(check_ptr("ws", ws));
    if (ws_bytes < w.total)
        return fail(HH_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w.total, ws_bytes);

    char *base = static_cast<char *>(ws);
    hipError_t e = launch_setup_fused(p.t, U, ldu, uses_lam(op) ? lam : nullptr, n, h, p.s.npad,
                                      base + w.ut, base + w.tau,
                                      uses_lam(op) ? base + w.lam : nullptr,
                                      reinterpret_cast<double *>(base + w.uh64),
                                      reinterpret_cast<double *>(base + w.nrm64), nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
    const size_t es = dtype_size(p.t);
    const int wvec = 16 / (int)es;
    FusedBwdArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.Xb = Xb;
    a.ldb = ldb;
    a.G = G;
    a.ldg = ldg;
    a.dX = dX;
    a.dXb = dXb;
    a.lddx = lddx;
    a.ut = base + w.ut;
    a.tau = base + w.tau;
    a.lam = base + w.lam;
    a.uh64 = reinterpret_cast<const double *>(base + w.uh64);
    a.nrm64 = reinterpret_cast<const double *>(base + w.nrm64);
    a.dU = dU;
    a.lddu = lddu;
    a.dlam = dlam;
    a.scratch = base + w.bwd;
    a.din = din;
    a.dout = dout;
    a.dots = saved;
    a.n = (int)n;
    a.h = (int)h;
    a.npad = p.s.npad;
    a.N = N;
    bool vec = (n % wvec == 0) && aligned16(X) && (ldx % wvec == 0);
    if (op == HH_OP_MAHAL_BWD) vec = vec && aligned16(Xb) && (ldb % wvec == 0);
    else vec = vec && aligned16(G) && (ldg % wvec == 0);
    if (dX) vec = vec && aligned16(dX) && (lddx % wvec == 0);
    if (dXb) vec = vec && aligned16(dXb) && (lddx % wvec == 0);
    a.vec_ok = vec ? 1 : 0;
    e = launch_fused_bwd(p, op, a, st);
    if (e != hipSuccess) return hip_fail(e, "fused backward launch");
    return HH_OK;
}

// ---------------------------------------------------------------------------
// Scratch of hh_forward_noalloc: a file-scope device array, one copy on each
// GPU the library's code object is loaded on, held until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address comes from hipGetSymbolAddress, once per device (with that
// device current), and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[HH_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static hh_status scratch_for(hipStream_t st, void **out) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int dev = cur;
    if (st) {
        e = hipStreamGetDevice(st, &dev);
        if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    }
    if (dev != cur)
        return fail(HH_ERR_INVALID_ARG,
                    "the stream belongs to device %d but device %d is current; make the stream's "
                    "device current", dev, cur);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HH_ERR_UNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(HH_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HH_OK;
}

}  // namespace hh

using namespace hh;

extern "C" {

hh_status hh_forward_noalloc(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                             const void *lam, const void *X, int64_t ldx, const void *Xb,
                             int64_t ldb, void *Y, int64_t ldy, hipStream_t stream) {
    if (!op_in(op, HH_OP_APPLY, HH_OP_MAHAL))
        return fail(HH_ERR_INVALID_ARG, "op must be a forward op");
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    size_t need = 0;
    HH_TRY(hh_workspace_size(op, d, &need));
    if (need > (size_t)HH_NOALLOC_SCRATCH_BYTES)
        return fail(HH_ERR_WORKSPACE,
                    "this call needs %zu bytes of scratch; the library's static scratch holds %zu "
                    "(use the entry point with a workspace argument)",
                    need, (size_t)HH_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    HH_TRY(scratch_for(stream, &ws));
    const bool two = op == HH_OP_MAHAL;
    return forward(op, d, U, ldu, (op == HH_OP_SYM || two) ? lam : nullptr, X, ldx,
                   two ? Xb : nullptr, two ? ldb : 0, Y, two ? 0 : ldy, ws,
                   (size_t)HH_NOALLOC_SCRATCH_BYTES, stream);
}

hh_status hh_workspace_size(hh_op op, const hh_desc *d, size_t *bytes) {
    if (!bytes) return fail(HH_ERR_INVALID_ARG, "bytes must not be null");
    if (!op_in(op, HH_OP_APPLY, HH_OP_MAHAL_BWD)) return fail(HH_ERR_INVALID_ARG, "unknown op");
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    if (algo == Algo::WY) return wy_workspace_size(op, d, bytes);
    FusedPlan p;
    if (is_bwd(op)) HH_TRY(make_fused_bwd_plan(d, &p));
    else HH_TRY(make_fused_plan(d, &p));
    if (is_bwd(op) && !fused_bwd_supported(op, p))
        return fail(HH_ERR_UNSUPPORTED, "fused backward needs all h reflectors in LDS");
    *bytes = fused_ws(op, p).total;
    return HH_OK;
}

hh_status hh_apply(const hh_desc *d, const void *U, int64_t ldu, const void *X, int64_t ldx,
                   void *Y, int64_t ldy, void *ws, size_t ws_bytes, hipStream_t stream) {
    return forward(HH_OP_APPLY, d, U, ldu, nullptr, X, ldx, nullptr, 0, Y, ldy, ws, ws_bytes,
                   stream);
}

hh_status hh_apply_T(const hh_desc *d, const void *U, int64_t ldu, const void *X, int64_t ldx,
                     void *Y, int64_t ldy, void *ws, size_t ws_bytes, hipStream_t stream) {
    return forward(HH_OP_APPLY_T, d, U, ldu, nullptr, X, ldx, nullptr, 0, Y, ldy, ws, ws_bytes,
                   stream);
}

hh_status hh_sym_apply(const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                       const void *X, int64_t ldx, void *Y, int64_t ldy, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
    return forward(HH_OP_SYM, d, U, ldu, lam, X, ldx, nullptr, 0, Y, ldy, ws, ws_bytes, stream);
}

hh_status hh_mahalanobis(const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                         const void *Xa, int64_t lda, const void *Xb, int64_t ldb, void *dist,
                         void *ws, size_t ws_bytes, hipStream_t stream) {
    return forward(HH_OP_MAHAL, d, U, ldu, lam, Xa, lda, Xb, ldb, dist, 0, ws, ws_bytes, stream);
}

hh_status hh_apply_backward(const hh_desc *d, const void *U, int64_t ldu, const void *X,
                            int64_t ldx, const void *dY, int64_t lddy, void *dX, int64_t lddx,
                            void *dU, int64_t lddu, void *ws, size_t ws_bytes,
                            hipStream_t stream) {
    return backward(HH_OP_APPLY_BWD, d, U, ldu, nullptr, X, ldx, nullptr, 0, dY, lddy, dX,
                    nullptr, lddx, dU, lddu, nullptr, ws, ws_bytes, stream);
}

hh_status hh_apply_T_backward(const hh_desc *d, const void *U, int64_t ldu, const void *X,
                              int64_t ldx, const void *dY, int64_t lddy, void *dX,
                              int64_t lddx, void *dU, int64_t lddu, void *ws, size_t ws_bytes,
                              hipStream_t stream) {
    return backward(HH_OP_APPLY_T_BWD, d, U, ldu, nullptr, X, ldx, nullptr, 0, dY, lddy, dX,
                    nullptr, lddx, dU, lddu, nullptr, ws, ws_bytes, stream);
}

hh_status hh_sym_apply_backward(const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                                const void *X, int64_t ldx, const void *dY, int64_t lddy,
                                void *dX, int64_t lddx, void *dU, int64_t lddu, void *dlam,
                                void *ws, size_t ws_bytes, hipStream_t stream) {
    return backward(HH_OP_SYM_BWD, d, U, ldu, lam, X, ldx, nullptr, 0, dY, lddy, dX, nullptr,
                    lddx, dU, lddu, dlam, ws, ws_bytes, stream);
}

hh_status hh_mahalanobis_backward(const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                                  const void *Xa, int64_t lda, const void *Xb, int64_t ldb,
                                  const void *ddist, void *dXa, void *dXb, int64_t lddx,
                                  void *dU, int64_t lddu, void *dlam, void *ws,
                                  size_t ws_bytes, hipStream_t stream) {
    return backward(HH_OP_MAHAL_BWD, d, U, ldu, lam, Xa, lda, Xb, ldb, ddist, 0, dXa, dXb, lddx,
                    dU, lddu, dlam, ws, ws_bytes, stream);
}

hh_status hh_saved_size(hh_op op, const hh_desc *d, size_t *bytes) {
    if (!bytes) return fail(HH_ERR_INVALID_ARG, "bytes must not be null");
    if (!op_in(op, HH_OP_APPLY, HH_OP_SYM))
        return fail(HH_ERR_INVALID_ARG, "op must be HH_OP_APPLY, HH_OP_APPLY_T or HH_OP_SYM");
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    if (algo != Algo::WY) return fail(HH_ERR_UNSUPPORTED, "a coefficient record exists on the WY path only");
    return wy_saved_size(op, d, bytes);
}

hh_status hh_forward_save(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                          const void *X, int64_t ldx, void *Y, int64_t ldy, void *saved,
                          size_t saved_bytes, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!op_in(op, HH_OP_APPLY, HH_OP_SYM))
        return fail(HH_ERR_INVALID_ARG, "op must be HH_OP_APPLY, HH_OP_APPLY_T or HH_OP_SYM");
    HH_TRY(check_ptr("saved", saved));
    return forward(op, d, U, ldu, op == HH_OP_SYM ? lam : nullptr, X, ldx, nullptr, 0, Y, ldy, ws,
                   ws_bytes, stream, saved, saved_bytes);
}

hh_status hh_forward_signed(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                            const void *lam, const void *d_in, const void *d_out, const void *X,
                            int64_t ldx, const void *Xb, int64_t ldb, void *Y, int64_t ldy,
                            void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!op_in(op, HH_OP_APPLY, HH_OP_MAHAL))
        return fail(HH_ERR_INVALID_ARG, "op must be a forward op");
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    const size_t es = dtype_size(d->param_dtype);
    if (((uintptr_t)d_in % es) != 0 || ((uintptr_t)d_out % es) != 0)
        return fail(HH_ERR_INVALID_ARG, "d_in and d_out must be aligned to their element size");
    return forward(op, d, U, ldu, (op == HH_OP_SYM || op == HH_OP_MAHAL) ? lam : nullptr, X, ldx,
                   op == HH_OP_MAHAL ? Xb : nullptr, ldb, Y, ldy, ws, ws_bytes, stream, nullptr, 0,
                   d_in, d_out);
}

hh_status hh_backward_signed(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                             const void *lam, const void *d_in, const void *d_out, const void *X,
                             int64_t ldx, const void *Xb, int64_t ldb, const void *dY, int64_t lddy,
                             void *dX, void *dXb, int64_t lddx, void *dU, int64_t lddu, void *dlam,
                             void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!op_in(op, HH_OP_APPLY_BWD, HH_OP_MAHAL_BWD))
        return fail(HH_ERR_INVALID_ARG, "op must be a backward op");
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    const size_t es = dtype_size(d->param_dtype);
    if (((uintptr_t)d_in % es) != 0 || ((uintptr_t)d_out % es) != 0)
        return fail(HH_ERR_INVALID_ARG, "d_in and d_out must be aligned to their element size");
    const bool mahal = op == HH_OP_MAHAL_BWD;
    const bool has_lam = op == HH_OP_SYM_BWD || mahal;
    return backward(op, d, U, ldu, has_lam ? lam : nullptr, X, ldx, mahal ? Xb : nullptr, ldb, dY,
                    mahal ? 0 : lddy, dX, mahal ? dXb : nullptr, lddx, dU, lddu,
                    has_lam ? dlam : nullptr, ws, ws_bytes, stream, nullptr, 0, d_in, d_out);
}

hh_status hh_backward_saved(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                            const void *lam, const void *X, int64_t ldx, const void *saved,
                            size_t saved_bytes, const void *dY, int64_t lddy, void *dX,
                            int64_t lddx, void *dU, int64_t lddu, void *dlam, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
    if (!op_in(op, HH_OP_APPLY_BWD, HH_OP_SYM_BWD))
        return fail(HH_ERR_INVALID_ARG,
                    "op must be HH_OP_APPLY_BWD, HH_OP_APPLY_T_BWD or HH_OP_SYM_BWD");
    HH_TRY(check_ptr("saved", saved));
    const bool sym = op == HH_OP_SYM_BWD;
    return backward(op, d, U, ldu, sym ? lam : nullptr, X, ldx, nullptr, 0, dY, lddy, dX, nullptr,
                    lddx, dU, lddu, sym ? dlam : nullptr, ws, ws_bytes, stream, saved, saved_bytes);
}

hh_status hh_mahalanobis_saved_size(const hh_desc *d, size_t *bytes) {
    if (!bytes) return fail(HH_ERR_INVALID_ARG, "bytes must not be null");
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    if (algo == Algo::WY) return fail(HH_ERR_UNSUPPORTED, "the distance record exists on the fused path only");
    FusedPlan p;
    HH_TRY(make_fused_plan(d, &p));
    *bytes = mahal_dots_bytes(d);
    return HH_OK;
}

hh_status hh_mahalanobis_save(const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                              const void *Xa, int64_t lda, const void *Xb, int64_t ldb, void *dist,
                              void *saved, size_t saved_bytes, void *ws, size_t ws_bytes,
                              hipStream_t stream) {
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    if (algo == Algo::WY) return fail(HH_ERR_UNSUPPORTED, "the distance record exists on the fused path only");
    if (d->N > 0 && d->h > 0) HH_TRY(check_ptr("saved", saved));
    return forward(HH_OP_MAHAL, d, U, ldu, lam, Xa, lda, Xb, ldb, dist, 0, ws, ws_bytes, stream,
                   d->N > 0 && d->h > 0 ? saved : nullptr, saved_bytes);
}

hh_status hh_mahalanobis_backward_saved(const hh_desc *d, const void *U, int64_t ldu,
                                        const void *lam, const void *Xa, int64_t lda,
                                        const void *Xb, int64_t ldb, const void *saved,
                                        size_t saved_bytes, const void *ddist, void *dXa,
                                        void *dXb, int64_t lddx, void *dU, int64_t lddu,
                                        void *dlam, void *ws, size_t ws_bytes, hipStream_t stream) {
    Algo algo;
    HH_TRY(check_desc(d, &algo));
    if (algo == Algo::WY) return fail(HH_ERR_UNSUPPORTED, "the distance record exists on the fused path only");
    if (d->N > 0 && d->h > 0) HH_TRY(check_ptr("saved", saved));
    return backward(HH_OP_MAHAL_BWD, d, U, ldu, lam, Xa, lda, Xb, ldb, ddist, 0, dXa, dXb, lddx, dU,
                    lddu, dlam, ws, ws_bytes, stream, d->N > 0 && d->h > 0 ? saved : nullptr,
                    saved_bytes);
}

const char *hh_status_string(hh_status s) {
    switch (s) {
    case HH_OK: return "HH_OK";
    case HH_ERR_INVALID_ARG: return "HH_ERR_INVALID_ARG: invalid argument";
    case HH_ERR_UNSUPPORTED: return "HH_ERR_UNSUPPORTED: unsupported combination";
    case HH_ERR_WORKSPACE: return "HH_ERR_WORKSPACE: workspace too small";
    case HH_ERR_HIP: return "HH_ERR_HIP: HIP runtime error";
    }
    return "unknown hh_status";
}

const char *hh_last_error(void) { return g_last_error.c_str(); }

int hh_version(void) { return 410; }  // 0.4.1: distance record (hh_mahalanobis_save)

}  // extern "C"

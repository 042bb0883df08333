/*
 * Memory and undefined-behaviour check of the library's host code (test
 * infrastructure): the C ABI's validation, workspace and record size
 * arithmetic, built host-only under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Every call here is refused (or only sizes a
 * buffer) before any device work: the pointers are fake, nothing is launched.
 * It sweeps hh_workspace_size / hh_saved_size over ops, types and sizes up to
 * the library's limits (integer overflow in the size arithmetic is what UBSan
 * would report) and checks the status of a table of invalid calls.
 * Exit status 0 means clean.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "hh.h"

static int failures = 0;
#define EXPECT(call, want)                                                              \
    do {                                                                                \
        hh_status _s = (call);                                                          \
        if (_s != (want)) {                                                             \
            ++failures;                                                                 \
            printf("FAIL line %d: %s -> %d (want %d): %s\n", __LINE__, #call, (int)_s,  \
                   (int)(want), hh_last_error());                                      \
        }                                                                               \
    } while (0)

#define FAKE(a) ((void *)(uintptr_t)(a))

int main(void) {
    static const int64_t ns[] = {1, 7, 8, 512, 513, 1024, 4096, 6144, 8192, 8193, (1 << 30) - 1};
    static const int64_t hs[] = {0, 1, 9, 64, 100, 128, 129, 5000};
    static const int64_t Ns[] = {0, 1, 33, 1 << 20, (int64_t)1 << 31, (int64_t)1 << 40};
    static const hh_dtype comps[] = {HH_F64, HH_F32, HH_BF16, HH_F16};
    size_t sweeps = 0;
    for (size_t a = 0; a < sizeof(ns) / sizeof(ns[0]); ++a)
        for (size_t b = 0; b < sizeof(hs) / sizeof(hs[0]); ++b)
            for (size_t c = 0; c < sizeof(Ns) / sizeof(Ns[0]); ++c)
                for (int ci = 0; ci < 4; ++ci)
                    for (int io32 = 0; io32 < 2; ++io32)
                        for (int op = HH_OP_APPLY; op <= HH_OP_MAHAL_BWD; ++op) {
                            hh_desc d;
                            memset(&d, 0, sizeof(d));
                            d.n = ns[a];
                            d.h = hs[b];
                            d.N = Ns[c];
                            d.compute_dtype = comps[ci];
                            d.param_dtype = ci < 2 ? comps[ci] : HH_F32;
                            d.io_dtype = io32 && ci >= 2 ? HH_F32 : comps[ci];
                            d.algo = HH_ALGO_AUTO;
                            size_t bytes = 0;
                            hh_status s = hh_workspace_size((hh_op)op, &d, &bytes);
                            if (s != HH_OK && s != HH_ERR_UNSUPPORTED) {
                                ++failures;
                                printf("FAIL: workspace size status %d for n=%lld h=%lld N=%lld op=%d: %s\n",
                                       (int)s, (long long)d.n, (long long)d.h, (long long)d.N, op,
                                       hh_last_error());
                            }
                            if (op <= HH_OP_SYM) (void)hh_saved_size((hh_op)op, &d, &bytes);
                            ++sweeps;
                        }

    hh_desc d;
    memset(&d, 0, sizeof(d));
    d.n = 64; d.h = 4; d.N = 100;
    d.param_dtype = d.io_dtype = d.compute_dtype = HH_F32;
    d.algo = HH_ALGO_AUTO;
    void *U = FAKE(0x1000), *X = FAKE(0x2000), *Y = FAKE(0x3000), *ws = FAKE(0x4000);
    EXPECT(hh_apply(NULL, U, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    EXPECT(hh_apply(&d, U, 63, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    EXPECT(hh_apply(&d, U, 64, X, 63, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 0, NULL), HH_ERR_WORKSPACE);
    EXPECT(hh_apply(&d, NULL, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    EXPECT(hh_apply(&d, U, 64, X, 64, X, 65, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    EXPECT(hh_mahalanobis(&d, U, 64, NULL, X, 64, Y, 64, FAKE(0x5000), ws, 1 << 20, NULL),
           HH_ERR_INVALID_ARG);
    EXPECT(hh_sym_apply_backward(&d, U, 64, FAKE(0x6000), X, 64, Y, 64, NULL, 64, NULL, 64, NULL,
                                 ws, 0, NULL), HH_ERR_WORKSPACE);
    d.n = 0;
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    d.n = 64; d.h = -1;
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    d.h = 4; d.N = -5;
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    d.N = 100; d.compute_dtype = (hh_dtype)9;
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_INVALID_ARG);
    d.compute_dtype = HH_BF16;  /* WY with F32 parameters only */
    d.io_dtype = HH_BF16;
    d.param_dtype = HH_F16;
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 1 << 20, NULL), HH_ERR_UNSUPPORTED);
    d.param_dtype = HH_F32;
    d.n = 100;  /* WY needs n % 8 == 0 */
    EXPECT(hh_apply(&d, U, 100, X, 100, Y, 100, ws, 1 << 24, NULL), HH_ERR_UNSUPPORTED);
    d.n = 64; d.h = 129;
    EXPECT(hh_apply(&d, U, 64, X, 64, Y, 64, ws, 1 << 24, NULL), HH_ERR_UNSUPPORTED);
    d.h = 4;
    EXPECT(hh_mahalanobis(&d, U, 64, FAKE(0x6000), X, 64, Y, 64, FAKE(0x5000), ws, 1 << 24, NULL),
           HH_ERR_UNSUPPORTED);
    EXPECT(hh_forward_signed(HH_OP_APPLY, &d, U, 64, NULL, FAKE(0x7000), NULL, X, 64, NULL, 0, Y,
                             64, ws, 1 << 24, NULL), HH_ERR_UNSUPPORTED);
    EXPECT(hh_forward_signed(HH_OP_APPLY_BWD, &d, U, 64, NULL, NULL, NULL, X, 64, NULL, 0, Y, 64,
                             ws, 1 << 24, NULL), HH_ERR_INVALID_ARG);
    EXPECT(hh_backward_saved(HH_OP_APPLY_BWD, &d, U, 64, NULL, X, 64, NULL, 0, Y, 64, NULL, 64,
                             NULL, 64, NULL, ws, 1 << 24, NULL), HH_ERR_INVALID_ARG);
    d.io_dtype = HH_F32; d.N = 4096; d.n = 4096; d.h = 64;  /* 64 MiB of 16-bit copies */
    EXPECT(hh_forward_noalloc(HH_OP_APPLY, &d, U, 4096, NULL, X, 4096, NULL, 0, Y, 4096, NULL),
           HH_ERR_WORKSPACE);
    EXPECT(hh_forward_noalloc(HH_OP_SYM_BWD, &d, U, 4096, NULL, X, 4096, NULL, 0, Y, 4096, NULL),
           HH_ERR_INVALID_ARG);
    size_t fb = 0;
    EXPECT(hh_factor_workspace_size(HH_FACTOR_QR, 4096, 4095, &fb), HH_OK);
    EXPECT(hh_factor_workspace_size(HH_FACTOR_QR, 4096, 4096, &fb), HH_ERR_INVALID_ARG);
    EXPECT(hh_factor_workspace_size((hh_factor_method)9, 64, 4, &fb), HH_ERR_INVALID_ARG);
    EXPECT(hh_factor_workspace_size(HH_FACTOR_CONSTRAINED, (int64_t)1 << 40, 4, &fb), HH_ERR_UNSUPPORTED);
    EXPECT(hh_factor_orthonormal(HH_FACTOR_UNCONSTRAINED, 16, 4, (const double *)U, 16, (double *)Y,
                                 16, NULL, NULL, ws, 16, NULL), HH_ERR_WORKSPACE);
    EXPECT(hh_workspace_size((hh_op)42, &d, (size_t *)ws), HH_ERR_INVALID_ARG);
    EXPECT(hh_workspace_size(HH_OP_APPLY, &d, NULL), HH_ERR_INVALID_ARG);
    printf("host sanitizer check: %zu size queries, %d failure(s)\n", sweeps, failures);
    return failures ? 1 : 0;
}

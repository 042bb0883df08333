/*
 * hh.h -- C ABI of the Householder-reflector transform library (libhh.so).
 *
 * The library applies an orthonormal operator built from a few Householder
 * reflectors to large batches of vectors on an AMD Instinct MI355X (gfx950):
 *
 *   H_k = I - 2 uh_k uh_k^T,  uh_k = u_k / ||u_k||_2        (paper Sec. II-A, eq. 2)
 *   Q   = H_1 H_2 ... H_h                                   (eq. 1, in the order
 *                                                            Result 3 uses, eq. theU2)
 *   Y = Q X,   Y = Q^T X                                    (Sec. II-A: 4nh ops/vector)
 *   Y = Q diag(lam) Q^T X                                   (Sec. III-A, eq. thesbar,
 *                                                            D = I: (8h+1)n ops/vector)
 *   d_j = || diag(sqrt(lam)) Q^T (xa_j - xb_j) ||^2         (Sec. IV-C: the learned
 *                                                            metric L = sqrt(Lambda) U)
 * and the gradients of each with respect to X, the reflector vectors and lam.
 * Q^{-1} = Q^T, so the solve of Sec. I is hh_apply_T; the inverse of the
 * symmetric form is hh_sym_apply with 1/lam.
 *
 * Reflector vectors are normalised inside the library in FP64.  A zero column
 * u_k gives H_k = I (Sec. II-B, after Result 1) and a zero gradient.  Any
 * h >= 0 is accepted (h = 0 is the identity); the bounds h < n/2 and
 * h < n/4 of Secs. II-A and III-A are efficiency bounds, not validity bounds.
 *
 * ---------------------------------------------------------------------------
 * Layout (column-major, BLAS style; every data pointer is a DEVICE pointer):
 *   U(i,k) = U[i + k*ldu]   i < n, k < h      reflector k is column k
 *   X(i,j) = X[i + j*ldx]   i < n, j < N      vector j is contiguous
 *   lam, dlam: n contiguous; dist, ddist: N contiguous.
 *   In torch terms U is an (h, n) tensor and X an (N, n) tensor.
 *
 * Ownership: the caller owns every buffer.  The library never allocates or
 * frees device memory; scratch space is the caller's workspace `ws` of at least
 * hh_workspace_size() bytes, 256-byte aligned.  Outputs dU and dlam are
 * overwritten, not accumulated.  Calls are stream-ordered and asynchronous:
 * each validates its arguments on the host, enqueues kernels on `stream` and
 * returns; outputs are valid once the stream has passed the call.  Calls that
 * share a workspace must be ordered on one stream.  No exception crosses the
 * ABI.  NaN and Inf propagate and are not detected.
 *
 * Numbers (hh_desc): the FUSED algorithm computes in F64 or F32 with parameters
 * and data of that same type.  The WY algorithm (compact form Q = I - Y T Y^T,
 * prior art of Bischof & Van Loan and Schreiber & Van Loan, not the paper)
 * computes in BF16 or F16 on the matrix cores with FP32 accumulation, F32
 * parameters, and data in the compute type or in F32 (F32 data is rounded to
 * the compute type, nearest even, into the workspace before the 16-bit kernels
 * run and their 16-bit results are widened back: the results are those of the
 * 16-bit path on the rounded data, at the cost of one extra pass over each
 * F32 operand; hh_workspace_size then grows with N).  HH_ALGO_AUTO picks
 * FUSED for F64/F32 compute and WY for BF16/F16 compute.  Any other
 * combination returns HH_ERR_UNSUPPORTED.
 *
 * Sizes (beyond them a call returns HH_ERR_UNSUPPORTED, nothing is enqueued):
 * FUSED forward n <= 8192 (F32) or 4096 (F64), any h (reflectors are staged
 * through on-chip memory in chunks); FUSED backward n <= 4096 (F32) or 2048
 * (F64), any h (the reflectors are staged in on-chip memory when they fit,
 * else read through the caches); WY n <= 8192,
 * h <= 128, n and every leading dimension multiples of 8, 16-bit data 16-byte
 * aligned.
 *
 * Validation (synchronous, before anything is enqueued): n >= 1, h >= 0,
 * N >= 0; every leading dimension >= n; required pointers non-null when
 * N > 0 (U may be null only when h == 0); ws_bytes >= the required size
 * (else HH_ERR_WORKSPACE).  N == 0 is a no-op for the forward calls; the
 * backward calls then write zero dU/dlam.  Y may alias X exactly (Y == X and
 * ldy == ldx) in hh_apply, hh_apply_T and hh_sym_apply; any other overlap
 * is undefined.  hh_last_error() returns a thread-local message for the last
 * failing call on the calling thread.
 */
#ifndef HH_H_
#define HH_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#if defined(__GNUC__)
#define HH_API __attribute__((visibility("default")))
#else
#define HH_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HH_OK = 0,
    HH_ERR_INVALID_ARG = 1,
    HH_ERR_UNSUPPORTED = 2,
    HH_ERR_WORKSPACE = 3,
    HH_ERR_HIP = 4
} hh_status;

typedef enum { HH_F64 = 0, HH_F32 = 1, HH_BF16 = 2, HH_F16 = 3 } hh_dtype;

/* HH_ALGO_FUSED_QR: the FUSED algorithm with forward kernels that leave out
 * each reflector's leading zeros, in whole 16-byte chunks of every lane's
 * slice (the first nonzero entry is found in the setup).  Reflectors of a
 * Householder QR have k - 1 leading zeros (the remark after Result 3: an
 * application costs 4(n - k + 1) operations instead of 4n); at h = n - 1 that
 * halves the work.  Results are those of FUSED (skipped terms are exact
 * zeros); any reflectors are accepted.  Backward calls run as FUSED. */
typedef enum { HH_ALGO_AUTO = 0, HH_ALGO_FUSED = 1, HH_ALGO_WY = 2, HH_ALGO_FUSED_QR = 3 } hh_algo;

typedef enum {
    HH_OP_APPLY = 0,
    HH_OP_APPLY_T = 1,
    HH_OP_SYM = 2,
    HH_OP_MAHAL = 3,
    HH_OP_APPLY_BWD = 4,
    HH_OP_APPLY_T_BWD = 5,
    HH_OP_SYM_BWD = 6,
    HH_OP_MAHAL_BWD = 7
} hh_op;

typedef struct {
    int64_t n;              /* vector length (rows of U and X)                   */
    int64_t h;              /* number of reflectors (columns of U)               */
    int64_t N;              /* number of vectors (pairs for the Mahalanobis ops) */
    hh_dtype param_dtype;   /* U, lam, dist, ddist, dU, dlam                     */
    hh_dtype io_dtype;      /* X, Xa, Xb, Y, dY, dX, dXa, dXb                    */
    hh_dtype compute_dtype; /* FUSED: F64 | F32 ; WY: BF16 | F16                 */
    hh_algo algo;
} hh_desc;

/* Bytes of workspace that `op` needs for descriptor `d` (0 is possible). */
HH_API hh_status hh_workspace_size(hh_op op, const hh_desc *d, size_t *bytes);

/* Y = Q X  (Sec. II-A, eqs. 1-2).  Y is n x N with leading dimension ldy. */
HH_API hh_status hh_apply(const hh_desc *d, const void *U, int64_t ldu, const void *X,
                   int64_t ldx, void *Y, int64_t ldy, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/* Y = Q^T X = H_h ... H_1 X  (Sec. II-A; also the solve Q^{-1} X). */
HH_API hh_status hh_apply_T(const hh_desc *d, const void *U, int64_t ldu, const void *X,
                     int64_t ldx, void *Y, int64_t ldy, void *ws, size_t ws_bytes,
                     hipStream_t stream);

/* Y = Q diag(lam) Q^T X  (Sec. III-A, eq. thesbar with D = I). */
HH_API hh_status hh_sym_apply(const hh_desc *d, const void *U, int64_t ldu,
                       const void *lam, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, void *ws, size_t ws_bytes, hipStream_t stream);

/* dist[j] = sum_i lam_i ((Q^T (xa_j - xb_j))_i)^2  (Sec. IV-C).  N pairs.
 * dist has param_dtype.  lam >= 0 is the metric's meaning but is not checked. */
HH_API hh_status hh_mahalanobis(const hh_desc *d, const void *U, int64_t ldu,
                         const void *lam, const void *Xa, int64_t lda,
                         const void *Xb, int64_t ldb, void *dist, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* Gradients of L with upstream dY = dL/dY for Y = Q X (hh_apply_backward) or
 * Y = Q^T X (hh_apply_T_backward).  dX (nullable, n x N, lddx) receives
 * dL/dX; dU (nullable, n x h, lddu, param_dtype) receives dL/dU for the raw U:
 * dU_k = (I - uh_k uh_k^T) (dL/duh_k) / ||u_k||; at unit norm this is the
 * tangent projection the paper applies to its gradient before each step on
 * the sphere (Sec. III-B, after eq. gradient); zero for a zero column.  The
 * sum over the N vectors is deterministic for a given device and shape. */
HH_API hh_status hh_apply_backward(const hh_desc *d, const void *U, int64_t ldu,
                            const void *X, int64_t ldx, const void *dY,
                            int64_t lddy, void *dX, int64_t lddx, void *dU,
                            int64_t lddu, void *ws, size_t ws_bytes,
                            hipStream_t stream);
HH_API hh_status hh_apply_T_backward(const hh_desc *d, const void *U, int64_t ldu,
                              const void *X, int64_t ldx, const void *dY,
                              int64_t lddy, void *dX, int64_t lddx, void *dU,
                              int64_t lddu, void *ws, size_t ws_bytes,
                              hipStream_t stream);

/* Gradients of L for Y = Q diag(lam) Q^T X: dX = S dY (S symmetric),
 * dlam_i = sum_j (Q^T dY)_ij (Q^T X)_ij, dU as above.  All outputs nullable. */
HH_API hh_status hh_sym_apply_backward(const hh_desc *d, const void *U, int64_t ldu,
                                const void *lam, const void *X, int64_t ldx,
                                const void *dY, int64_t lddy, void *dX,
                                int64_t lddx, void *dU, int64_t lddu, void *dlam,
                                void *ws, size_t ws_bytes, hipStream_t stream);

/* Gradients of L for dist = hh_mahalanobis(...), with ddist[j] = dL/ddist_j
 * (param_dtype, N long).  dXa = -dXb = Q (2 ddist_j lam .* z_j) with
 * z_j = Q^T (xa_j - xb_j); dlam_i = sum_j ddist_j z_ij^2; dU as above.
 * dXa and dXb share lddx.  All outputs nullable. */
HH_API hh_status hh_mahalanobis_backward(const hh_desc *d, const void *U, int64_t ldu,
                                  const void *lam, const void *Xa, int64_t lda,
                                  const void *Xb, int64_t ldb, const void *ddist,
                                  void *dXa, void *dXb, int64_t lddx, void *dU,
                                  int64_t lddu, void *dlam, void *ws,
                                  size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Saved forward record (WY algorithm only; not in the paper).  The WY backward
 * of Q X, Q^T X and Q diag(lam) Q^T X needs, per vector, the h coefficients
 * of its compact-WY forward: T Y^T x for Q x, T^T Y^T x for Q^T x, and for
 * the symmetric form both T^T Y^T x and T Y^T (diag(lam) Q^T x); and it needs
 * the reflector setup (normalised and rounded reflectors, T, the spectrum).
 * The plain backward calls form both again, the coefficients by a pass over X.
 * A forward that writes them to a caller-owned record spares the backward that
 * pass and that setup (h scalars per vector are kept, not h copies of the
 * vector).
 *
 * Record: 16-bit coefficient rows in the compute type (m = h rounded up to 64
 * or 128, twice that for the symmetric form; row stride N rounded up to 32,
 * at least 32; columns past N zero), followed by the setup.  Its contents are
 * internal to the library; it stays valid for the same U, lam, X, n, h, N and
 * dtypes.
 *
 * hh_saved_size: bytes of the record for forward op HH_OP_APPLY, HH_OP_APPLY_T
 * or HH_OP_SYM; HH_ERR_UNSUPPORTED for the fused algorithm, whose backward
 * recomputes each vector's dot products in registers. */
HH_API hh_status hh_saved_size(hh_op op, const hh_desc *d, size_t *bytes);

/* The forward op (HH_OP_APPLY, HH_OP_APPLY_T or HH_OP_SYM; lam is read for
 * HH_OP_SYM only, else ignored) with the same Y as hh_apply / hh_apply_T /
 * hh_sym_apply, which also fills the record `saved` (device, non-null,
 * 16-byte aligned, saved_bytes >= hh_saved_size).  The record takes the place
 * of the workspace: with data in the compute type ws may be null and ws_bytes
 * 0; F32 data still needs hh_workspace_size(op) bytes for its conversion.
 * With N == 0 only the setup is recorded. */
HH_API hh_status hh_forward_save(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                          const void *lam, const void *X, int64_t ldx, void *Y,
                          int64_t ldy, void *saved, size_t saved_bytes, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/* The backward op (HH_OP_APPLY_BWD, HH_OP_APPLY_T_BWD or HH_OP_SYM_BWD) from
 * the record hh_forward_save filled for the matching forward op on the same
 * inputs: the results of hh_apply_backward / hh_apply_T_backward /
 * hh_sym_apply_backward (lam and dlam are used for HH_OP_SYM_BWD only; U and
 * lam are validated, their setup is taken from the record) without their pass
 * over X and their setup.  X is still read: dU needs it.  Workspace: that of
 * the backward op.  A record of other inputs gives wrong gradients, not an
 * error. */
HH_API hh_status hh_backward_saved(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                            const void *lam, const void *X, int64_t ldx,
                            const void *saved, size_t saved_bytes, const void *dY,
                            int64_t lddy, void *dX, int64_t lddx, void *dU,
                            int64_t lddu, void *dlam, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Record of the fused distance (FUSED algorithm only; not in the paper).  The
 * backward of the distance d = sum_i lam_i ((Q^T (xa - xb))_i)^2 (Sec. IV-C)
 * walks each pair's reflector chain forward again to rebuild s_h = Q^T (xa -
 * xb), which takes the h dot products a_k = u_k^T s_{k-1} of Sec. II-A with
 * their reductions.  hh_mahalanobis_save is hh_mahalanobis that also writes
 * those dot products, as the forward formed them, into a caller-owned record;
 * hh_mahalanobis_backward_saved reads them and rebuilds s_h by the updates
 * alone.  Same results as the plain calls up to the rounding of the dot
 * products (the forward's reduction order instead of the backward's).
 *
 * Record: N rows of the compute type, row j holding the h dot products of
 * pair j (a_1 first) padded with zeros to a multiple of 16 bytes; device memory, at least hh_mahalanobis_saved_size bytes (HH_ERR_WORKSPACE
 * if smaller); may be null when N == 0 or h == 0.  It stays valid for the same
 * U, lam, Xa, Xb, n, h, N and dtypes; a record of other inputs gives wrong
 * gradients, not an error.  The WY algorithm returns HH_ERR_UNSUPPORTED.
 * Other arguments, validation and workspaces as for hh_mahalanobis and
 * hh_mahalanobis_backward. */
HH_API hh_status hh_mahalanobis_saved_size(const hh_desc *d, size_t *bytes);
HH_API hh_status hh_mahalanobis_save(const hh_desc *d, const void *U, int64_t ldu,
                                     const void *lam, const void *Xa, int64_t lda,
                                     const void *Xb, int64_t ldb, void *dist, void *saved,
                                     size_t saved_bytes, void *ws, size_t ws_bytes,
                                     hipStream_t stream);
HH_API hh_status hh_mahalanobis_backward_saved(const hh_desc *d, const void *U, int64_t ldu,
                                               const void *lam, const void *Xa, int64_t lda,
                                               const void *Xb, int64_t ldb, const void *saved,
                                               size_t saved_bytes, const void *ddist, void *dXa,
                                               void *dXb, int64_t lddx, void *dU, int64_t lddu,
                                               void *dlam, void *ws, size_t ws_bytes,
                                               hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Diagonal D on either side (Sec. II-A, eq. 1: the factorisation is D times
 * the reflector product, with D = diag(d), d in {+1, -1}^n; Result 3 puts D
 * on the right of the product instead; Sec. III-A, eq. thesbar: D on both
 * sides of the symmetric form).  The forward op with the input scaled by
 * diag(d_in) and the output by diag(d_out):
 *
 *   HH_OP_APPLY    Y = diag(d_out) Q diag(d_in) X
 *   HH_OP_APPLY_T  Y = diag(d_out) Q^T diag(d_in) X
 *   HH_OP_SYM      Y = diag(d_out) Q diag(lam) Q^T diag(d_in) X
 *   HH_OP_MAHAL    dist_j = sum_i lam_i (Q^T diag(d_in) (xa_j - xb_j))_i^2
 *
 * so eq. 1's operator U = D Q is HH_OP_APPLY with d_out = d and its transpose
 * HH_OP_APPLY_T with d_in = d; Result 3's Q D is HH_OP_APPLY with d_in = d
 * (transpose: HH_OP_APPLY_T with d_out = d); eq. thesbar is HH_OP_SYM with
 * d_in = d_out = d, and its metric HH_OP_MAHAL with d_in = d.  d_in and d_out
 * are device arrays of n param_dtype values, each nullable (null = identity),
 * aligned to their element size; d_out must be null for HH_OP_MAHAL.  Entries
 * of +-1 keep the operator orthonormal; other values are applied as given.
 * Arguments otherwise as for hh_apply / hh_apply_T / hh_sym_apply (Xb, ldb
 * ignored) and hh_mahalanobis (X, ldx = Xa, lda; Y = dist, ldy ignored), same
 * workspace.  The diagonals are multiplied in registers on the vectors' one
 * pass through the chip (no extra pass over HBM).  FUSED algorithm only
 * (HH_ERR_UNSUPPORTED on WY), at the fused forward's sizes. */
HH_API hh_status hh_forward_signed(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                            const void *lam, const void *d_in, const void *d_out,
                            const void *X, int64_t ldx, const void *Xb, int64_t ldb,
                            void *Y, int64_t ldy, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Gradients of L = <dY, Y> for the Y of hh_forward_signed (same op, d_in,
 * d_out): with X' = diag(d_in) X and dY' = diag(d_out) dY, dU and dlam are
 * those of the plain op at (X', dY') and dX = diag(d_in) times the plain op's
 * dX at (X', dY'); for HH_OP_MAHAL_BWD (dY = ddist, N values; d_out null)
 * dXa = -dXb = diag(d_in) times the plain dXa at diag(d_in)(xa - xb).
 * Arguments otherwise as for the backward entry points above (Xb, dXb:
 * HH_OP_MAHAL_BWD only; lam, dlam: HH_OP_SYM_BWD and HH_OP_MAHAL_BWD only;
 * lddy ignored for HH_OP_MAHAL_BWD), same workspace and sizes.  FUSED
 * algorithm only (HH_ERR_UNSUPPORTED on WY). */
HH_API hh_status hh_backward_signed(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                             const void *lam, const void *d_in, const void *d_out,
                             const void *X, int64_t ldx, const void *Xb, int64_t ldb,
                             const void *dY, int64_t lddy, void *dX, void *dXb,
                             int64_t lddx, void *dU, int64_t lddu, void *dlam, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Orthonormal factorisation front-end (Sec. II-B to II-D), FP64 on the GPU:
 * reflectors R (n x h, column k = unit vector u_k or zero, ld ldr >= n) that
 * approximate a given orthonormal U (n x n, ld ldu >= n) as
 * Q = H_1 ... H_h (the order every call above uses), ready for hh_apply etc.
 *   HH_FACTOR_CONSTRAINED   Result 1: mutually orthogonal reflectors, the
 *                           eigenvectors of the negative eigenvalues of
 *                           Z = U + U^T, smallest first; error
 *                           2n - 2 tr U + 2 sum of those eigenvalues
 *                           (eq. bestortho at h = n_-).
 *   HH_FACTOR_UNCONSTRAINED Result 2: Case 1 / Case 2 reflectors along the
 *                           spectrum of Z (eq. theu2); error 2 n_+ - sum of
 *                           the nonnegative z at h = n_- (eq. result2).
 *   HH_FACTOR_QR            Result 3: the first h <= n - 1 reflectors of the
 *                           Householder QR of U and the +-1 diagonal d with
 *                           U ~ Q diag(d) (hh_forward_signed with d_in = d);
 *                           reflector k has k - 1 leading zeros
 *                           (HH_ALGO_FUSED_QR skips them).
 * Reflectors beyond the useful ones (no negative eigenvalue left) are zero
 * columns, i.e. identity factors.  d (n values, nullable): the QR diagonal,
 * all ones for the other methods.  z (n values, nullable): the eigenvalues of
 * U + U^T in ascending order (eigen methods; untouched for QR).  Sizes:
 * n <= 1024 for the eigen methods (cyclic Jacobi, at most 16 sweeps), n <=
 * 4096 for QR.  Workspace of hh_factor_workspace_size bytes; stream-ordered
 * and asynchronous like the transform calls. */
typedef enum {
    HH_FACTOR_CONSTRAINED = 0,
    HH_FACTOR_UNCONSTRAINED = 1,
    HH_FACTOR_QR = 2
} hh_factor_method;

HH_API hh_status hh_factor_workspace_size(hh_factor_method method, int64_t n, int64_t h,
                                          size_t *bytes);
HH_API hh_status hh_factor_orthonormal(hh_factor_method method, int64_t n, int64_t h,
                                       const double *U, int64_t ldu, double *R, int64_t ldr,
                                       double *d, double *z, void *ws, size_t ws_bytes,
                                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Symmetric Householder Factorisation (Sec. III-B, Algorithm 1), FP64 on the
 * GPU: for a symmetric S (n x n, ld lds >= n) finds reflectors R (n x h,
 * column k = u_k, ld ldr >= n), a spectrum sbar (n) and a +-1 diagonal d (n)
 * with Sbar = D U_1 ... U_h diag(sbar) U_h ... U_1 D (eq. thesbar) close to S:
 * the initial reflectors of eq. combine, then K sweeps of the sphere descent
 * of eq. iterate over all reflectors, each followed by the update of D
 * (eq. optimaldiagonal) and, with spectrum_update != 0 (SHF-SU), of sbar
 * (eq. updateofsbar); stops early when a sweep gains less than 1e-8 of the
 * error.  err (K + 1 values, nullable) receives ||S - Sbar||_F^2 after the
 * initialisation and after each sweep (repeated once stopped).  Sbar x is
 * then hh_forward_signed(HH_OP_SYM, lam = sbar, d_in = d_out = d) with these
 * reflectors.  n <= 512; one workgroup runs the whole algorithm (a set-up
 * step).  Workspace of hh_shf_workspace_size bytes; asynchronous. */
HH_API hh_status hh_shf_workspace_size(int64_t n, int64_t h, int64_t K, size_t *bytes);
HH_API hh_status hh_shf(int64_t n, int64_t h, int64_t K, int spectrum_update, const double *S,
                        int64_t lds, double *R, int64_t ldr, double *sbar, double *d, double *err,
                        void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * k nearest neighbours in the learned metric (Sec. IV-C: new points are
 * transformed, x <- L x with L = sqrt(Lambda) U, then k-NN runs on them).
 * Zq (Nq transformed queries) and Zd (Nd transformed database vectors) are
 * FP32 n-vectors (column-major, ld >= n; e.g. hh_forward_signed(HH_OP_APPLY_T,
 * d_out = sqrt(lam)) of the raw data, so that ||z_a - z_b||^2 is the
 * Mahalanobis distance of hh_mahalanobis).  For every query: the k smallest
 * squared distances in ascending order into dist (Nq x k, row q contiguous)
 * and their database indices into idx (Nq x k); equal distances keep the
 * smaller index.  Candidates are ranked by ||a||^2 + ||b||^2 - 2 a^T b (the
 * products on the matrix cores in FP32); the k returned distances are
 * recomputed from the differences.  n <= 224, 1 <= k <= 32, k <= Nd; a
 * workspace of hh_knn_workspace_size bytes holds the per-split lists and the
 * squared norms of both sets. */
HH_API hh_status hh_knn_workspace_size(int64_t n, int64_t Nq, int64_t Nd, int64_t k,
                                       size_t *bytes);
HH_API hh_status hh_knn(int64_t n, int64_t Nq, int64_t Nd, int64_t k, const float *Zq, int64_t ldq,
                        const float *Zd, int64_t ldd, float *dist, int64_t *idx, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* Size of the static device scratch of hh_forward_noalloc (16 MiB, held by
 * each GPU the library runs on until the process ends). */
#define HH_NOALLOC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory or provide a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the forward ops of hh_apply (op = HH_OP_APPLY), hh_apply_T
 * (HH_OP_APPLY_T), hh_sym_apply (HH_OP_SYM, lam) and hh_mahalanobis
 * (HH_OP_MAHAL: X, ldx = Xa, lda; Xb, ldb; Y = dist, ldy ignored), same
 * arguments and results, with the workspace taken from a static device array
 * of HH_NOALLOC_SCRATCH_BYTES inside the library instead of an argument.  The
 * caller still passes inputs and outputs.  Nothing is allocated (no hipMalloc,
 * hipFree or allocating library call); the array's device address is looked
 * up once per device on the first call there.  A call whose workspace
 * (hh_workspace_size) exceeds HH_NOALLOC_SCRATCH_BYTES returns
 * HH_ERR_WORKSPACE and enqueues nothing: 16-bit WY calls fit at every
 * supported size (n <= 8192, h <= 128), FUSED calls while h * n * (4 or 8)
 * bytes of padded reflectors fit, and WY calls with F32 data only while their
 * 16-bit copies of X and Y fit.  The stream must belong to the current
 * device (else HH_ERR_INVALID_ARG).  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (different streams, or
 * threads) race and give undefined results; calls ordered on one stream are
 * safe.  The array keeps the last call's contents; no kernel of these ops
 * reads scratch it has not written in the same call. */
HH_API hh_status hh_forward_noalloc(hh_op op, const hh_desc *d, const void *U, int64_t ldu,
                                    const void *lam, const void *X, int64_t ldx,
                                    const void *Xb, int64_t ldb, void *Y, int64_t ldy,
                                    hipStream_t stream);

/* Static text for a status code. */
HH_API const char *hh_status_string(hh_status s);

/* Detail of the last failing call on this thread ("" if none). */
HH_API const char *hh_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
HH_API int hh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HH_H_ */

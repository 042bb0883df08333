// Internal interface of the compact-WY path (matrix-core GEMMs).
#pragma once

#include "hh_internal.h"

namespace hh {

// Data in FP32 (io_dtype F32) is converted to the compute type on the way in
// and back on the way out around the 16-bit kernels (hh_wy_io.hip); the *16
// functions take data in the compute type only.
hh_status wy_workspace_size(hh_op op, const hh_desc *d, size_t *bytes);
hh_status wy_workspace_size16(hh_op op, const hh_desc *d, size_t *bytes);
// Bytes of the coefficient record of forward op `op` (APPLY, APPLY_T, SYM):
// m rows of 16-bit values over N columns rounded up to 32, m = HP (2 HP for
// the symmetric form); the columns past N are zero.
hh_status wy_saved_size(hh_op op, const hh_desc *d, size_t *bytes);
// saved (nullable, saved_bytes long): the forward also writes the record;
// the backward takes it in place of its own pass over X.
hh_status wy_forward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                     const void *X, int64_t ldx, const void *Xb, int64_t ldb, void *Y,
                     int64_t ldy, void *saved, size_t saved_bytes, void *ws, size_t ws_bytes,
                     hipStream_t st);
hh_status wy_forward16(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                       const void *X, int64_t ldx, const void *Xb, int64_t ldb, void *Y,
                       int64_t ldy, void *saved, size_t saved_bytes, void *ws, size_t ws_bytes,
                       hipStream_t st);
hh_status wy_backward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                      const void *X, int64_t ldx, const void *Xb, int64_t ldb, const void *G,
                      int64_t ldg, void *dX, void *dXb, int64_t lddx, void *dU, int64_t lddu,
                      void *dlam, const void *saved, size_t saved_bytes, void *ws,
                      size_t ws_bytes, hipStream_t st);
hh_status wy_backward16(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                        const void *X, int64_t ldx, const void *Xb, int64_t ldb, const void *G,
                        int64_t ldg, void *dX, void *dXb, int64_t lddx, void *dU, int64_t lddu,
                        void *dlam, const void *saved, size_t saved_bytes, void *ws,
                        size_t ws_bytes, hipStream_t st);

}  // namespace hh

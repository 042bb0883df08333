// Internal interface of the compact-WY path (matrix-core GEMMs).
#pragma once

#include "hh_internal.h"

namespace hh {

hh_status wy_workspace_size(hh_op op, const hh_desc *d, size_t *bytes);
hh_status wy_forward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                     const void *X, int64_t ldx, const void *Xb, int64_t ldb, void *Y,
                     int64_t ldy, void *ws, size_t ws_bytes, hipStream_t st);
hh_status wy_backward(hh_op op, const hh_desc *d, const void *U, int64_t ldu, const void *lam,
                      const void *X, int64_t ldx, const void *Xb, int64_t ldb, const void *G,
                      int64_t ldg, void *dX, void *dXb, int64_t lddx, void *dU, int64_t lddu,
                      void *dlam, void *ws, size_t ws_bytes, hipStream_t st);

}  // namespace hh

// Internal interface of the fused backward kernels.
#pragma once

#include "hh_internal.h"

namespace hh {

struct FusedBwdArgs {
    const void *X;    // X, or Xa for the Mahalanobis op
    int64_t ldx;
    const void *Xb;   // Mahalanobis only
    int64_t ldb;
    const void *G;    // dY, or ddist (N scalars) for the Mahalanobis op
    int64_t ldg;
    void *dX;         // nullable; dXa for the Mahalanobis op
    void *dXb;        // nullable; Mahalanobis only
    int64_t lddx;
    const void *ut, *tau, *lam;
    const double *uh64, *nrm64;
    void *dU;         // nullable
    int64_t lddu;
    void *dlam;       // nullable
    void *scratch;    // per-block partial sums
    const void *din;  // n diagonal entries on the forward's input, or null
    const void *dout; // n diagonal entries on the forward's output, or null
    const void *dots; // Mahalanobis, nullable: the forward's dot products, rows of h padded to 16 bytes
    int n, h, npad;
    int64_t N;
    int vec_ok;
};

bool fused_bwd_plan(hh_dtype t, int64_t n, int64_t h, int64_t N, FusedPlan *p);
bool fused_bwd_supported(hh_op op, const FusedPlan &p);
size_t fused_bwd_ws_bytes(hh_op op, const FusedPlan &p);
hipError_t launch_fused_bwd(const FusedPlan &p, hh_op op, const FusedBwdArgs &a, hipStream_t st);

}  // namespace hh

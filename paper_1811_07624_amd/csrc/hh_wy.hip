// Compact-WY path: placeholder until the matrix-core kernels land.
#include "hh_wy.h"

namespace hh {

hh_status wy_workspace_size(hh_op, const hh_desc *, size_t *) {
    return set_error(HH_ERR_UNSUPPORTED, "WY path not built yet");
}
hh_status wy_forward(hh_op, const hh_desc *, const void *, int64_t, const void *, const void *,
                     int64_t, const void *, int64_t, void *, int64_t, void *, size_t,
                     hipStream_t) {
    return set_error(HH_ERR_UNSUPPORTED, "WY path not built yet");
}
hh_status wy_backward(hh_op, const hh_desc *, const void *, int64_t, const void *, const void *,
                      int64_t, const void *, int64_t, const void *, int64_t, void *, void *,
                      int64_t, void *, int64_t, void *, void *, size_t, hipStream_t) {
    return set_error(HH_ERR_UNSUPPORTED, "WY path not built yet");
}

}  // namespace hh

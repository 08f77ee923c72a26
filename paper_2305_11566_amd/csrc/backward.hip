// Backward pass of the refinement network (placeholder until the kernels land).
#include "net.h"

namespace sv {

size_t net_bwd_workspace(const NetShape &ns, const Levels &lv, int B) {
    (void)ns; (void)lv; (void)B;
    return 0;
}

sv_status net_backward(const NetShape &, const void *, const void *, int, int, int, const float *,
                       const float *, float, float *, void *, hipStream_t) {
    return SV_ERR_UNSUPPORTED;
}

}  // namespace sv

// Instantiates the convolution kernels for one compute dtype.
#include "conv_impl.h"

namespace sv {

sv_status launch_conv_f32(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st) {
    return launch_dt<SV_F32>(ks, stride, cfg, p, pg, st);
}

}  // namespace sv

// Instantiates the 5x5 stride-2 convolution kernels for one compute dtype.
#include "conv_impl.h"

namespace sv {

sv_status launch_conv5_s2_f32(int cfg, const ConvParams &p, int pg, hipStream_t st) {
    return launch_dt5<SV_F32, 2>(cfg, p, pg, st);
}

bool conv5_fits_s2_f32(int tile) { return fits_dt5<SV_F32, 2>(tile); }

}  // namespace sv

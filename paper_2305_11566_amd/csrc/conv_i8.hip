// Instantiates the INT8 convolution kernels (3x3 and 1x1, the configurable network).
#include "conv_impl.h"

namespace sv {

sv_status launch_conv_i8(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st) {
    return launch_dt<SV_I8>(ks, stride, cfg, p, pg, st);
}

bool conv_fits_i8(int ks, int stride, int tile) { return fits_dt<SV_I8>(ks, stride, tile); }

}  // namespace sv

// Instantiates the convolution kernels for one compute dtype.
#include "conv_impl.h"

namespace sv {

sv_status launch_conv_f16(int ks, int stride, int cfg, const ConvParams &p, int pg, hipStream_t st) {
    return launch_dt<SV_F16>(ks, stride, cfg, p, pg, st);
}

bool conv_fits_f16(int ks, int stride, int tile) { return fits_dt<SV_F16>(ks, stride, tile); }

sv_status launch_split_sum_f16(const ConvParams &p, hipStream_t st) { return launch_reduce<SV_F16>(p, st); }

}  // namespace sv

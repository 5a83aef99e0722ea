// Instantiation of the direct-convolution kernel for the JCOL epilogue (all odd P <= 63),
// and of its two-pass form for rank-one stamps.
#include "conv_impl.h"

namespace apx {
hipError_t launch_conv_jcol(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    return launch_conv_kind<CONV_JCOL>(p, L, io, st);
}
hipError_t launch_conv_sep(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    return launch_conv_sep_impl(p, L, io, st);
}
}  // namespace apx

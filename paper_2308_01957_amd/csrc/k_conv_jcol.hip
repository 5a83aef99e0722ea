// Instantiation of the direct-convolution kernel for the JCOL epilogue (all odd P <= 63).
#include "conv_impl.h"

namespace apx {
hipError_t launch_conv_jcol(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    return launch_conv_kind<CONV_JCOL>(p, L, io, st);
}
}  // namespace apx

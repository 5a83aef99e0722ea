// Instantiation of the direct-convolution kernel for the FWD epilogue (all odd P <= 63).
#include "conv_impl.h"

namespace apx {
hipError_t launch_conv_fwd(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    return launch_conv_kind<CONV_FWD>(p, L, io, st);
}
}  // namespace apx

// Instantiation of the direct-convolution kernel for the FP64 objective (forward model,
// residual and chi^2 partials in double precision; all odd P <= 63).
#include "conv_impl.h"

namespace apx {
hipError_t launch_conv_fwd64(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    return launch_conv_kind<CONV_FWD, double>(p, L, io, st);
}
}  // namespace apx

// Instantiation of the direct-convolution kernel for the ADJ epilogue (all odd P <= 63).
#include "conv_impl.h"

namespace apx {
hipError_t launch_conv_adj(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    return launch_conv_kind<CONV_ADJ>(p, L, io, st);
}
}  // namespace apx

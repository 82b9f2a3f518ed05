// Fused last pass + contraction: instantiations for lengths 160, 192
// (shapes of SB_FUSED_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<160>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<160, 8, 4, 4, 2, 5>(a, s);
}

template <> hipError_t launch_last_for<192>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<192, 16, 4, 4, 4, 3>(a, s);
}

}  // namespace sb

// Fused last pass + contraction: instantiations for lengths 512
// (shapes of SB_FUSED_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<512>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<512, 64, 8, 8, 8>(a, s);
}

}  // namespace sb

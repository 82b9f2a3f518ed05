// Fused last pass + contraction: instantiations for lengths 512.
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<512>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<512, 32, 8, 8, 8>(a, s);
}

}  // namespace sb

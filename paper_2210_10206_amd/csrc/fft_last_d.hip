// Fused last pass + contraction: instantiations for lengths 256.
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<256>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<256, 16, 8, 8, 4>(a, s);
}

}  // namespace sb

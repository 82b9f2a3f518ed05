// Fused last pass + contraction: instantiations for lengths 160, 192.
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<160>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<160, 4, 4, 8, 5>(a, s);
}

template <> hipError_t launch_last_for<192>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<192, 8, 8, 8, 3>(a, s);
}

}  // namespace sb

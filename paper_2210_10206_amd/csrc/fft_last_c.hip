// Fused last pass + contraction: instantiations for lengths 160, 192
// (shapes of SB_LAST_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<160>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<160, 8, 4, 4, 2, 5>(a, s);
}
template <> int last_rows<160>(int nb) { return fftlast::last_rows_for<160, 8>(nb); }

template <> hipError_t launch_last_for<192>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<192, 16, 4, 4, 4, 3>(a, s);
}
template <> int last_rows<192>(int nb) { return fftlast::last_rows_for<192, 16>(nb); }

}  // namespace sb

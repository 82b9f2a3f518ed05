// Fused last pass + contraction: instantiations for lengths 256
// (shapes of SB_LAST_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<256>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<256, 32, 8, 8, 4>(a, s);
}
template <> int last_rows<256>(int nb) { return fftlast::last_rows_for<256, 32>(nb); }

}  // namespace sb

// Fused last pass + contraction: instantiations for lengths 512
// (shapes of SB_LAST_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<512>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<512, 32, 8, 8, 8>(a, s);
}
template <> int last_rows<512>(int nb) { return fftlast::last_rows_for<512, 32>(nb); }

}  // namespace sb

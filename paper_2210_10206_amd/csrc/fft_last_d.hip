// Fused last pass + contraction: instantiations for lengths 256
// (shapes of SB_LAST_CONFIGS).
#include "fft_last.h"

namespace sb {

// 256 = 16 x 16: the register-resident form, one row per tile
template <> hipError_t launch_last_for<256>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_reg<16, 16>(a, s);
}
template <> int last_rows<256>(int nb) { return nb <= 16 ? 1 : 0; }

}  // namespace sb

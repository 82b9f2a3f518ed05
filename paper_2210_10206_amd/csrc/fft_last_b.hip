// Fused last pass + contraction: instantiations for lengths 64, 96, 128
// (all three register-resident).
#include "fft_last.h"

namespace sb {

// 64 = 8 x 8 and 128 = 16 x 8: the register-resident form, one row per tile
template <> hipError_t launch_last_for<64>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_reg<8, 8>(a, s);
}
template <> int last_rows<64>(int nb) { return nb <= 16 ? 1 : 0; }

template <> hipError_t launch_last_for<96>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_rs<96, 12, 4, 2>(a, s);
}
template <> int last_rows<96>(int nb) { return nb <= 16 ? 1 : 0; }

template <> hipError_t launch_last_for<128>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_reg<16, 8>(a, s);
}
template <> int last_rows<128>(int nb) { return nb <= 16 ? 1 : 0; }

}  // namespace sb

// Fused last pass + contraction: instantiations for lengths 64, 96, 128
// (shapes of SB_LAST_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<64>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<64, 8, 8, 8>(a, s);
}
template <> int last_rows<64>(int nb) { return fftlast::last_rows_for<64, 8>(nb); }

template <> hipError_t launch_last_for<96>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<96, 8, 4, 4, 2, 3>(a, s);
}
template <> int last_rows<96>(int nb) { return fftlast::last_rows_for<96, 8>(nb); }

template <> hipError_t launch_last_for<128>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<128, 16, 8, 8, 2>(a, s);
}
template <> int last_rows<128>(int nb) { return fftlast::last_rows_for<128, 16>(nb); }

}  // namespace sb

// Fused last pass + contraction: instantiations for lengths 8, 12, 16, 24, 32, 48
// (shapes of SB_LAST_CONFIGS).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<8>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<8, 1, 8>(a, s);
}
template <> int last_rows<8>(int nb) { return fftlast::last_rows_for<8, 1>(nb); }

template <> hipError_t launch_last_for<12>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<12, 1, 4, 3>(a, s);
}
template <> int last_rows<12>(int nb) { return fftlast::last_rows_for<12, 1>(nb); }

template <> hipError_t launch_last_for<16>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<16, 4, 4, 4>(a, s);
}
template <> int last_rows<16>(int nb) { return fftlast::last_rows_for<16, 4>(nb); }

template <> hipError_t launch_last_for<24>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<24, 2, 4, 2, 3>(a, s);
}
template <> int last_rows<24>(int nb) { return fftlast::last_rows_for<24, 2>(nb); }

template <> hipError_t launch_last_for<32>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<32, 4, 4, 8>(a, s);
}
template <> int last_rows<32>(int nb) { return fftlast::last_rows_for<32, 4>(nb); }

template <> hipError_t launch_last_for<48>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<48, 4, 4, 4, 3>(a, s);
}
template <> int last_rows<48>(int nb) { return fftlast::last_rows_for<48, 4>(nb); }

}  // namespace sb

// Fused last pass + contraction: instantiations for lengths 512 and 1024 (shapes of
// SB_LAST_CONFIGS; 1024 = 16 x 16 x 4 register-resident stages, 64 threads per pencil).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<512>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_nb<512, 32, 8, 8, 8>(a, s);
}
template <> int last_rows<512>(int nb) { return fftlast::last_rows_for<512, 32>(nb); }

template <> hipError_t launch_last_for<1024>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_rs<1024, 16, 16, 4>(a, s);
}
template <> int last_rows<1024>(int nb) { return nb <= 12 ? 1 : 0; }   // 16-bin tiles would spill

}  // namespace sb

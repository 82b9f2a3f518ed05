// Fused last pass + contraction: instantiations for lengths 160, 192 (register-resident
// stages: 160 = 20 x 4 x 2, 192 = 12 x 4 x 4).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<160>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_rs<160, 20, 4, 2>(a, s);
}
template <> int last_rows<160>(int nb) { return nb <= 16 ? 1 : 0; }

template <> hipError_t launch_last_for<192>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_rs<192, 12, 4, 4>(a, s);
}
template <> int last_rows<192>(int nb) { return nb <= 16 ? 1 : 0; }

}  // namespace sb

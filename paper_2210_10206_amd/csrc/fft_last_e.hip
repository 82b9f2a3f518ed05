// Fused last pass + contraction: instantiations for lengths 512 and 1024, both register-resident
// with the skewed LDS layout (512 = 16 x 8 x 4 stages, 32 threads per pencil, up to 16 bins;
// 1024 = 16 x 16 x 4 stages, 64 threads per pencil, up to 12 bins).
#include "fft_last.h"

namespace sb {

template <> hipError_t launch_last_for<512>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_rs<512, 16, 8, 4>(a, s);
}
template <> int last_rows<512>(int nb) { return nb <= 16 ? 1 : 0; }

template <> hipError_t launch_last_for<1024>(const LastArgs &a, hipStream_t s) {
    return fftlast::launch_last_rs<1024, 16, 16, 4>(a, s);
}
template <> int last_rows<1024>(int nb) { return nb <= 12 ? 1 : 0; }   // 16-bin tiles would spill

}  // namespace sb

// Matrix-core 4PCF contraction: ordered Lambdas (both parities) with l1 in {0, 1}.
#include "quad_mfma.h"

namespace sb {

hipError_t launch_quad_mfma_part0(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s) {
    const int key = la * 100 + lb * 10 + lc;
    switch (key) {
        case 0: return quadm::launch_lambda<0, 0, 0>(a, s);
        case 11: return quadm::launch_lambda<0, 1, 1>(a, s);
        case 22: return quadm::launch_lambda<0, 2, 2>(a, s);
        case 33: return quadm::launch_lambda<0, 3, 3>(a, s);
        case 44: return quadm::launch_lambda<0, 4, 4>(a, s);
        case 101: return quadm::launch_lambda<1, 0, 1>(a, s);
        case 110: return quadm::launch_lambda<1, 1, 0>(a, s);
        case 111: return quadm::launch_lambda<1, 1, 1>(a, s);
        case 112: return quadm::launch_lambda<1, 1, 2>(a, s);
        case 121: return quadm::launch_lambda<1, 2, 1>(a, s);
        case 122: return quadm::launch_lambda<1, 2, 2>(a, s);
        case 123: return quadm::launch_lambda<1, 2, 3>(a, s);
        case 132: return quadm::launch_lambda<1, 3, 2>(a, s);
        case 133: return quadm::launch_lambda<1, 3, 3>(a, s);
        case 134: return quadm::launch_lambda<1, 3, 4>(a, s);
        case 143: return quadm::launch_lambda<1, 4, 3>(a, s);
        case 144: return quadm::launch_lambda<1, 4, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sb

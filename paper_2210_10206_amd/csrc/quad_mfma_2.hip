// Matrix-core 4PCF contraction: ordered Lambdas (both parities) with l1 in {4}.
#include "quad_mfma.h"

namespace sb {

hipError_t launch_quad_mfma_part2(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s) {
    const int key = la * 100 + lb * 10 + lc;
    switch (key) {
        case 404: return quadm::launch_lambda<4, 0, 4>(a, s);
        case 413: return quadm::launch_lambda<4, 1, 3>(a, s);
        case 414: return quadm::launch_lambda<4, 1, 4>(a, s);
        case 422: return quadm::launch_lambda<4, 2, 2>(a, s);
        case 423: return quadm::launch_lambda<4, 2, 3>(a, s);
        case 424: return quadm::launch_lambda<4, 2, 4>(a, s);
        case 431: return quadm::launch_lambda<4, 3, 1>(a, s);
        case 432: return quadm::launch_lambda<4, 3, 2>(a, s);
        case 433: return quadm::launch_lambda<4, 3, 3>(a, s);
        case 434: return quadm::launch_lambda<4, 3, 4>(a, s);
        case 440: return quadm::launch_lambda<4, 4, 0>(a, s);
        case 441: return quadm::launch_lambda<4, 4, 1>(a, s);
        case 442: return quadm::launch_lambda<4, 4, 2>(a, s);
        case 443: return quadm::launch_lambda<4, 4, 3>(a, s);
        case 444: return quadm::launch_lambda<4, 4, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sb

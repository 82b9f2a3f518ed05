// Matrix-core 4PCF contraction: ordered Lambdas (both parities) with l1 in {2, 3}.
#include "quad_mfma.h"

namespace sb {

hipError_t launch_quad_mfma_part1(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s) {
    const int key = la * 100 + lb * 10 + lc;
    switch (key) {
        case 202: return quadm::launch_lambda<2, 0, 2>(a, s);
        case 211: return quadm::launch_lambda<2, 1, 1>(a, s);
        case 212: return quadm::launch_lambda<2, 1, 2>(a, s);
        case 213: return quadm::launch_lambda<2, 1, 3>(a, s);
        case 220: return quadm::launch_lambda<2, 2, 0>(a, s);
        case 221: return quadm::launch_lambda<2, 2, 1>(a, s);
        case 222: return quadm::launch_lambda<2, 2, 2>(a, s);
        case 223: return quadm::launch_lambda<2, 2, 3>(a, s);
        case 224: return quadm::launch_lambda<2, 2, 4>(a, s);
        case 231: return quadm::launch_lambda<2, 3, 1>(a, s);
        case 232: return quadm::launch_lambda<2, 3, 2>(a, s);
        case 233: return quadm::launch_lambda<2, 3, 3>(a, s);
        case 234: return quadm::launch_lambda<2, 3, 4>(a, s);
        case 242: return quadm::launch_lambda<2, 4, 2>(a, s);
        case 243: return quadm::launch_lambda<2, 4, 3>(a, s);
        case 244: return quadm::launch_lambda<2, 4, 4>(a, s);
        case 303: return quadm::launch_lambda<3, 0, 3>(a, s);
        case 312: return quadm::launch_lambda<3, 1, 2>(a, s);
        case 313: return quadm::launch_lambda<3, 1, 3>(a, s);
        case 314: return quadm::launch_lambda<3, 1, 4>(a, s);
        case 321: return quadm::launch_lambda<3, 2, 1>(a, s);
        case 322: return quadm::launch_lambda<3, 2, 2>(a, s);
        case 323: return quadm::launch_lambda<3, 2, 3>(a, s);
        case 324: return quadm::launch_lambda<3, 2, 4>(a, s);
        case 330: return quadm::launch_lambda<3, 3, 0>(a, s);
        case 331: return quadm::launch_lambda<3, 3, 1>(a, s);
        case 332: return quadm::launch_lambda<3, 3, 2>(a, s);
        case 333: return quadm::launch_lambda<3, 3, 3>(a, s);
        case 334: return quadm::launch_lambda<3, 3, 4>(a, s);
        case 341: return quadm::launch_lambda<3, 4, 1>(a, s);
        case 342: return quadm::launch_lambda<3, 4, 2>(a, s);
        case 343: return quadm::launch_lambda<3, 4, 3>(a, s);
        case 344: return quadm::launch_lambda<3, 4, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sb

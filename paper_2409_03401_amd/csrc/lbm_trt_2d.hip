// 2D families with the two-relaxation-time collision: D2Q5 or the paper's D2Q9
// for g, h^A, h^B, with or without the D2Q9 fluid; all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_trt_2d(int scalar, int fluid, int prec) {
    if (scalar == 5) {
        if (fluid == 0) return family_all_prec_noadj<D2Q5K, NoLattice, 256, 1, COLL_TRT>(prec);
        if (fluid == 9) return family_all_prec_noadj<D2Q5K, D2Q9K, 256, 1, COLL_TRT>(prec);
    } else if (scalar == 9) {
        if (fluid == 0) return family_all_prec_noadj<D2Q9K, NoLattice, 256, 1, COLL_TRT>(prec);
        if (fluid == 9) return family_all_prec_noadj<D2Q9K, D2Q9K, 256, 1, COLL_TRT>(prec);
    }
    return nullptr;
}

}  // namespace lbm

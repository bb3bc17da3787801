// 3D families with the two-relaxation-time collision: D3Q7 or the paper's D3Q19
// for g, h^A, h^B, with or without the D3Q19 fluid; all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_trt_3d(int scalar, int fluid, int prec) {
    if (scalar == 7) {
        if (fluid == 0) return family_all_prec_noadj<D3Q7K, NoLattice, 64, 4, COLL_TRT>(prec);
        if (fluid == 19) return family_all_prec_noadj<D3Q7K, D3Q19K, 64, 4, COLL_TRT>(prec);
    } else if (scalar == 19) {
        if (fluid == 0) return family_all_prec_noadj<D3Q19K, NoLattice, 64, 4, COLL_TRT>(prec);
        if (fluid == 19) return family_all_prec_noadj<D3Q19K, D3Q19K, 64, 4, COLL_TRT>(prec);
    }
    return nullptr;
}

}  // namespace lbm

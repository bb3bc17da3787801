// 3D families of the variable-density flow model: D3Q19 fluid with D3Q7 or D3Q19
// scalars, BGK or TRT collision; all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_vd_3d(int scalar, bool trt, int prec) {
    if (scalar == 7)
        return trt ? family_all_prec_noadj<D3Q7K, D3Q19K, 64, 4, COLL_VD | COLL_TRT>(prec)
                   : family_all_prec_noadj<D3Q7K, D3Q19K, 64, 4, COLL_VD>(prec);
    if (scalar == 19)
        return trt ? family_all_prec_noadj<D3Q19K, D3Q19K, 64, 4, COLL_VD | COLL_TRT>(prec)
                   : family_all_prec_noadj<D3Q19K, D3Q19K, 64, 4, COLL_VD>(prec);
    return nullptr;
}

}  // namespace lbm

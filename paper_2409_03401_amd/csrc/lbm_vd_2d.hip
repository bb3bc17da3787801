// 2D families of the variable-density flow model (rho(phi) in the inertia, pressure
// and viscous forces): D2Q9 fluid with D2Q5 or D2Q9 scalars, BGK or TRT collision;
// all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_vd_2d(int scalar, bool trt, int prec) {
    if (scalar == 5)
        return trt ? family_all_prec_noadj<D2Q5K, D2Q9K, 256, 1, COLL_VD | COLL_TRT>(prec)
                   : family_all_prec_noadj<D2Q5K, D2Q9K, 256, 1, COLL_VD>(prec);
    if (scalar == 9)
        return trt ? family_all_prec_noadj<D2Q9K, D2Q9K, 256, 1, COLL_VD | COLL_TRT>(prec)
                   : family_all_prec_noadj<D2Q9K, D2Q9K, 256, 1, COLL_VD>(prec);
    return nullptr;
}

}  // namespace lbm

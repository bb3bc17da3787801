// 2D families with general curvature matrices of the free energies (2 x 2 closure
// per node): D2Q5 or D2Q9 scalars, with or without the D2Q9 fluid; BGK, Boussinesq;
// all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_gk_2d(int scalar, int fluid, int prec) {
    if (scalar == 5) {
        if (fluid == 0) return family_all_prec_noadj<D2Q5K, NoLattice, 256, 1, COLL_GK>(prec);
        if (fluid == 9) return family_all_prec_noadj<D2Q5K, D2Q9K, 256, 1, COLL_GK>(prec);
    } else if (scalar == 9) {
        if (fluid == 0) return family_all_prec_noadj<D2Q9K, NoLattice, 256, 1, COLL_GK>(prec);
        if (fluid == 9) return family_all_prec_noadj<D2Q9K, D2Q9K, 256, 1, COLL_GK>(prec);
    }
    return nullptr;
}

}  // namespace lbm

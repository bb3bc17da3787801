// 3D families with general curvature matrices of the free energies: D3Q7 or D3Q19
// scalars, with or without the D3Q19 fluid; BGK, Boussinesq; all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_gk_3d(int scalar, int fluid, int prec) {
    if (scalar == 7) {
        if (fluid == 0) return family_all_prec_noadj<D3Q7K, NoLattice, 64, 4, COLL_GK>(prec);
        if (fluid == 19) return family_all_prec_noadj<D3Q7K, D3Q19K, 64, 4, COLL_GK>(prec);
    } else if (scalar == 19) {
        if (fluid == 0) return family_all_prec_noadj<D3Q19K, NoLattice, 64, 4, COLL_GK>(prec);
        if (fluid == 19) return family_all_prec_noadj<D3Q19K, D3Q19K, 64, 4, COLL_GK>(prec);
    }
    return nullptr;
}

}  // namespace lbm

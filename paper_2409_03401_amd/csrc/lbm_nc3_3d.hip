// A third independent composition (N components, the conclusion's extension with the
// quadratic free energies of Eq. Taylor) in 3D: D3Q7 for phi and the three compositions,
// with or without the D3Q19 fluid; BGK Boussinesq step, all four storage precisions,
// 64 x 4 node columns per work-group.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_nc3_3d(int fluid, int prec) {
    if (fluid == 0) return family_nc3<D3Q7K, NoLattice, 64, 4>(prec);
    if (fluid == 19) return family_nc3<D3Q7K, D3Q19K, 64, 4>(prec);
    return nullptr;
}

}  // namespace lbm

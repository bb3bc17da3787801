// A third independent composition (N components, the conclusion's extension with the
// quadratic free energies of Eq. Taylor) in 2D: D2Q5 for phi and the three compositions,
// with or without the D2Q9 fluid; BGK Boussinesq step, all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_nc3_2d(int fluid, int prec) {
    if (fluid == 0) return family_nc3<D2Q5K, NoLattice, 256, 1>(prec);
    if (fluid == 9) return family_nc3<D2Q5K, D2Q9K, 256, 1>(prec);
    return nullptr;
}

}  // namespace lbm

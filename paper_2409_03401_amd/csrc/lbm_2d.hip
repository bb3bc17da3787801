// 2D lattice families (D2Q5 scalars, optional D2Q9 fluid), run in the x-z plane
// of the kernel frame with one row of 64 nodes per work-group.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_2d(int fluid, int prec) {
    if (fluid == 0) return family_for_prec<D2Q5K, NoLattice, 64, 1>(prec);
    if (fluid == 9) return family_for_prec<D2Q5K, D2Q9K, 64, 1>(prec);
    return nullptr;
}

}  // namespace lbm

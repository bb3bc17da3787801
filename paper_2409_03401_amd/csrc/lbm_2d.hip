// 2D lattice families (D2Q5 scalars, optional D2Q9 fluid), run in the x-z plane
// of the kernel frame with one row segment of TX nodes per work-group.  256 nodes by
// default (against 64: +11% on a 512^2 droplet with flow, +3-4% on a 4096^2 ripening
// box); 64 and 128 stay selectable for tuning.
#include "family.hpp"

namespace lbm {

template <class FL>
static const KernelSet* by_tile(int prec, int tx) {
    switch (tx) {
        case 64: return family_for_prec<D2Q5K, FL, 64, 1>(prec);
        case 128: return family_for_prec<D2Q5K, FL, 128, 1>(prec);
        default: return family_for_prec<D2Q5K, FL, 256, 1>(prec);
    }
}

const KernelSet* kernels_2d(int fluid, int prec, int tx) {
    if (fluid == 0) return by_tile<NoLattice>(prec, tx);
    if (fluid == 9) return by_tile<D2Q9K>(prec, tx);
    return nullptr;
}

}  // namespace lbm

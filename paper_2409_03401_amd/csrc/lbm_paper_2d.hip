// The paper's own 2D discretisation: D2Q9 for phi and both compositions (Section 3
// uses the fluid's velocity set for every equation), with or without the D2Q9 fluid.
// All four storage precisions, the adjoint at FP64 / FP32; one row of 64 nodes per
// work-group.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_paper_2d(int fluid, int prec) {
    if (fluid == 0) return family_for_prec<D2Q9K, NoLattice, 64, 1>(prec);
    if (fluid == 9) return family_for_prec<D2Q9K, D2Q9K, 64, 1>(prec);
    return nullptr;
}

}  // namespace lbm

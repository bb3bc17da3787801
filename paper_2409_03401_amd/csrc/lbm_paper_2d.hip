// The paper's own 2D discretisation: D2Q9 for phi and both compositions (Section 3
// uses the fluid's velocity set for every equation), with or without the D2Q9 fluid.
// All four storage precisions, the adjoint at FP64 / FP32; a row segment of 256 nodes
// per work-group (on the 4096^2 box: +8% FP32, +10% BF16 storage over 64 nodes, from
// fewer lines pulled across segment edges).
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_paper_2d(int fluid, int prec) {
    if (fluid == 0) return family_for_prec<D2Q9K, NoLattice, 256, 1>(prec);
    if (fluid == 9) return family_for_prec<D2Q9K, D2Q9K, 256, 1>(prec);
    return nullptr;
}

}  // namespace lbm

// The paper's own 3D discretisation: D3Q19 for phi and both compositions (Section 3),
// with or without the D3Q19 fluid.  All four storage precisions, the adjoint at
// FP64 / FP32; 64 x 4 node columns per work-group.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_paper_3d(int fluid, int prec) {
    if (fluid == 0) return family_for_prec<D3Q19K, NoLattice, 64, 4>(prec);
    if (fluid == 19) return family_for_prec<D3Q19K, D3Q19K, 64, 4>(prec);
    return nullptr;
}

}  // namespace lbm

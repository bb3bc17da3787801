// MRT, D3Q19 scalars with the D3Q19 fluid: FP16 and BF16 storage of the moving
// populations.
#include "family.hpp"

namespace lbm {

const KernelSet* mrt3d_q19_flow_16(int prec) {
    if (prec == P16) return family_one_prec<D3Q19K, D3Q19K, 64, 4, COLL_MRT, P16>();
    if (prec == PB16) return family_one_prec<D3Q19K, D3Q19K, 64, 4, COLL_MRT, PB16>();
    return nullptr;
}

}  // namespace lbm

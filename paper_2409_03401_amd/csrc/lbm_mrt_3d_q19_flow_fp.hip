// MRT, D3Q19 scalars with the D3Q19 fluid: FP64 and FP32 storage.
#include "family.hpp"

namespace lbm {

const KernelSet* mrt3d_q19_flow_fp(int prec) {
    if (prec == P64) return family_one_prec<D3Q19K, D3Q19K, 64, 4, COLL_MRT, P64>();
    if (prec == P32) return family_one_prec<D3Q19K, D3Q19K, 64, 4, COLL_MRT, P32>();
    return nullptr;
}

}  // namespace lbm

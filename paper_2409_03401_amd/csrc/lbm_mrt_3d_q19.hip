// MRT, D3Q19 scalars without a fluid: all four storage precisions.
#include "family.hpp"

namespace lbm {

const KernelSet* mrt3d_q19(int, int prec) { return family_all_prec_noadj<D3Q19K, NoLattice, 64, 4, COLL_MRT>(prec); }

}  // namespace lbm

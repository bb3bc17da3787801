// 3D families with the multiple-relaxation-time collision: D3Q7 or the paper's D3Q19
// for g, h^A, h^B, with or without the D3Q19 fluid; all four storage precisions.  The
// D3Q19 families are compiled in translation units of their own (lbm_mrt_3d_*.hip).
#include "family.hpp"

namespace lbm {

const KernelSet* mrt3d_q19(int fluid, int prec);
const KernelSet* mrt3d_q19_flow_fp(int prec);
const KernelSet* mrt3d_q19_flow_16(int prec);

const KernelSet* kernels_mrt_3d(int scalar, int fluid, int prec) {
    if (scalar == 7) {
        if (fluid == 0) return family_all_prec_noadj<D3Q7K, NoLattice, 64, 4, COLL_MRT>(prec);
        if (fluid == 19) return family_all_prec_noadj<D3Q7K, D3Q19K, 64, 4, COLL_MRT>(prec);
    } else if (scalar == 19) {
        if (fluid == 0) return mrt3d_q19(fluid, prec);
        if (fluid == 19) return (prec == P64 || prec == P32) ? mrt3d_q19_flow_fp(prec) : mrt3d_q19_flow_16(prec);
    }
    return nullptr;
}

}  // namespace lbm

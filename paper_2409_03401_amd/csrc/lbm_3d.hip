// 3D lattice families (D3Q7 scalars, optional D3Q19 fluid) with 32 x 8 node
// columns per work-group.
#include "family.hpp"

namespace lbm {

const KernelSet* kernels_3d(int fluid, int prec) {
    if (fluid == 0) return family_for_prec<D3Q7K, NoLattice, 32, 8>(prec);
    if (fluid == 19) return family_for_prec<D3Q7K, D3Q19K, 32, 8>(prec);
    return nullptr;
}

void launch_sum_partials(const double* v, long long n, double* partials, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_sum_partials<256>), dim3(nblocks), dim3(256), 0, s, v, n, partials);
}

void launch_finalize(const double* partials, int nparts, int width, int maxslot, double scale0,
                     double* out, hipStream_t s) {
    if (width == 1)
        hipLaunchKernelGGL((k_finalize<1>), dim3(1), dim3(256), 0, s, partials, nparts, maxslot, scale0, out);
    else
        hipLaunchKernelGGL((k_finalize<8>), dim3(1), dim3(256), 0, s, partials, nparts, maxslot, scale0, out);
}

}  // namespace lbm

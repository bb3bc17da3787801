// 3D lattice families (D3Q7 scalars, optional D3Q19 fluid) with 64 x 4 node
// columns per work-group (32 x 8 on request).
#include "family.hpp"

namespace lbm {

template <class FL>
static const KernelSet* by_tile(int prec, int tx, int ty) {
    if (tx == 32 && ty == 8) return family_for_prec<D3Q7K, FL, 32, 8>(prec);
    return family_for_prec<D3Q7K, FL, 64, 4>(prec);
}

const KernelSet* kernels_3d(int fluid, int prec, int tx, int ty) {
    if (fluid == 0) return by_tile<NoLattice>(prec, tx, ty);
    if (fluid == 19) return by_tile<D3Q19K>(prec, tx, ty);
    return nullptr;
}

void launch_sum_partials(const double* v, long long n, double* partials, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_sum_partials<256>), dim3(nblocks), dim3(256), 0, s, v, n, partials);
}

void launch_finalize(const double* partials, int nparts, int width, int maxslot, double scale0,
                     double* out, hipStream_t s) {
    if (width == 1)
        hipLaunchKernelGGL((k_finalize<1>), dim3(1), dim3(256), 0, s, partials, nparts, maxslot, scale0, out);
    else if (width == 9)
        hipLaunchKernelGGL((k_finalize<9, false, 10>), dim3(1), dim3(256), 0, s, partials, nparts, maxslot, scale0,
                           out);
    else
        hipLaunchKernelGGL((k_finalize<8>), dim3(1), dim3(256), 0, s, partials, nparts, maxslot, scale0, out);
}

void launch_sum6(const double* partials, int nparts, double* out, bool accumulate, hipStream_t s) {
    if (accumulate)
        hipLaunchKernelGGL((k_finalize<6, true>), dim3(1), dim3(256), 0, s, partials, nparts, -1, 1.0, out);
    else
        hipLaunchKernelGGL((k_finalize<6, false>), dim3(1), dim3(256), 0, s, partials, nparts, -1, 1.0, out);
}

void launch_euler(const unsigned char* mask, const EulerGeom& g, double* partials, int nblocks, hipStream_t s) {
    if (g.d == 3) hipLaunchKernelGGL((k_euler<3>), dim3(nblocks), dim3(256), 0, s, mask, g, partials);
    else hipLaunchKernelGGL((k_euler<2>), dim3(nblocks), dim3(256), 0, s, mask, g, partials);
}

void launch_zero(double* p, long long n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL((k_zero_f64<256>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, n);
}

}  // namespace lbm

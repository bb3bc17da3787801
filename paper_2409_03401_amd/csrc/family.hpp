// Instantiation helper: the launchers of one (scalar lattice, fluid lattice,
// collision / model variant, number of independent compositions) family for the four
// storage precisions.
#pragma once

#include "dispatch.hpp"
#include "kernels.hpp"

namespace lbm {

template <class SL, class FL, int PREC, int TX, int TY, bool ADJ = true, int COLL = COLL_BGK, int NC = 2>
struct Family {
    static void fused(int mode, dim3 grid, const KParams& kp, hipStream_t s) {
        const dim3 block(TX, TY);
        switch (mode) {
            case MODE_STEP:
                hipLaunchKernelGGL((k_lbm<SL, FL, MODE_STEP, PREC, TX, TY, COLL, NC>), grid, block, 0, s, kp);
                break;
            case MODE_STEP_PHI:
                if constexpr (NC == 2)
                    hipLaunchKernelGGL((k_lbm<SL, FL, MODE_STEP_PHI, PREC, TX, TY, COLL>), grid, block, 0, s, kp);
                break;
            case MODE_MOMENTS:
                hipLaunchKernelGGL((k_lbm<SL, FL, MODE_MOMENTS, PREC, TX, TY, (COLL & (COLL_VD | COLL_GK)), NC>), grid,
                                   block, 0, s, kp);
                break;
            default:
                hipLaunchKernelGGL((k_lbm<SL, FL, MODE_DIAG, PREC, TX, TY, (COLL & (COLL_VD | COLL_GK)), NC>), grid,
                                   block, 0, s, kp);
                break;
        }
    }
    static void init(const KParams& kp, const double* phi0, const double* muA0, const double* muB0,
                     const double* muC0, hipStream_t s) {
        const dim3 grid((kp.nx + 255) / 256, kp.ny, kp.nz);
        hipLaunchKernelGGL((k_init<SL, FL, PREC, NC>), grid, dim3(256), 0, s, kp, phi0, muA0, muB0, muC0);
    }
    static void get_pops(const KParams& kp, int, long long nodes, double* out, hipStream_t s) {
        const dim3 grid(unsigned((nodes + 255) / 256));
        hipLaunchKernelGGL((k_pops<SL, FL, PREC, false, NC>), grid, dim3(256), 0, s, kp, nodes, out);
    }
    static void set_pops(const KParams& kp, int, long long nodes, const double* in, hipStream_t s) {
        const dim3 grid(unsigned((nodes + 255) / 256));
        hipLaunchKernelGGL((k_pops<SL, FL, PREC, true, NC>), grid, dim3(256), 0, s, kp, nodes,
                           const_cast<double*>(in));
    }
    static void walls(const KParams& kp, int axis, hipStream_t s) {
        const long long n[3] = {kp.nx, kp.ny, kp.nz};
        const long long face = n[axis == 0 ? 1 : 0] * n[axis == 2 ? 1 : 2];
        const dim3 grid(unsigned((2 * face + 255) / 256));
        hipLaunchKernelGGL((k_walls<SL, FL, PREC, NC>), grid, dim3(256), 0, s, kp, axis);
    }
    // the adjoint covers the ternary fluid (two compositions) at FP64 / FP32
    static constexpr bool kAdj = ADJ && NC == 2 && (PREC == P32 || PREC == P64);
    static void adj_step(const KParams& kp, long long nodes, const void* phi, hipStream_t s) {
        if constexpr (kAdj)
            hipLaunchKernelGGL((k_adj_node<SL, FL, PREC>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s, kp,
                               nodes, static_cast<const typename Stor<PREC>::C*>(phi));
    }
    static void adj_seed(const KParams& kp, long long nodes, const double* dL_dphi, hipStream_t s) {
        if constexpr (kAdj)
            hipLaunchKernelGGL((k_adj_seed<SL, FL, PREC>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s,
                               kp, nodes, dL_dphi);
    }
    static void adj_gather(const KParams& kp, long long nodes, int mode, double* grad_phi0, hipStream_t s) {
        const dim3 grid(unsigned((nodes + 255) / 256));
        if constexpr (kAdj) {
            if (mode == 0) hipLaunchKernelGGL((k_adj_gather<SL, FL, 0>), grid, dim3(256), 0, s, kp, nodes, grad_phi0);
            else hipLaunchKernelGGL((k_adj_gather<SL, FL, 1>), grid, dim3(256), 0, s, kp, nodes, grad_phi0);
        }
    }
    static void adj_init_local(const KParams& kp, long long nodes, const double* phi0, const double* muA0,
                               const double* muB0, hipStream_t s) {
        if constexpr (kAdj)
            hipLaunchKernelGGL((k_adj_init_local<SL, FL>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s,
                               kp, nodes, phi0, muA0, muB0);
    }
    static void adj_copy(const KParams& kp, int nslots, long long nodes, double* buf, bool set_, hipStream_t s) {
        const dim3 grid(unsigned((nodes + 255) / 256), nslots);
        if constexpr (kAdj) {
            if (set_) hipLaunchKernelGGL((k_adj_copy<SL, FL, true>), grid, dim3(256), 0, s, kp, nodes, buf);
            else hipLaunchKernelGGL((k_adj_copy<SL, FL, false>), grid, dim3(256), 0, s, kp, nodes, buf);
        }
    }
    static constexpr KernelSet set{&fused, &init, &get_pops, &set_pops, &walls,
                                   kAdj ? &adj_step : nullptr, kAdj ? &adj_seed : nullptr,
                                   kAdj ? &adj_gather : nullptr, kAdj ? &adj_init_local : nullptr,
                                   kAdj ? &adj_copy : nullptr, TX, TY};
};

template <class SL, class FL, int TX, int TY>
const KernelSet* family_for_prec(int prec) {
    switch (prec) {
        case P64: return &Family<SL, FL, P64, TX, TY>::set;
        case P32: return &Family<SL, FL, P32, TX, TY>::set;
        case P16: return &Family<SL, FL, P16, TX, TY>::set;
        case PB16: return &Family<SL, FL, PB16, TX, TY>::set;
        default: return nullptr;
    }
}

// the TRT / MRT collisions, the variable-density model and general curvatures: all
// four storage precisions, no adjoint
template <class SL, class FL, int TX, int TY, int COLL = COLL_BGK>
const KernelSet* family_all_prec_noadj(int prec) {
    switch (prec) {
        case P64: return &Family<SL, FL, P64, TX, TY, false, COLL>::set;
        case P32: return &Family<SL, FL, P32, TX, TY, false, COLL>::set;
        case P16: return &Family<SL, FL, P16, TX, TY, false, COLL>::set;
        case PB16: return &Family<SL, FL, PB16, TX, TY, false, COLL>::set;
        default: return nullptr;
    }
}

// a third independent composition (N components): BGK Boussinesq step, all four
// storage precisions, no adjoint
template <class SL, class FL, int TX, int TY>
const KernelSet* family_nc3(int prec) {
    switch (prec) {
        case P64: return &Family<SL, FL, P64, TX, TY, false, COLL_BGK, 3>::set;
        case P32: return &Family<SL, FL, P32, TX, TY, false, COLL_BGK, 3>::set;
        case P16: return &Family<SL, FL, P16, TX, TY, false, COLL_BGK, 3>::set;
        case PB16: return &Family<SL, FL, PB16, TX, TY, false, COLL_BGK, 3>::set;
        default: return nullptr;
    }
}

// one precision of a family without adjoint (for splitting large families over
// translation units)
template <class SL, class FL, int TX, int TY, int COLL, int PREC>
const KernelSet* family_one_prec() {
    return &Family<SL, FL, PREC, TX, TY, false, COLL>::set;
}

}  // namespace lbm

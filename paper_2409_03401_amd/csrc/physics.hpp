// Thermodynamics of the model (Section 2) and the node moments of Section 3,
// shared by the step, adjoint and initialisation kernels.
#pragma once

#include "params.hpp"

namespace lbm {


__device__ __forceinline__ double interp_p(double f) { return f * f * (3.0 - 2.0 * f); }
__device__ __forceinline__ double interp_dp(double f) { return 6.0 * f * (1.0 - f); }
__device__ __forceinline__ double dwell(double f) { return 8.0 * f * f * (1.0 - f) * (1.0 - f); }
__device__ __forceinline__ double dwell_d(double f) { return 16.0 * f * (1.0 - f) * (1.0 - 2.0 * f); }

struct Scalars {
    double phi, muA, muB, S;
};

// Potentials from compositions, Eq. PotChem with p(1 - phi) = 1 - p(phi),
// and the source S_phi of Eq. SourceTerm_Phi with Delta omega = -sum mu (c_0 - c_1).
__device__ __forceinline__ void potentials_and_source(double phi, double cA, double cB,
                                                      const KParams& P, double& muA,
                                                      double& muB, double& S) {
    const double pp = interp_p(phi);
    muA = cA - P.c0A - pp * (P.c1A - P.c0A);
    muB = cB - P.c0B - pp * (P.c1B - P.c0B);
    const double domega = -(muA * (P.c0A - P.c1A) + muB * (P.c0B - P.c1B));
    S = P.mphi_w2 * (P.lam * interp_dp(phi) * domega - dwell_d(phi));
}

// Moments of one node, Eqs. Moment0_c_alpha and Moment0_Phi.  phi = sum g + S/2
// is implicit in phi; it is resolved by one predictor evaluation of S at sum g.
__device__ __forceinline__ Scalars node_scalars(double phis, double cA, double cB,
                                                const KParams& P) {
    Scalars s;
    double muA, muB, S;
    potentials_and_source(phis, cA, cB, P, muA, muB, S);
    s.phi = phis + 0.5 * S;
    potentials_and_source(s.phi, cA, cB, P, s.muA, s.muB, s.S);
    return s;
}

}  // namespace lbm

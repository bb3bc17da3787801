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
// GK (general curvature matrices kappa_pi = K (K_pi)^-1 of Eq. Taylor): the closure
// c - c^eq(phi) = kappa(phi) mu, kappa(phi) = kappa_0 + p (kappa_1 - kappa_0), is a
// 2 x 2 solve, and Delta omega gains -1/2 mu . (kappa_0 - kappa_1) mu.
template <bool GK = false>
__device__ __forceinline__ void potentials_and_source(double phi, double cA, double cB,
                                                      const KParams& P, double& muA,
                                                      double& muB, double& S) {
    const double pp = interp_p(phi);
    double domega;
    if constexpr (!GK) {
        muA = cA - P.c0A - pp * (P.c1A - P.c0A);
        muB = cB - P.c0B - pp * (P.c1B - P.c0B);
        domega = -(muA * (P.c0A - P.c1A) + muB * (P.c0B - P.c1B));
    } else {
        const double rA = cA - P.c0A - pp * (P.c1A - P.c0A);
        const double rB = cB - P.c0B - pp * (P.c1B - P.c0B);
        const double kAA = P.kap0[0] + pp * (P.kap1[0] - P.kap0[0]);
        const double kAB = P.kap0[1] + pp * (P.kap1[1] - P.kap0[1]);
        const double kBB = P.kap0[2] + pp * (P.kap1[2] - P.kap0[2]);
        const double det = kAA * kBB - kAB * kAB;
        muA = (kBB * rA - kAB * rB) / det;
        muB = (kAA * rB - kAB * rA) / det;
        const double dAA = P.kap0[0] - P.kap1[0], dAB = P.kap0[1] - P.kap1[1], dBB = P.kap0[2] - P.kap1[2];
        domega = -0.5 * (dAA * muA * muA + 2.0 * dAB * muA * muB + dBB * muB * muB) -
                 (muA * (P.c0A - P.c1A) + muB * (P.c0B - P.c1B));
    }
    S = P.mphi_w2 * (P.lam * interp_dp(phi) * domega - dwell_d(phi));
}

// Moments of one node, Eqs. Moment0_c_alpha and Moment0_Phi.  phi = sum g + S/2
// is implicit in phi; it is resolved by one predictor evaluation of S at sum g.
template <bool GK = false>
__device__ __forceinline__ Scalars node_scalars(double phis, double cA, double cB,
                                                const KParams& P) {
    Scalars s;
    double muA, muB, S;
    potentials_and_source<GK>(phis, cA, cB, P, muA, muB, S);
    s.phi = phis + 0.5 * S;
    potentials_and_source<GK>(s.phi, cA, cB, P, s.muA, s.muB, s.S);
    return s;
}

// Three independent compositions (N components, the conclusion's extension with the
// quadratic free energies of Eq. Taylor): the same closure per composition, and
// Delta omega = -sum_alpha mu_alpha (c_0 - c_1)_alpha over A, B, C.
struct Scalars3 {
    double phi, muA, muB, muC, S;
};

__device__ __forceinline__ void potentials_and_source3(double phi, double cA, double cB, double cC,
                                                       const KParams& P, double& muA, double& muB,
                                                       double& muC, double& S) {
    const double pp = interp_p(phi);
    muA = cA - P.c0A - pp * (P.c1A - P.c0A);
    muB = cB - P.c0B - pp * (P.c1B - P.c0B);
    muC = cC - P.c0C - pp * (P.c1C - P.c0C);
    const double domega = -(muA * (P.c0A - P.c1A) + muB * (P.c0B - P.c1B) + muC * (P.c0C - P.c1C));
    S = P.mphi_w2 * (P.lam * interp_dp(phi) * domega - dwell_d(phi));
}

__device__ __forceinline__ Scalars3 node_scalars3(double phis, double cA, double cB, double cC, const KParams& P) {
    Scalars3 s;
    double muA, muB, muC, S;
    potentials_and_source3(phis, cA, cB, cC, P, muA, muB, muC, S);
    s.phi = phis + 0.5 * S;
    potentials_and_source3(s.phi, cA, cB, cC, P, s.muA, s.muB, s.muC, s.S);
    return s;
}

// bulk free-energy density above the reference, in units of K: |mu|^2 / 2, or
// 1/2 mu . kappa(phi) mu with general curvatures
template <bool GK = false>
__device__ __forceinline__ double bulk_free_energy(double phi, double muA, double muB, const KParams& P) {
    if constexpr (!GK) {
        return 0.5 * (muA * muA + muB * muB);
    } else {
        const double pp = interp_p(phi);
        const double kAA = P.kap0[0] + pp * (P.kap1[0] - P.kap0[0]);
        const double kAB = P.kap0[1] + pp * (P.kap1[1] - P.kap0[1]);
        const double kBB = P.kap0[2] + pp * (P.kap1[2] - P.kap0[2]);
        return 0.5 * (kAA * muA * muA + 2.0 * kAB * muA * muB + kBB * muB * muB);
    }
}

}  // namespace lbm

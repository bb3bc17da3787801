// Hand-written reverse mode of one node of the coupled step (adjoint of the local
// part of Section 3's time step), evaluated in FP64.
//
// The step at node x maps the arriving populations P(x) = (f, g, h^A, h^B) and the
// stencil inputs of phi at the neighbours,
//     G = 3 sum_k w_k e_k phi(x + e_k)           (Eq. Grad)
//     N = 3 sum_{k != 0} w_k phi(x + e_k)        (lap = 2 N - 6 (1 - w_0) phi, Eq. Laplacian)
// to the post-collision populations Q(x).  Given mu = dL/dQ(x), node_adjoint returns
// dL/dP(x) through every local path (the node's own phi included), dL/dG, dL/dN and
// the partial derivatives with respect to the parameters
//     theta = (M_phi, M^A_0, M^A_1, M^B_0, M^B_1, W).
// The neighbour dependence closes in a gather pass: phi(y) of a neighbour receives
// 3 w_k (e_k . dL/dG(x) + dL/dN(x)) and enters P(y) through dPhi/dP(y).
#pragma once

#include <type_traits>

#include "lattice.hpp"
#include "params.hpp"
#include "physics.hpp"

namespace lbm {

constexpr int kNumTheta = 6;  // M_phi, MA0, MA1, MB0, MB1, W

__device__ __forceinline__ double interp_ddp(double f) { return 6.0 - 12.0 * f; }  // p''
__device__ __forceinline__ double dwell_dd(double f) {                                // omega_dw''
    return 16.0 * (1.0 - 6.0 * f + 6.0 * f * f);
}

// d phi / d(phi*, c^A, c^B) of the moment phi = phi* + S(phi*, mu(c, phi*)) / 2
__device__ __forceinline__ void dphi_dmoments(double phis, double cA, double cB, const KParams& P,
                                              double (&d)[3]) {
    const double dA = P.c1A - P.c0A, dB = P.c1B - P.c0B;  // c_1 - c_0
    const double eA = -dA, eB = -dB;                      // c_0 - c_1
    const double pp = interp_p(phis), dp = interp_dp(phis);
    const double muA = cA - P.c0A - pp * dA, muB = cB - P.c0B - pp * dB;
    const double dw = -(muA * eA + muB * eB);
    const double K = P.mphi_w2;
    const double ddw_dphis = dp * (eA * dA + eB * dB);
    d[0] = 1.0 + 0.5 * K * (P.lam * (interp_ddp(phis) * dw + dp * ddw_dphis) - dwell_dd(phis));
    d[1] = 0.5 * K * P.lam * dp * (-eA);
    d[2] = 0.5 * K * P.lam * dp * (-eB);
}

// d phi / dK at fixed sums, K = M_phi / W^2: the predictor phi = phi* + S(phi*) / 2
// with S proportional to K
__device__ __forceinline__ double dphi_dK(double phis, double cA, double cB, const KParams& P) {
    const double dA = P.c1A - P.c0A, dB = P.c1B - P.c0B;
    const double pp = interp_p(phis);
    const double muA = cA - P.c0A - pp * dA, muB = cB - P.c0B - pp * dB;
    const double dw = muA * dA + muB * dB;  // Delta omega = -sum mu (c_0 - c_1)
    return 0.5 * (P.lam * interp_dp(phis) * dw - dwell_d(phis));
}

// Reverse mode of the node update.  Inputs: arriving populations (f, g, a = h^A,
// b = h^B), stencil inputs G, N, the LDS value pc of phi at the node (equal to the
// node's phi rounded to the compute type), phi_ref of the buoyancy, mu = dL/dQ.
// Outputs: fb, gb, ab, bb = dL/dP; Gb, Nb; th (accumulated).
template <class SL, class FL>
__device__ __forceinline__ void node_adjoint(const double* f, const double* g, const double* a,
                                             const double* b, const double (&G)[3], double N, double pc,
                                             double phi_ref, const KParams& P, const double* muf,
                                             const double* mug, const double* mua, const double* mub,
                                             double* fb, double* gb, double* ab, double* bb, double (&Gb)[3],
                                             double& Nb, double (&th)[kNumTheta]) {
    constexpr int QS = SL::Q, QF = FL::Q;
    constexpr bool FLOW = QF > 0;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    const double inv_cs2s = 1.0 / SL::cs2;
    const double dA = P.c1A - P.c0A, dB = P.c1B - P.c0B;
    const double eA = -dA, eB = -dB;
    const double K = P.mphi_w2, lam = P.lam;

    // ---------------- forward recompute ----------------
    double phis = 0.0, cA = 0.0, cB = 0.0;
    for (int k = 0; k < QS; ++k) { phis += g[k]; cA += a[k]; cB += b[k]; }
    const double pps = interp_p(phis), dps = interp_dp(phis);
    const double muAs = cA - P.c0A - pps * dA, muBs = cB - P.c0B - pps * dB;
    const double dws = -(muAs * eA + muBs * eB);
    const double Ss = K * (lam * dps * dws - dwell_d(phis));
    const double phi = phis + 0.5 * Ss;
    const double pp = interp_p(phi), dp = interp_dp(phi);
    const double muA = cA - P.c0A - pp * dA, muB = cB - P.c0B - pp * dB;
    const double dw = -(muA * eA + muB * eB);
    const double S = K * (lam * dp * dw - dwell_d(phi));

    double lap = 0.0, bracket = 0.0, F[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0}, p_h = 0.0;
    const double w0s = STL::w(0);
    if constexpr (FLOW) {
        lap = 2.0 * N - 6.0 * (1.0 - w0s) * pc;
        bracket = P.cap * (dwell_d(phi) * P.inv_W2 - lap);
        const double buoy = (phi - phi_ref) * P.drho;
        F[0] = buoy * P.gx + bracket * G[0];
        F[1] = buoy * P.gy + bracket * G[1];
        F[2] = buoy * P.gz + bracket * G[2];
        double j[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < QF; ++k) {
            p_h += f[k];
            j[0] += FL::ex(k) * f[k];
            j[1] += FL::ey(k) * f[k];
            j[2] += FL::ez(k) * f[k];
        }
        for (int d = 0; d < 3; ++d) u[d] = (3.0 * j[d] + 0.5 * F[d]) / P.rho0;
    }

    // ---------------- reverse ----------------
    double phi_b = 0.0, S_b = 0.0, muA_b = 0.0, muB_b = 0.0, cA_b = 0.0, cB_b = 0.0;
    double u_b[3] = {0.0, 0.0, 0.0}, F_b[3] = {0.0, 0.0, 0.0}, p_b = 0.0, K_b = 0.0;

    // h^A, h^B: rest h*_0 = h_0 - w (h_0 - (c - (1 - w_0) mu)),
    // moving h*_k = (1 - w) h_k + w w_k (mu + c e_k.u / c_s^2)
    auto h_adj = [&](const double* h, const double* muh, double* hb, double c, double mu, double M0,
                     double M1, double& c_b, double& mu_b, int th0) {
        const double M = M0 * (1.0 - phi) + M1 * phi;
        const double w = 1.0 / (M * inv_cs2s + 0.5);
        double w_b = 0.0;
        const double E0 = c - (1.0 - SL::w(0)) * mu;
        hb[0] += muh[0] * (1.0 - w);
        w_b += -muh[0] * (h[0] - E0);
        c_b += muh[0] * w;
        mu_b += -(1.0 - SL::w(0)) * muh[0] * w;
        for (int k = 1; k < QS; ++k) {
            const double eu = SL::ex(k) * u[0] + SL::ey(k) * u[1] + SL::ez(k) * u[2];
            const double wk = SL::w(k);
            hb[k] += muh[k] * (1.0 - w);
            w_b += muh[k] * (-h[k] + wk * (mu + c * eu * inv_cs2s));
            mu_b += muh[k] * wk * w;
            c_b += muh[k] * wk * w * eu * inv_cs2s;
            const double eu_b = muh[k] * wk * w * c * inv_cs2s;
            u_b[0] += eu_b * SL::ex(k);
            u_b[1] += eu_b * SL::ey(k);
            u_b[2] += eu_b * SL::ez(k);
        }
        const double M_b = w_b * (-w * w * inv_cs2s);
        phi_b += M_b * (M1 - M0);
        th[th0] += M_b * (1.0 - phi);
        th[th0 + 1] += M_b * phi;
    };
    h_adj(a, mua, ab, cA, muA, P.MA0, P.MA1, cA_b, muA_b, 1);
    h_adj(b, mub, bb, cB, muB, P.MB0, P.MB1, cB_b, muB_b, 3);

    // g: g*_k = (1 - w) g_k + w_k (w phi (1 + e_k.u / c_s^2) + (1 - w/2) S)
    {
        const double w = P.omega_g;
        double w_b = 0.0;
        for (int k = 0; k < QS; ++k) {
            const double eu = SL::ex(k) * u[0] + SL::ey(k) * u[1] + SL::ez(k) * u[2];
            const double wk = SL::w(k);
            gb[k] += mug[k] * (1.0 - w);
            w_b += mug[k] * (-g[k] + wk * (phi * (1.0 + eu * inv_cs2s) - 0.5 * S));
            phi_b += mug[k] * wk * w * (1.0 + eu * inv_cs2s);
            S_b += mug[k] * wk * (1.0 - 0.5 * w);
            const double eu_b = mug[k] * wk * w * phi * inv_cs2s;
            u_b[0] += eu_b * SL::ex(k);
            u_b[1] += eu_b * SL::ey(k);
            u_b[2] += eu_b * SL::ez(k);
        }
        // w = 1 / (M_phi / c_s^2 + 1/2)
        th[0] += w_b * (-w * w * inv_cs2s);
    }

    if constexpr (FLOW) {
        // f: f*_k = (1 - w) f_k + w feq_k + (1 - w/2) F_k
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        const double nu = P.nu0 * (1.0 - phi) + P.nu1 * phi;
        const double w = 1.0 / (3.0 * nu + 0.5);
        const double rho0 = P.rho0;
        const double g0 = 1.0 - 1.5 * uu, e0 = p_h - 0.5 * rho0 * uu;
        double w_b = 0.0, g0_b = 0.0, e0_b = 0.0, uF_b = 0.0;
        for (int k = 0; k < QF; ++k) {
            const double ex = FL::ex(k), ey = FL::ey(k), ez = FL::ez(k), wk = FL::w(k);
            const double eu = ex * u[0] + ey * u[1] + ez * u[2];
            const double eF = ex * F[0] + ey * F[1] + ez * F[2];
            const double gam = wk * (g0 + eu * (3.0 + 4.5 * eu));
            const double Fk = gam * (eF - uF);
            const double feq = wk * (e0 + rho0 * eu * (1.0 + 1.5 * eu));
            fb[k] += muf[k] * (1.0 - w);
            w_b += muf[k] * (-f[k] + feq - 0.5 * Fk);
            const double feq_b = muf[k] * w;
            const double Fk_b = muf[k] * (1.0 - 0.5 * w);
            const double gam_b = Fk_b * (eF - uF);
            const double eF_b = Fk_b * gam;
            uF_b += -Fk_b * gam;
            g0_b += gam_b * wk;
            double eu_b = gam_b * wk * (3.0 + 9.0 * eu);
            e0_b += feq_b * wk;
            eu_b += feq_b * wk * rho0 * (1.0 + 3.0 * eu);
            u_b[0] += eu_b * ex; u_b[1] += eu_b * ey; u_b[2] += eu_b * ez;
            F_b[0] += eF_b * ex; F_b[1] += eF_b * ey; F_b[2] += eF_b * ez;
        }
        double uu_b = -1.5 * g0_b - 0.5 * rho0 * e0_b;
        p_b += e0_b;
        for (int d = 0; d < 3; ++d) {
            u_b[d] += 2.0 * uu_b * u[d] + uF_b * F[d];
            F_b[d] += uF_b * u[d];
        }
        const double nu_b = w_b * (-3.0 * w * w);
        phi_b += nu_b * (P.nu1 - P.nu0);
        // u = (3 j + F / 2) / rho0, p_h = sum f, j = sum f e
        double j_b[3];
        for (int d = 0; d < 3; ++d) {
            j_b[d] = 3.0 * u_b[d] / rho0;
            F_b[d] += 0.5 * u_b[d] / rho0;
        }
        for (int k = 0; k < QF; ++k)
            fb[k] += p_b + FL::ex(k) * j_b[0] + FL::ey(k) * j_b[1] + FL::ez(k) * j_b[2];
        // F = (phi - phi_ref) drho g + bracket G, bracket = cap (omega_dw'(phi) / W^2 - lap)
        phi_b += P.drho * (F_b[0] * P.gx + F_b[1] * P.gy + F_b[2] * P.gz);
        const double bracket_b = F_b[0] * G[0] + F_b[1] * G[1] + F_b[2] * G[2];
        for (int d = 0; d < 3; ++d) Gb[d] = bracket * F_b[d];
        phi_b += bracket_b * P.cap * P.inv_W2 * dwell_dd(phi);
        const double lap_b = -bracket_b * P.cap;
        // cap = 3/2 sigma W: bracket = 3/2 sigma (omega_dw' / W - W lap)
        th[5] += bracket_b * (P.cap / P.W) * (-dwell_d(phi) * P.inv_W2 - lap);
        // lap = 2 N - 6 (1 - w_0) pc, pc the node's own phi
        Nb = 2.0 * lap_b;
        phi_b += -6.0 * (1.0 - w0s) * lap_b;
    } else {
        Gb[0] = Gb[1] = Gb[2] = 0.0;
        Nb = 0.0;
    }

    // S = K (lambda p'(phi) dw - omega_dw'(phi))
    K_b += S_b * (lam * dp * dw - dwell_d(phi));
    phi_b += S_b * K * (lam * interp_ddp(phi) * dw - dwell_dd(phi));
    const double dw_b = S_b * K * lam * dp;
    muA_b += -dw_b * eA;
    muB_b += -dw_b * eB;
    // mu = c - c_0 - p(phi) (c_1 - c_0)
    cA_b += muA_b;
    cB_b += muB_b;
    phi_b += (-muA_b * dA - muB_b * dB) * dp;
    // phi = phi* + S*/2
    double phis_b = phi_b;
    const double Ss_b = 0.5 * phi_b;
    K_b += Ss_b * (lam * dps * dws - dwell_d(phis));
    phis_b += Ss_b * K * (lam * interp_ddp(phis) * dws - dwell_dd(phis));
    const double dws_b = Ss_b * K * lam * dps;
    const double muAs_b = -dws_b * eA, muBs_b = -dws_b * eB;
    cA_b += muAs_b;
    cB_b += muBs_b;
    phis_b += (-muAs_b * dA - muBs_b * dB) * dps;
    // K = M_phi / W^2
    th[0] += K_b / (P.W * P.W);
    th[5] += K_b * (-2.0 * K / P.W);
    // sums
    for (int k = 0; k < QS; ++k) {
        gb[k] += phis_b;
        ab[k] += cA_b;
        bb[k] += cB_b;
    }
}

}  // namespace lbm

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

// Sensitivities of the moment phi = phi* + S(phi*, mu(c, phi*)) / 2 (Eq. Moment0_Phi
// with the predictor) at fixed sums phi* = sum g, c^A, c^B:
//   d0 = dphi/dphi*,  dphi/dc^A = q (c^A_1 - c^A_0),  dphi/dc^B = q (c^B_1 - c^B_0),
//   dK = dphi/dK with K = M_phi / W^2 (S is proportional to K).
struct PhiSens {
    double d0, q, dK;
};

__device__ __forceinline__ PhiSens phi_sensitivities(double phis, double cA, double cB, const KParams& P) {
    const double dA = P.c1A - P.c0A, dB = P.c1B - P.c0B;  // c_1 - c_0
    const double pp = interp_p(phis), dp = interp_dp(phis);
    const double muA = cA - P.c0A - pp * dA, muB = cB - P.c0B - pp * dB;
    const double dw = muA * dA + muB * dB;  // Delta omega = -sum mu (c_0 - c_1)
    const double K = P.mphi_w2;
    PhiSens r;
    // d(dw)/dphi* = -p'(phi*) (dA^2 + dB^2)
    r.d0 = 1.0 + 0.5 * K * (P.lam * (interp_ddp(phis) * dw - dp * dp * (dA * dA + dB * dB)) - dwell_dd(phis));
    r.q = 0.5 * K * P.lam * dp;
    r.dK = 0.5 * (P.lam * dp * dw - dwell_d(phis));
    return r;
}

// reciprocal in the compute type (the step kernel's rates use the same)
template <class T>
__device__ __forceinline__ T arcp(T x) {
    if constexpr (std::is_same<T, double>::value) return 1.0 / x;
    else return __builtin_amdgcn_rcpf(x);
}

// Reverse mode of the node update.  Inputs: arriving populations (f, g, a = h^A,
// b = h^B), stencil inputs G, N, the value pc of phi at the node as the stencil saw
// it, phi_ref of the buoyancy, and mu(IC<s>), which returns dL/dQ_s for slot s
// (canonical slot order).  out(IC<s>, v) receives dL/dP_s.  Also returns Gb = dL/dG,
// Nb = dL/dN and accumulates th = dL/dtheta.
//
// Pass 1 folds every mu_s into the per-node reverse sums; pass 2 writes
// dL/dP_s = (1 - w) mu_s + per-field terms.  The forward recompute of the moments,
// potentials and source runs in FP64 (differences of nearby compositions); the
// reverse sweep runs in T, the storage's compute type.
template <class SL, class FL, class T, class MU, class OUT>
__device__ __forceinline__ void node_adjoint(const T* f, const T* g, const T* a, const T* b, const double (&G)[3],
                                             double N, double pc, double phi_ref, const KParams& P, MU&& mu,
                                             OUT&& out, double (&Gb)[3], double& Nb, double (&th)[kNumTheta]) {
    constexpr int QS = SL::Q, QF = FL::Q;
    constexpr int G0 = QF, A0 = QF + QS, B0 = QF + 2 * QS;
    constexpr bool FLOW = QF > 0;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    using R = T;
    constexpr double inv_cs2d = 1.0 / SL::cs2;
    const R inv_cs2 = R(inv_cs2d);
    const R dA = R(P.c1A - P.c0A), dB = R(P.c1B - P.c0B);
    const R K = R(P.mphi_w2), lam = R(P.lam);

    // ---------------- forward recompute ----------------
    double phis = 0.0, cAd = 0.0, cBd = 0.0;
    for (int k = 0; k < QS; ++k) { phis += double(g[k]); cAd += double(a[k]); cBd += double(b[k]); }
    const double dAd = P.c1A - P.c0A, dBd = P.c1B - P.c0B;
    const double pps = interp_p(phis), dps_d = interp_dp(phis);
    const double dws_d = (cAd - P.c0A - pps * dAd) * dAd + (cBd - P.c0B - pps * dBd) * dBd;
    const double phi_d = phis + 0.5 * P.mphi_w2 * (P.lam * dps_d * dws_d - dwell_d(phis));
    const double pp_d = interp_p(phi_d);
    const double muA_d = cAd - P.c0A - pp_d * dAd, muB_d = cBd - P.c0B - pp_d * dBd;
    const double dw_d = muA_d * dAd + muB_d * dBd;
    const R phi = R(phi_d), dp = R(interp_dp(phi_d)), dw = R(dw_d), muA = R(muA_d), muB = R(muB_d);
    const R S = K * (lam * dp * dw - R(dwell_d(phi_d)));
    const R cA = R(cAd), cB = R(cBd);
    const R ps = R(phis), dps = R(dps_d), dws = R(dws_d);

    constexpr R w0s = R(STL::w(0));
    R lap = R(0), bracket = R(0), F[3] = {R(0), R(0), R(0)};
    T u[3] = {T(0), T(0), T(0)}, p_h = T(0);
    const R cap = R(P.cap), invW2 = R(P.inv_W2);
    if constexpr (FLOW) {
        lap = R(2) * R(N) - R(6) * (R(1) - w0s) * R(pc);
        bracket = cap * (R(dwell_d(phi_d)) * invW2 - lap);
        const R buoy = (phi - R(phi_ref)) * R(P.drho);
        F[0] = buoy * R(P.gx) + bracket * R(G[0]);
        F[1] = buoy * R(P.gy) + bracket * R(G[1]);
        F[2] = buoy * R(P.gz) + bracket * R(G[2]);
        T j[3] = {T(0), T(0), T(0)};
        static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            p_h += f[k];
            if constexpr (FL::ex(k) != 0) j[0] += FL::ex(k) > 0 ? f[k] : -f[k];
            if constexpr (FL::ey(k) != 0) j[1] += FL::ey(k) > 0 ? f[k] : -f[k];
            if constexpr (FL::ez(k) != 0) j[2] += FL::ez(k) > 0 ? f[k] : -f[k];
        });
        const T inv_rho0 = T(1.0 / P.rho0);
        for (int d = 0; d < 3; ++d) u[d] = (T(3) * j[d] + T(0.5) * F[d]) * inv_rho0;
    }

    // ---------------- pass 1: reverse sums ----------------
    R phi_b = R(0), S_b = R(0), muA_b = R(0), muB_b = R(0), cA_b = R(0), cB_b = R(0), K_b = R(0);
    T u_b[3] = {T(0), T(0), T(0)};
    auto add_eu = [&](auto lat_, auto k_, T v) __attribute__((always_inline)) {
        using L = typename decltype(lat_)::type;
        constexpr int k = decltype(k_)::value;
        if constexpr (L::ex(k) != 0) u_b[0] += L::ex(k) > 0 ? v : -v;
        if constexpr (L::ey(k) != 0) u_b[1] += L::ey(k) > 0 ? v : -v;
        if constexpr (L::ez(k) != 0) u_b[2] += L::ez(k) > 0 ? v : -v;
    };
    using SLT = std::common_type<SL>;
    using FLT = std::common_type<FL>;

    // h^A, h^B: rest h*_0 = h_0 - w (h_0 - (c - (1 - w_0) mu)),
    // moving h*_k = (1 - w) h_k + w w_k (mu + c e_k.u / c_s^2)
    auto h_adj = [&](auto base_, const T* h, R c, R muv, double M0, double M1, R& c_b, R& mu_b,
                     int th0) __attribute__((always_inline)) -> R {
        constexpr int B = decltype(base_)::value;
        const R M = R(M0) * (R(1) - phi) + R(M1) * phi;
        const R w = arcp<R>(M * inv_cs2 + R(0.5));
        const R m0 = mu(IC<B>{});
        R w_b = -m0 * (h[0] - (c - R(1.0 - SL::w(0)) * muv));
        c_b += m0 * w;
        mu_b += -R(1.0 - SL::w(0)) * m0 * w;
        const R cT = c * inv_cs2;
        R mu_bT = R(0), c_bT = R(0);
        static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            const T eu = edot<SL::ex(k), SL::ey(k), SL::ez(k)>(u[0], u[1], u[2]);
            const T wk = T(SL::w(k));
            const T m = mu(IC<B + k>{});
            w_b += m * (wk * (muv + cT * eu) - h[k]);
            const T mw = m * wk * w;
            mu_bT += mw;
            c_bT += mw * eu;
            add_eu(SLT{}, kc, mw * cT);
        });
        mu_b += mu_bT;
        c_b += c_bT * inv_cs2;
        const R M_b = w_b * (-w * w * inv_cs2);
        phi_b += M_b * R(M1 - M0);
        th[th0] += double(M_b * (R(1) - phi));
        th[th0 + 1] += double(M_b * phi);
        return w;
    };
    const R wA = h_adj(IC<A0>{}, a, cA, muA, P.MA0, P.MA1, cA_b, muA_b, 1);
    const R wB = h_adj(IC<B0>{}, b, cB, muB, P.MB0, P.MB1, cB_b, muB_b, 3);

    // g: g*_k = (1 - w) g_k + w_k (w phi (1 + e_k.u / c_s^2) + (1 - w/2) S)
    const R wg = R(P.omega_g);
    {
        const R half_S = R(0.5) * S;
        R w_b = R(0), phi_bT = R(0), S_bT = R(0);
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            const T eu = edot<SL::ex(k), SL::ey(k), SL::ez(k)>(u[0], u[1], u[2]);
            const T wk = T(SL::w(k));
            const T m = mu(IC<G0 + k>{});
            const T fac = T(1) + eu * inv_cs2;
            w_b += m * (wk * (phi * fac - half_S) - g[k]);
            phi_bT += m * wk * fac;
            S_bT += m * wk;
            add_eu(SLT{}, kc, m * wk * wg * phi * inv_cs2);
        });
        phi_b += phi_bT * wg;
        S_b += S_bT * (R(1) - R(0.5) * wg);
        // w = 1 / (M_phi / c_s^2 + 1/2)
        th[0] += double(w_b) * (-P.omega_g * P.omega_g * inv_cs2d);
    }

    R wf = R(0);
    T p_b = T(0), j_b[3] = {T(0), T(0), T(0)};
    if constexpr (FLOW) {
        // f: f*_k = (1 - w) f_k + w feq_k + (1 - w/2) F_k
        const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        const R nu = R(P.nu0) * (R(1) - phi) + R(P.nu1) * phi;
        wf = arcp<R>(R(3) * nu + R(0.5));
        const T half = T(1) - T(0.5) * wf;
        const T rho0 = T(P.rho0);
        const T g0 = T(1) - T(1.5) * uu, e0 = p_h - T(0.5) * rho0 * uu;
        T w_b = T(0), g0_b = T(0), e0_b = T(0), uF_b = T(0);
        T F_b[3] = {T(0), T(0), T(0)};
        static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            constexpr int ex = FL::ex(k), ey = FL::ey(k), ez = FL::ez(k);
            const T wk = T(FL::w(k));
            const T eu = edot<ex, ey, ez>(u[0], u[1], u[2]);
            const T eF = edot<ex, ey, ez>(F[0], F[1], F[2]);
            const T gam = wk * (g0 + eu * (T(3) + T(4.5) * eu));
            const T Fk = gam * (eF - uF);
            const T feq = wk * (e0 + rho0 * eu * (T(1) + T(1.5) * eu));
            const T m = mu(IC<k>{});
            w_b += m * (feq - T(0.5) * Fk - f[k]);
            const T feq_b = m * wf;
            const T Fk_b = m * half;
            const T gam_b = Fk_b * (eF - uF);
            const T eF_b = Fk_b * gam;
            uF_b -= eF_b;
            g0_b += gam_b * wk;
            e0_b += feq_b * wk;
            add_eu(FLT{}, kc, gam_b * wk * (T(3) + T(9) * eu) + feq_b * wk * rho0 * (T(1) + T(3) * eu));
            if constexpr (ex != 0) F_b[0] += ex > 0 ? eF_b : -eF_b;
            if constexpr (ey != 0) F_b[1] += ey > 0 ? eF_b : -eF_b;
            if constexpr (ez != 0) F_b[2] += ez > 0 ? eF_b : -eF_b;
        });
        const T uu_b = T(-1.5) * g0_b - T(0.5) * rho0 * e0_b;
        p_b = e0_b;
        for (int d = 0; d < 3; ++d) {
            u_b[d] += T(2) * uu_b * u[d] + uF_b * F[d];
            F_b[d] += uF_b * u[d];
        }
        phi_b += w_b * (-R(3) * wf * wf) * R(P.nu1 - P.nu0);
        // u = (3 j + F / 2) / rho0, p_h = sum f, j = sum f e
        const T inv_rho0 = T(1.0 / P.rho0);
        for (int d = 0; d < 3; ++d) {
            j_b[d] = T(3) * u_b[d] * inv_rho0;
            F_b[d] += T(0.5) * u_b[d] * inv_rho0;
        }
        // F = (phi - phi_ref) drho g + bracket G, bracket = cap (omega_dw'(phi) / W^2 - lap)
        phi_b += R(P.drho) * (F_b[0] * R(P.gx) + F_b[1] * R(P.gy) + F_b[2] * R(P.gz));
        const R bracket_b = F_b[0] * R(G[0]) + F_b[1] * R(G[1]) + F_b[2] * R(G[2]);
        for (int d = 0; d < 3; ++d) Gb[d] = double(bracket * F_b[d]);
        phi_b += bracket_b * cap * invW2 * R(dwell_dd(phi_d));
        const R lap_b = -bracket_b * cap;
        // bracket = cap omega_dw' / W^2 - cap lap with cap = 3/2 sigma W
        th[5] += double(bracket_b) * (P.dcap_dW * (dwell_d(phi_d) * P.inv_W2 - double(lap)) +
                                      P.cap * dwell_d(phi_d) * (-2.0 * P.inv_W2 / P.W));
        // lap = 2 N - 6 (1 - w_0) pc, pc the node's own phi
        Nb = double(R(2) * lap_b);
        phi_b += -R(6) * (R(1) - w0s) * lap_b;
    } else {
        Gb[0] = Gb[1] = Gb[2] = 0.0;
        Nb = 0.0;
    }

    // S = K (lambda p'(phi) dw - omega_dw'(phi)), dw = mu^A dA + mu^B dB
    K_b += S_b * (lam * dp * dw - R(dwell_d(phi_d)));
    phi_b += S_b * K * (lam * R(interp_ddp(phi_d)) * dw - R(dwell_dd(phi_d)));
    const R dw_b = S_b * K * lam * dp;
    muA_b += dw_b * dA;
    muB_b += dw_b * dB;
    // mu = c - c_0 - p(phi) (c_1 - c_0)
    cA_b += muA_b;
    cB_b += muB_b;
    phi_b += (-muA_b * dA - muB_b * dB) * dp;
    // phi = phi* + S*/2
    R phis_b = phi_b;
    const R Ss_b = R(0.5) * phi_b;
    K_b += Ss_b * (lam * dps * dws - R(dwell_d(phis)));
    phis_b += Ss_b * K * (lam * R(interp_ddp(phis)) * dws - R(dwell_dd(phis)));
    const R dws_b = Ss_b * K * lam * dps;
    cA_b += dws_b * dA;
    cB_b += dws_b * dB;
    phis_b += -dws_b * (dA * dA + dB * dB) * dps;
    // K = M_phi / W^2
    th[0] += double(K_b) * P.inv_W2;
    th[5] += double(K_b) * P.dK_dW;
    (void)ps;

    // ---------------- pass 2: dL/dP ----------------
    // every population's direct use is its own collision, (1 - w) P; the moments add
    // one term per field; f also enters p_h and j
    if constexpr (FLOW) {
        const T keep = T(1) - wf;
        static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            T v = mu(IC<k>{}) * keep + p_b;
            if constexpr (FL::ex(k) != 0) v += FL::ex(k) > 0 ? j_b[0] : -j_b[0];
            if constexpr (FL::ey(k) != 0) v += FL::ey(k) > 0 ? j_b[1] : -j_b[1];
            if constexpr (FL::ez(k) != 0) v += FL::ez(k) > 0 ? j_b[2] : -j_b[2];
            out(IC<k>{}, v);
        });
    }
    {
        const T keep = T(1) - wg;
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            out(IC<G0 + kc.value>{}, mu(IC<G0 + kc.value>{}) * keep + phis_b);
        });
    }
    {
        const T keepA = T(1) - wA, keepB = T(1) - wB;
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            out(IC<A0 + kc.value>{}, mu(IC<A0 + kc.value>{}) * keepA + cA_b);
            out(IC<B0 + kc.value>{}, mu(IC<B0 + kc.value>{}) * keepB + cB_b);
        });
    }
}

}  // namespace lbm

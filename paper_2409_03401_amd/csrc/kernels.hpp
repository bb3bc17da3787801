// HIP kernels of the coupled lattice-Boltzmann step for gfx950.
//
// One fused kernel per (lattice family, mode, storage precision).  A work-group
// owns a TX x TY column of nodes and marches along z over `zc` planes.  When the
// capillary force (or the free-energy diagnostic) needs grad phi and lap phi,
// phi of three consecutive planes, each with a one-node ring, is staged in LDS:
// the work-group computes phi of plane z+1 (its own nodes from registers kept for
// the next iteration, ring nodes from L2-resident neighbour populations), then
// updates plane z.  Populations live in two copies (read one, write the other),
// so ring reads never race with writes.  Streaming is a push: each node writes
// its post-collision populations into the neighbour slots of the other copy,
// or back into its own node in the opposite direction across a wall.
#pragma once

#include <type_traits>

#include "lattice.hpp"
#include "params.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// thermodynamics (Section 2)

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

// ---------------------------------------------------------------------------
// population storage

template <int PREC>
__device__ __forceinline__ typename Stor<PREC>::C ld_pop(const void* base, int idx, bool rest,
                                                         float wref, float inv_scale) {
    if constexpr (PREC == P64) {
        return static_cast<const double*>(base)[idx];
    } else if constexpr (PREC == P32) {
        return static_cast<const float*>(base)[idx];
    } else {
        if (rest) return static_cast<const float*>(base)[idx];
        using T = typename Stor<PREC>::T;
        const T d = static_cast<const T*>(base)[idx];
        float v;
        if constexpr (PREC == P16) v = __half2float(d);
        else v = __bfloat162float(d);
        return fmaf(v, inv_scale, wref);
    }
}

template <int PREC>
__device__ __forceinline__ void st_pop(void* base, int idx, bool rest, float wref, float scale,
                                       typename Stor<PREC>::C v) {
    if constexpr (PREC == P64) {
        static_cast<double*>(base)[idx] = v;
    } else if constexpr (PREC == P32) {
        static_cast<float*>(base)[idx] = v;
    } else {
        if (rest) {
            static_cast<float*>(base)[idx] = v;
            return;
        }
        using T = typename Stor<PREC>::T;
        const float d = (v - wref) * scale;
        T q;
        if constexpr (PREC == P16) q = __float2half_rn(d);
        else q = __float2bfloat16(d);
        static_cast<T*>(base)[idx] = q;
    }
}

// compile-time loop: f(std::integral_constant<int, k>) for k in [B, E)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// periodic wrap / mirror ghost of a coordinate in [-1, n]
__device__ __forceinline__ int map_coord(int c, int n, int wall) {
    if (c < 0) return wall ? 0 : n - 1;
    if (c >= n) return wall ? n - 1 : 0;
    return c;
}

// ---------------------------------------------------------------------------
// block reduction of N doubles (entry `maxslot` takes a max, the others a sum),
// fixed order, one result per work-group

template <int N, int NT>
__device__ __forceinline__ void block_reduce_store(double (&v)[N], int maxslot, double* out) {
    static_assert(NT % 64 == 0, "work-group must be whole waves");
    __shared__ double red[NT / 64][N];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double o = __shfl_down(v[i], off, 64);
            v[i] = (i == maxslot) ? fmax(v[i], o) : v[i] + o;
        }
    }
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) red[tid >> 6][i] = v[i];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double a = red[0][i];
            for (int w = 1; w < NT / 64; ++w) a = (i == maxslot) ? fmax(a, red[w][i]) : a + red[w][i];
            out[i] = a;
        }
    }
}

// ---------------------------------------------------------------------------
// the fused step / moments / diagnostics kernel

template <class SL, class FL, int MODE, int PREC, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k_lbm(const KParams P) {
    using C = typename Stor<PREC>::C;
    constexpr int QS = SL::Q;
    constexpr int QF = FL::Q;
    constexpr bool FLOW = QF > 0;
    constexpr bool STENCIL = FLOW || MODE == MODE_DIAG;
    constexpr bool HAS_Y = SL::DIM == 3;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    constexpr int LX = TX + 2;
    constexpr int LY = HAS_Y ? TY + 2 : 1;
    constexpr int OY = HAS_Y ? 1 : 0;
    constexpr int NSLOT = STENCIL ? 3 : 1;
    constexpr int NT = TX * TY;
    constexpr int G0 = QF, A0 = QF + QS, B0 = QF + 2 * QS;  // slot offsets
    constexpr C inv_cs2s = C(1.0 / SL::cs2);
    static_assert(TY == 1 || HAS_Y, "2D problems use one row per work-group");

    __shared__ C sphi[NSLOT][LY][LX];

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    const int x = blockIdx.x * TX + tx;
    const int y = blockIdx.y * TY + ty;
    const bool active = (x < P.nx) && (y < P.ny);
    const int z0 = blockIdx.z * P.zc;
    const int z1 = min(z0 + P.zc, P.nz);

    auto load_scalars = [&](int idx, C (&gg)[QS], C (&aa)[QS], C (&bb)[QS], double& phis,
                            double& cA, double& cB) __attribute__((always_inline)) {
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            gg[k] = ld_pop<PREC>(P.src[G0 + k], idx, k == 0, P.swref[G0 + k], P.sinv[G0 + k]);
            aa[k] = ld_pop<PREC>(P.src[A0 + k], idx, k == 0, P.swref[A0 + k], P.sinv[A0 + k]);
            bb[k] = ld_pop<PREC>(P.src[B0 + k], idx, k == 0, P.swref[B0 + k], P.sinv[B0 + k]);
        });
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int k = 0; k < QS; ++k) {
            s0 += double(gg[k]);
            s1 += double(aa[k]);
            s2 += double(bb[k]);
        }
        phis = s0;
        cA = s1;
        cB = s2;
    };

    auto node_phi = [&](int xx, int yy, int zz) __attribute__((always_inline)) -> C {
        C tg[QS], ta[QS], tb[QS];
        double ps, ca, cb;
        load_scalars((zz * P.ny + yy) * P.nx + xx, tg, ta, tb, ps, ca, cb);
        return C(node_scalars(ps, ca, cb, P).phi);
    };

    // scalar populations and sums of this thread's node: current plane (c*) and next plane (n*)
    C cg[QS], ca[QS], cb[QS], ng[QS], na[QS], nb[QS];
    double c_ps = 0.0, c_cA = 0.0, c_cB = 0.0, n_ps = 0.0, n_cA = 0.0, n_cB = 0.0;

    // phi of plane zz (tile + ring) into LDS slot `slot`; this thread's own node
    // populations go to (gg, aa, bb) when the node is inside the domain
    auto fill_plane = [&](int zz, int slot, C (&gg)[QS], C (&aa)[QS], C (&bb)[QS], double& ps,
                          double& cA, double& cB) __attribute__((always_inline)) {
        const int zm = map_coord(zz, P.nz, P.wall_z);
        if (active) {
            load_scalars((zm * P.ny + y) * P.nx + x, gg, aa, bb, ps, cA, cB);
            sphi[slot][ty + OY][tx + 1] = C(node_scalars(ps, cA, cB, P).phi);
        } else if (x <= P.nx && y <= P.ny) {
            // ghost column / row just beyond the domain edge
            sphi[slot][ty + OY][tx + 1] = node_phi(map_coord(x, P.nx, P.wall_x),
                                                   HAS_Y ? map_coord(y, P.ny, P.wall_y) : 0, zm);
        }
        constexpr int NH = HAS_Y ? 2 * LX + 2 * TY : 2;
        for (int i = tid; i < NH; i += NT) {
            int hx, hy;
            if constexpr (HAS_Y) {
                if (i < LX) { hx = i; hy = 0; }
                else if (i < 2 * LX) { hx = i - LX; hy = TY + 1; }
                else if (i < 2 * LX + TY) { hx = 0; hy = i - 2 * LX + 1; }
                else { hx = LX - 1; hy = i - 2 * LX - TY + 1; }
            } else {
                hx = (i == 0) ? 0 : LX - 1;
                hy = 0;
            }
            const int gx = int(blockIdx.x * TX) + hx - 1;
            const int gy = HAS_Y ? int(blockIdx.y * TY) + hy - 1 : 0;
            if (gx > P.nx || gy > P.ny) continue;  // beyond the ghost layer: never read
            sphi[slot][hy][hx] = node_phi(map_coord(gx, P.nx, P.wall_x),
                                          HAS_Y ? map_coord(gy, P.ny, P.wall_y) : 0, zm);
        }
    };

    constexpr int NACC = (MODE == MODE_DIAG) ? 8 : 1;
    double acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = 0.0;

    const double phi_ref = P.mean_subtract ? *P.phi_ref : 0.0;

    if constexpr (STENCIL) {
        if (z0 < z1) {
            fill_plane(z0 - 1, 0, ng, na, nb, n_ps, n_cA, n_cB);  // ring only; registers discarded
            fill_plane(z0, 1, cg, ca, cb, c_ps, c_cA, c_cB);
        }
    }

    for (int z = z0; z < z1; ++z) {
        int sm = 0, sc = 0, sp = 0;
        if constexpr (STENCIL) {
            sm = (z - z0) % 3;
            sc = (z - z0 + 1) % 3;
            sp = (z - z0 + 2) % 3;
            fill_plane(z + 1, sp, ng, na, nb, n_ps, n_cA, n_cB);
            __syncthreads();
        } else {
            if (active) load_scalars((z * P.ny + y) * P.nx + x, cg, ca, cb, c_ps, c_cA, c_cB);
        }
        const C(&g)[QS] = cg;
        const C(&a)[QS] = ca;
        const C(&b)[QS] = cb;
        const double sA = c_cA, sB = c_cB;

        if (active) {
            const int idx = (z * P.ny + y) * P.nx + x;
            const Scalars m = node_scalars(c_ps, sA, sB, P);
            const C phi = C(m.phi);

            C grad[3] = {C(0), C(0), C(0)};
            C lap = C(0);
            if constexpr (STENCIL) {
                const C pc = sphi[sc][ty + OY][tx + 1];
#pragma unroll
                for (int k = 1; k < STL::Q; ++k) {
                    const int ez = STL::ez(k);
                    const int slot = ez == 0 ? sc : (ez > 0 ? sp : sm);
                    const C v = sphi[slot][ty + OY + STL::ey(k)][tx + 1 + STL::ex(k)];
                    const C w3 = C(3.0 * STL::w(k));
                    grad[0] += w3 * C(STL::ex(k)) * v;
                    grad[1] += w3 * C(STL::ey(k)) * v;
                    grad[2] += w3 * C(STL::ez(k)) * v;
                    lap += C(2.0) * w3 * (v - pc);
                }
            }

            C u[3] = {C(0), C(0), C(0)};
            C p_h = C(0);
            C fpop[QF > 0 ? QF : 1];
            C F[3] = {C(0), C(0), C(0)};
            if constexpr (FLOW) {
                static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                    constexpr int k = decltype(kc)::value;
                    fpop[k] = ld_pop<PREC>(P.src[k], idx, k == 0, P.swref[k], P.sinv[k]);
                });
                // Eq. SurfaceTension_Force plus buoyancy (phi - phi_ref) drho g
                const C bracket = C(P.cap) * (C(dwell_d(m.phi)) * C(P.inv_W2) - lap);
                const C buoy = C((m.phi - phi_ref) * P.drho);
                F[0] = buoy * C(P.gx) + bracket * grad[0];
                F[1] = buoy * C(P.gy) + bracket * grad[1];
                F[2] = buoy * C(P.gz) + bracket * grad[2];
                // Eqs. HydroPressure and Velocity
                C j0 = C(0), j1 = C(0), j2 = C(0);
#pragma unroll
                for (int k = 0; k < QF; ++k) {
                    p_h += fpop[k];
                    if (FL::ex(k)) j0 += C(FL::ex(k)) * fpop[k];
                    if (FL::ey(k)) j1 += C(FL::ey(k)) * fpop[k];
                    if (FL::ez(k)) j2 += C(FL::ez(k)) * fpop[k];
                }
                const C inv_rho0 = C(1.0 / P.rho0);
                u[0] = (C(3) * j0 + C(0.5) * F[0]) * inv_rho0;
                u[1] = (C(3) * j1 + C(0.5) * F[1]) * inv_rho0;
                u[2] = (C(3) * j2 + C(0.5) * F[2]) * inv_rho0;
            }

            if constexpr (MODE == MODE_STEP) {
                if (P.mean_subtract) acc[0] += m.phi;

                // ---- streaming targets ----
                // push the post-collision value of slot S (direction (ex, ey, ez)) to the
                // neighbour; across a wall it returns to this node in slot SOPP
                auto push = [&](auto sc_, auto sopp_, int ex, int ey, int ez, C v) __attribute__((always_inline)) {
                    constexpr int S = decltype(sc_)::value;
                    constexpr int SOPP = decltype(sopp_)::value;
                    int xt = x + ex, yt = y + ey, zt = z + ez;
                    bool bounce = false;
                    if (ex) {
                        if (xt < 0 || xt >= P.nx) { if (P.wall_x) bounce = true; else xt = xt < 0 ? P.nx - 1 : 0; }
                    }
                    if (ey) {
                        if (yt < 0 || yt >= P.ny) { if (P.wall_y) bounce = true; else yt = yt < 0 ? P.ny - 1 : 0; }
                    }
                    if (ez) {
                        if (zt < 0 || zt >= P.nz) { if (P.wall_z) bounce = true; else zt = zt < 0 ? P.nz - 1 : 0; }
                    }
                    if (bounce)
                        st_pop<PREC>(P.dst[SOPP], idx, false, P.swref[SOPP], P.sscale[SOPP], v);
                    else
                        st_pop<PREC>(P.dst[S], (zt * P.ny + yt) * P.nx + xt, P.srest[S] != 0, P.swref[S],
                                     P.sscale[S], v);
                };

                // ---- f: Eqs. LBE_FluidFlow, ForcingTerm, GammaFunction, Feq ----
                if constexpr (FLOW) {
                    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                    const C nu = C(P.nu0 * (1.0 - m.phi) + P.nu1 * m.phi);
                    const C wf = C(1) / (C(3) * nu + C(0.5));
                    const C rho0 = C(P.rho0);
                    static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        const C eu = C(FL::ex(k)) * u[0] + C(FL::ey(k)) * u[1] + C(FL::ez(k)) * u[2];
                        const C wk = C(FL::w(k));
                        const C gam = wk * (C(1) + C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu);
                        const C Fk = gam * ((C(FL::ex(k)) - u[0]) * F[0] + (C(FL::ey(k)) - u[1]) * F[1] +
                                            (C(FL::ez(k)) - u[2]) * F[2]);
                        const C feq = wk * (p_h + rho0 * (eu + C(1.5) * eu * eu - C(0.5) * uu)) - C(0.5) * Fk;
                        const C post = fpop[k] - wf * (fpop[k] - feq) + Fk;
                        push(std::integral_constant<int, k>{}, std::integral_constant<int, FL::opp(k)>{},
                             FL::ex(k), FL::ey(k), FL::ez(k), post);
                    });
                }

                // ---- g: Eqs. LBE_Phi, Geq, Source_LBE_Phi ----
                {
                    const C wg = C(P.omega_g);
                    const C S = C(m.S);
                    static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        const C eu = C(SL::ex(k)) * u[0] + C(SL::ey(k)) * u[1] + C(SL::ez(k)) * u[2];
                        const C Gk = C(SL::w(k)) * S;
                        const C geq = C(SL::w(k)) * phi * (C(1) + eu * inv_cs2s) - C(0.5) * Gk;
                        const C post = g[k] - wg * (g[k] - geq) + Gk;
                        push(std::integral_constant<int, G0 + k>{}, std::integral_constant<int, G0 + SL::opp(k)>{},
                             SL::ex(k), SL::ey(k), SL::ez(k), post);
                    });
                }

                // ---- h^A, h^B: Eqs. LBE_c_alpha, Heq; mobility interpolated in phi ----
                {
                    const double MA = P.MA0 * (1.0 - m.phi) + P.MA1 * m.phi;
                    const double MB = P.MB0 * (1.0 - m.phi) + P.MB1 * m.phi;
                    const double whA = 1.0 / (MA / SL::cs2 + 0.5);
                    const double whB = 1.0 / (MB / SL::cs2 + 0.5);
                    // rest populations in double: they carry the conserved composition
                    {
                        const double eqA = sA - (1.0 - SL::w(0)) * m.muA;
                        const double eqB = sB - (1.0 - SL::w(0)) * m.muB;
                        const double pa = double(a[0]) - whA * (double(a[0]) - eqA);
                        const double pb = double(b[0]) - whB * (double(b[0]) - eqB);
                        push(std::integral_constant<int, A0>{}, std::integral_constant<int, A0>{}, 0, 0, 0, C(pa));
                        push(std::integral_constant<int, B0>{}, std::integral_constant<int, B0>{}, 0, 0, 0, C(pb));
                    }
                    const C wA = C(whA), wB = C(whB);
                    const C muA = C(m.muA), muB = C(m.muB);
                    const C cAc = C(sA), cBc = C(sB);
                    static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        const C eu = (C(SL::ex(k)) * u[0] + C(SL::ey(k)) * u[1] + C(SL::ez(k)) * u[2]) * inv_cs2s;
                        const C wk = C(SL::w(k));
                        const C eqA = wk * (muA + cAc * eu);
                        const C eqB = wk * (muB + cBc * eu);
                        push(std::integral_constant<int, A0 + k>{}, std::integral_constant<int, A0 + SL::opp(k)>{},
                             SL::ex(k), SL::ey(k), SL::ez(k), a[k] - wA * (a[k] - eqA));
                        push(std::integral_constant<int, B0 + k>{}, std::integral_constant<int, B0 + SL::opp(k)>{},
                             SL::ex(k), SL::ey(k), SL::ez(k), b[k] - wB * (b[k] - eqB));
                    });
                }
            } else if constexpr (MODE == MODE_MOMENTS) {
                const double vals[kNumMom] = {m.phi, sA, sB, m.muA, m.muB, double(p_h),
                                              double(u[0]), double(u[1]), double(u[2])};
#pragma unroll
                for (int i = 0; i < kNumMom; ++i) {
                    if (P.mout[i]) {
                        if (P.mout_f32) static_cast<float*>(P.mout[i])[idx] = float(vals[i]);
                        else static_cast<double*>(P.mout[i])[idx] = vals[i];
                    }
                }
            } else {  // MODE_DIAG
                const double u2 = double(u[0]) * double(u[0]) + double(u[1]) * double(u[1]) +
                                  double(u[2]) * double(u[2]);
                const double g2 = double(grad[0]) * double(grad[0]) + double(grad[1]) * double(grad[1]) +
                                  double(grad[2]) * double(grad[2]);
                acc[0] += sA;
                acc[1] += sB;
                acc[2] += m.phi;
                acc[3] += 0.5 * P.rho0 * u2;
                acc[4] = fmax(acc[4], sqrt(u2));
                acc[5] += (4.0 / P.W) * m.phi * (1.0 - m.phi);
                acc[6] += 0.5 * P.W * P.W * g2 + dwell(m.phi) + 0.5 * P.lam * (m.muA * m.muA + m.muB * m.muB);
                acc[7] += (isfinite(m.phi) && isfinite(sA) && isfinite(sB)) ? 0.0 : 1.0;
            }
        }
        if constexpr (STENCIL) {
            // the next plane becomes the current one
#pragma unroll
            for (int k = 0; k < QS; ++k) { cg[k] = ng[k]; ca[k] = na[k]; cb[k] = nb[k]; }
            c_ps = n_ps; c_cA = n_cA; c_cB = n_cB;
            __syncthreads();
        }
    }

    if constexpr (MODE == MODE_DIAG) {
        const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_reduce_store<8, NT>(acc, 4, P.partials + 8 * bid);
    } else if constexpr (MODE == MODE_STEP) {
        if (P.mean_subtract) {
            const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            block_reduce_store<1, NT>(acc, -1, P.partials + bid);
        }
    }
}

// ---------------------------------------------------------------------------
// initialisation at rest (Section 4.2.1): equilibrium populations from (phi_0, mu_0)

template <class SL, class FL, int PREC>
__global__ void __launch_bounds__(256) k_init(const KParams P, const double* __restrict__ phi0,
                                              const double* __restrict__ muA0,
                                              const double* __restrict__ muB0) {
    constexpr int QS = SL::Q;
    constexpr int QF = FL::Q;
    constexpr int G0 = QF, A0 = QF + QS, B0 = QF + 2 * QS;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= P.nx) return;
    const int idx = (z * P.ny + y) * P.nx + x;
    const double phi = phi0[idx], muA = muA0[idx], muB = muB0[idx];
    const double pp = interp_p(phi);
    const double cA = muA + P.c0A + pp * (P.c1A - P.c0A);  // Eq. species_closure
    const double cB = muB + P.c0B + pp * (P.c1B - P.c0B);
    const double domega = -(muA * (P.c0A - P.c1A) + muB * (P.c0B - P.c1B));
    const double S0 = P.mphi_w2 * (P.lam * interp_dp(phi) * domega - dwell_d(phi));
#pragma unroll
    for (int k = 0; k < QS; ++k) {
        const double wk = SL::w(k);
        st_pop<PREC>(P.dst[G0 + k], idx, k == 0, P.swref[G0 + k], P.sscale[G0 + k],
                     typename Stor<PREC>::C(wk * phi - 0.5 * wk * S0));
        const double hA = k == 0 ? cA - (1.0 - wk) * muA : wk * muA;
        const double hB = k == 0 ? cB - (1.0 - wk) * muB : wk * muB;
        st_pop<PREC>(P.dst[A0 + k], idx, k == 0, P.swref[A0 + k], P.sscale[A0 + k], typename Stor<PREC>::C(hA));
        st_pop<PREC>(P.dst[B0 + k], idx, k == 0, P.swref[B0 + k], P.sscale[B0 + k], typename Stor<PREC>::C(hB));
    }
    if constexpr (QF > 0) {
        double grad[3] = {0.0, 0.0, 0.0}, lap = 0.0;
#pragma unroll
        for (int k = 1; k < STL::Q; ++k) {
            const int xn = map_coord(x + STL::ex(k), P.nx, P.wall_x);
            const int yn = map_coord(y + STL::ey(k), P.ny, P.wall_y);
            const int zn = map_coord(z + STL::ez(k), P.nz, P.wall_z);
            const double v = phi0[(zn * P.ny + yn) * P.nx + xn];
            grad[0] += 3.0 * STL::w(k) * STL::ex(k) * v;
            grad[1] += 3.0 * STL::w(k) * STL::ey(k) * v;
            grad[2] += 3.0 * STL::w(k) * STL::ez(k) * v;
            lap += 6.0 * STL::w(k) * (v - phi);
        }
        const double phi_ref = P.mean_subtract ? *P.phi_ref : 0.0;
        const double bracket = P.cap * (dwell_d(phi) * P.inv_W2 - lap);
        const double buoy = (phi - phi_ref) * P.drho;
        const double F[3] = {buoy * P.gx + bracket * grad[0], buoy * P.gy + bracket * grad[1],
                             buoy * P.gz + bracket * grad[2]};
#pragma unroll
        for (int k = 0; k < QF; ++k) {
            const double eF = FL::ex(k) * F[0] + FL::ey(k) * F[1] + FL::ez(k) * F[2];
            // f^eq at p_h = 0, u = 0 minus F_k / 2 with Gamma_k(u = 0) = w_k
            st_pop<PREC>(P.dst[k], idx, k == 0, P.swref[k], P.sscale[k],
                         typename Stor<PREC>::C(-0.5 * FL::w(k) * eF));
        }
    }
}

// ---------------------------------------------------------------------------
// canonical FP64 population access and reductions

template <int PREC>
__global__ void __launch_bounds__(256) k_get_pops(const KParams P, int nslots, long long nodes,
                                                  double* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nodes || s >= nslots) return;
    const bool rest = P.srest[s] != 0;
    out[s * nodes + i] = double(ld_pop<PREC>(P.src[s], int(i), rest, P.swref[s], P.sinv[s]));
}

template <int PREC>
__global__ void __launch_bounds__(256) k_set_pops(const KParams P, int nslots, long long nodes,
                                                  const double* __restrict__ in) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nodes || s >= nslots) return;
    const bool rest = P.srest[s] != 0;
    st_pop<PREC>(P.dst[s], int(i), rest, P.swref[s], P.sscale[s],
                 typename Stor<PREC>::C(in[s * nodes + i]));
}

// per-work-group sums of a double field (grid-stride, fixed order)
template <int NT = 256>
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ v, long long n,
                                                      double* __restrict__ partials) {
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        acc[0] += v[i];
    block_reduce_store<1, 256>(acc, -1, partials + blockIdx.x);
}

// final fixed-order reduction of per-work-group partials (one work-group).
// partials are [nparts][N]; out[i] = scale[i] * reduce_i(partials[.][i])
template <int N>
__global__ void __launch_bounds__(256) k_finalize(const double* __restrict__ partials, int nparts,
                                                  int maxslot, double scale0, double* __restrict__ out) {
    double acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 256) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double v = partials[p * N + i];
            acc[i] = (i == maxslot) ? fmax(acc[i], v) : acc[i] + v;
        }
    }
    double res[N];
    block_reduce_store<N, 256>(acc, maxslot, res);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = (i == 0) ? res[i] * scale0 : res[i];
    }
}

}  // namespace lbm

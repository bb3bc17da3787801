"""Closed-form solutions used to pin the oracle (test infrastructure only)."""

import math

import numpy as np
from scipy.optimize import brentq
from scipy.special import erfc


def tanh_profile(x, W):
    """Equilibrium plane interface, Eq. tanh: phi_0(x) = (1 + tanh(2x / W)) / 2."""
    return 0.5 * (1.0 + np.tanh(2.0 * np.asarray(x) / W))


# ----------------------------------------------------------------------------------------
# Ternary diffusion couple, Section 4.1 (Eqs. Stefan ... Solution_Mu)
#
# Phase 0 occupies x < x_I(t), phase 1 occupies x > x_I(t).  In each bulk phase
# c^alpha = mu^alpha + c_pi^alpha,eq, so mu^alpha diffuses with the mobility of that
# phase: M_L on the left (phase 0), M_R on the right (phase 1); Section 2.3 lets the
# mobility depend on the phase.  The similarity solution x_I = xi sqrt(t) of
# Eq. InterfPosition has the erfc profiles of Eq. Solution_Mu on each side,
#   mu_L = mu_-inf + A_L erfc(-x / (2 sqrt(M_L t))),  mu_R = mu_+inf + A_R erfc(x / (2 sqrt(M_R t))),
# both equal to mu_int at x_I.  The composition balance Eq. StefanInt2 across the
# moving interface, V [c] = J_L - J_R with J = -M d mu / dx, V = xi / (2 sqrt(t)) and
# [c] = c_0,eq - c_1,eq, gives for each component (eta_s = xi / (2 sqrt(M_s)),
# a_L = sqrt(M_L) exp(-eta_L^2) / erfc(-eta_L), a_R = sqrt(M_R) exp(-eta_R^2) / erfc(eta_R)):
#
#   mu_int (a_L + a_R) = a_L mu_-inf + a_R mu_+inf - (xi/2) dc sqrt(pi)
#
# and the interface condition omega_0(mu_int) = omega_1(mu_int) (Section 4.1),
# i.e. sum_alpha dc^alpha mu_int^alpha = 0, closes the system for xi.  With
# M_L = M_R this restates the transcendental equation the paper cites but does not
# print.  A mobility M given as one number applies to both sides; a pair is
# (phase 0, phase 1).

def _sides(M):
    if np.ndim(M) == 0:
        return float(M), float(M)
    return float(M[0]), float(M[1])


def dc_interface_mu(xi, mu_minus, mu_plus, dc, M):
    """Interface potential of one component for a given xi (see above)."""
    ML, MR = _sides(M)
    eL, eR = xi / (2.0 * math.sqrt(ML)), xi / (2.0 * math.sqrt(MR))
    aL = math.sqrt(ML) * math.exp(-eL * eL) / erfc(-eL)
    aR = math.sqrt(MR) * math.exp(-eR * eR) / erfc(eR)
    return (aL * mu_minus + aR * mu_plus - 0.5 * xi * dc * math.sqrt(math.pi)) / (aL + aR)


def dc_residual(xi, mu_minus, mu_plus, dc, M):
    """sum_alpha dc^alpha mu_int^alpha(xi); zero at the self-similar solution."""
    return sum(dc[a] * dc_interface_mu(xi, mu_minus[a], mu_plus[a], dc[a], M[a]) for a in range(2))


def dc_roots(mu_minus, mu_plus, dc, M, lo=-4.0, hi=4.0, n=4001):
    """All roots of the residual in [lo, hi]: sign changes on a fine grid, each refined
    by bisection (Brent).  The scan is used because the equation may have several
    solutions.  M[alpha] is the mobility of component alpha (one number, or the pair of
    phase 0 and phase 1)."""
    xs = np.linspace(lo, hi, n)
    r = np.array([dc_residual(x, mu_minus, mu_plus, dc, M) for x in xs])
    roots = []
    for i in range(n - 1):
        if r[i] == 0.0:
            roots.append(xs[i])
        elif r[i] * r[i + 1] < 0.0:
            roots.append(brentq(dc_residual, xs[i], xs[i + 1], args=(mu_minus, mu_plus, dc, M),
                                xtol=1e-15, rtol=1e-15))
    return roots


def dc_mu_profile(x, t, xi, mu_minus, mu_plus, dc, M):
    """mu^alpha(x, t) of Eq. Solution_Mu for one component (M one number, or the pair
    of phase 0 on the left and phase 1 on the right)."""
    ML, MR = _sides(M)
    x = np.asarray(x, dtype=float)
    mu_int = dc_interface_mu(xi, mu_minus, mu_plus, dc, M)
    left = mu_minus + (mu_int - mu_minus) * erfc(-x / (2.0 * math.sqrt(ML * t))) / erfc(-xi / (2.0 * math.sqrt(ML)))
    right = mu_plus + (mu_int - mu_plus) * erfc(x / (2.0 * math.sqrt(MR * t))) / erfc(xi / (2.0 * math.sqrt(MR)))
    return np.where(x < xi * math.sqrt(t), left, right)


# ----------------------------------------------------------------------------------------
# Other closed forms

def poiseuille(z, N, F, rho0, nu):
    """Steady plane Poiseuille flow driven by a body force F between half-way walls at
    z = -1/2 and z = N - 1/2: u(z) = F (z + 1/2)(N - 1/2 - z) / (2 rho0 nu)."""
    z = np.asarray(z, dtype=float)
    return F * (z + 0.5) * (N - 0.5 - z) / (2.0 * rho0 * nu)


def shrinking_disk_r2(R0, M_phi, t, dim=2):
    """Curvature-driven motion with no thermodynamic driving force: from the
    Gibbs-Thomson relation Eq. Gibbs-Thomson with Delta omega = 0 and equal
    compositions, V = -(delta/beta) kappa = -M_phi kappa (Eqs. Delta, KineticCoeff),
    so R^2 = R0^2 - 2 (dim - 1) M_phi t."""
    return R0 ** 2 - 2.0 * (dim - 1) * M_phi * t


def laplace_jump(sigma, R, dim=2):
    """Pressure jump across a static drop interface: (dim - 1) sigma / R."""
    return (dim - 1) * sigma / R

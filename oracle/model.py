"""Thermodynamics and source terms of the model (test infrastructure only).

Each function follows one formula of Section 2 of the paper; names follow its
notation (phi = phase field, mu = dimensionless diffusion potential mu-bar,
c_eq[pi][alpha] = equilibrium composition of phase pi for component alpha).
All functions are elementwise on numpy arrays and keep the input dtype, so
complex inputs propagate complex-step derivatives.
"""

import numpy as np


def p(phi):
    """Interpolation function p(phi) = 3 phi^2 - 2 phi^3 (Section 2.2)."""
    return 3.0 * phi ** 2 - 2.0 * phi ** 3


def dp(phi):
    """p'(phi) = 6 phi (1 - phi)."""
    return 6.0 * phi * (1.0 - phi)


def omega_dw(phi):
    """Double well omega_dw(phi) = 8 phi^2 (1 - phi)^2 (Section 2.2)."""
    return 8.0 * phi ** 2 * (1.0 - phi) ** 2


def domega_dw(phi):
    """omega_dw'(phi) = 16 phi (1 - phi) (1 - 2 phi)."""
    return 16.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi)


def grand_potential(mu, c_eq_pi, kappa_pi=None):
    """Dimensionless grand potential of phase pi, Eq. dimless_grand_potentials:
    omega_pi(mu) = -1/2 sum_alpha (mu_alpha^2 + 2 mu_alpha c_pi^alpha,eq).
    ``mu`` holds the potentials of the independent compositions (mu_A, mu_B for the
    ternary fluid; more for the N-component extension of the conclusion, with the same
    quadratic free energies of Eq. Taylor); ``c_eq_pi`` the phase-pi compositions.

    General curvatures (Eq. Taylor with a full matrix K_pi^{alpha beta}): with
    kappa_pi = K (K_pi)^-1 (K the reference curvature that scales mu and omega) the
    Legendre transform of the quadratic free energy gives
    omega_pi(mu) = -1/2 mu . kappa_pi mu - mu . c_pi^eq; kappa_pi = identity is the
    paper's model.  kappa_pi = (k_AA, k_AB, k_BB), symmetric."""
    if kappa_pi is None:
        return -0.5 * sum(mu[a] ** 2 + 2.0 * mu[a] * c_eq_pi[a] for a in range(len(mu)))
    kAA, kAB, kBB = kappa_pi
    quad = kAA * mu[0] ** 2 + 2.0 * kAB * mu[0] * mu[1] + kBB * mu[1] ** 2
    return -0.5 * quad - (mu[0] * c_eq_pi[0] + mu[1] * c_eq_pi[1])


def delta_omega(mu, c_eq, kappa=None):
    """Driving force Delta omega = omega_0 - omega_1 (Section 2.2); kappa = (kappa_0,
    kappa_1) or None for the paper's equal unit curvatures."""
    if kappa is None:
        return grand_potential(mu, c_eq[0]) - grand_potential(mu, c_eq[1])
    return grand_potential(mu, c_eq[0], kappa[0]) - grand_potential(mu, c_eq[1], kappa[1])


def _kappa_phi(phi, kappa):
    """kappa(phi) = p(1 - phi) kappa_0 + p(phi) kappa_1: the d c / d mu of the
    interpolated grand potential."""
    return tuple(p(1.0 - phi) * kappa[0][i] + p(phi) * kappa[1][i] for i in range(3))


def closure_mu(c, phi, c_eq, kappa=None):
    """Inversion of the species closure, Eq. PotChem (Section 2.3/2.5):
    mu^alpha = c^alpha - p(1 - phi) c_0^alpha,eq - p(phi) c_1^alpha,eq.
    ``c`` holds the compositions (c_A, c_B, ...); returns their potentials.  With
    general curvatures (two compositions) c - c^eq(phi) = kappa(phi) mu is solved for
    mu (a 2 x 2 system)."""
    if kappa is None:
        return tuple(c[a] - p(1.0 - phi) * c_eq[0][a] - p(phi) * c_eq[1][a] for a in range(len(c)))
    r = [c[a] - p(1.0 - phi) * c_eq[0][a] - p(phi) * c_eq[1][a] for a in range(2)]
    kAA, kAB, kBB = _kappa_phi(phi, kappa)
    det = kAA * kBB - kAB * kAB
    return ((kBB * r[0] - kAB * r[1]) / det, (kAA * r[1] - kAB * r[0]) / det)


def closure_c(mu, phi, c_eq, kappa=None):
    """Forward closure, Eq. species_closure: c^alpha = -d omega/d mu^alpha with the
    parabolic grand potentials, i.e. c = mu + p(1 - phi) c_0 + p(phi) c_1; with general
    curvatures c = c^eq(phi) + kappa(phi) mu."""
    if kappa is None:
        return tuple(mu[a] + p(1.0 - phi) * c_eq[0][a] + p(phi) * c_eq[1][a] for a in range(len(mu)))
    kAA, kAB, kBB = _kappa_phi(phi, kappa)
    return (p(1.0 - phi) * c_eq[0][0] + p(phi) * c_eq[1][0] + kAA * mu[0] + kAB * mu[1],
            p(1.0 - phi) * c_eq[0][1] + p(phi) * c_eq[1][1] + kAB * mu[0] + kBB * mu[1])


def bulk_free_energy(mu, phi, kappa=None):
    """Bulk free-energy density above the reference equilibrium, in units of K:
    1/2 mu . kappa(phi) mu (|mu|^2 / 2 for the paper's unit curvatures)."""
    if kappa is None:
        return 0.5 * sum(m ** 2 for m in mu)
    kAA, kAB, kBB = _kappa_phi(phi, kappa)
    return 0.5 * (kAA * mu[0] ** 2 + 2.0 * kAB * mu[0] * mu[1] + kBB * mu[1] ** 2)


def tau_phi(W, M_phi):
    """Phase-field relaxation time from the scaled mobility M_phi = W^2 / tau_phi (Section 2.2)."""
    return W ** 2 / M_phi


def source_phi(phi, mu, prm):
    """Phase-field source term, Eq. SourceTerm_Phi:
    S = -(1/tau_phi) omega_dw'(phi) + (lambda / tau_phi) p'(phi) Delta omega(mu)."""
    tp = tau_phi(prm.W, prm.M_phi)
    return -domega_dw(phi) / tp + (prm.lam / tp) * dp(phi) * delta_omega(mu, prm.c_eq, prm.kappa)


def mobility(phi, M_pair):
    """Linear mobility interpolation M(phi) = M_0 (1 - phi) + M_1 phi (Section 2.3)."""
    return M_pair[0] * (1.0 - phi) + M_pair[1] * phi


def viscosity(phi, nu_pair):
    """Phase-dependent kinematic viscosity.  The paper calls nu(phi) phase dependent
    (Eq. QDM) without a law; the reading taken is the same linear interpolation as
    the mobility: nu(phi) = nu_0 (1 - phi) + nu_1 phi."""
    return nu_pair[0] * (1.0 - phi) + nu_pair[1] * phi


def lambda_star(W, M_phi, M_alpha, c_eq):
    """Coupling constant that cancels the kinetic coefficient beta of
    Eq. KineticCoeff (Section 2.4):
    beta = (2/3) W / (lambda M_phi) - (19/120) sum_alpha W (c_0 - c_1)^2 / M^alpha = 0."""
    s = sum((c_eq[0][a] - c_eq[1][a]) ** 2 / M_alpha[a] for a in range(len(M_alpha)))
    return (2.0 / 3.0) / (M_phi * (19.0 / 120.0) * s)


def capillary_length(W, lam):
    """delta = (2/3) W / lambda, Eq. Delta (Section 2.4)."""
    return (2.0 / 3.0) * W / lam

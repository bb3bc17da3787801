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


def grand_potential(mu, c_eq_pi):
    """Dimensionless grand potential of phase pi, Eq. dimless_grand_potentials:
    omega_pi(mu) = -1/2 sum_alpha (mu_alpha^2 + 2 mu_alpha c_pi^alpha,eq).
    ``mu`` is a pair (mu_A, mu_B); ``c_eq_pi`` the pair of phase-pi compositions."""
    return -0.5 * sum(mu[a] ** 2 + 2.0 * mu[a] * c_eq_pi[a] for a in range(2))


def delta_omega(mu, c_eq):
    """Driving force Delta omega = omega_0 - omega_1 (Section 2.2)."""
    return grand_potential(mu, c_eq[0]) - grand_potential(mu, c_eq[1])


def closure_mu(c, phi, c_eq):
    """Inversion of the species closure, Eq. PotChem (Section 2.3/2.5):
    mu^alpha = c^alpha - p(1 - phi) c_0^alpha,eq - p(phi) c_1^alpha,eq.
    ``c`` is a pair (c_A, c_B); returns the pair (mu_A, mu_B)."""
    return tuple(c[a] - p(1.0 - phi) * c_eq[0][a] - p(phi) * c_eq[1][a] for a in range(2))


def closure_c(mu, phi, c_eq):
    """Forward closure, Eq. species_closure: c^alpha = -d omega/d mu^alpha with the
    parabolic grand potentials, i.e. c = mu + p(1 - phi) c_0 + p(phi) c_1."""
    return tuple(mu[a] + p(1.0 - phi) * c_eq[0][a] + p(phi) * c_eq[1][a] for a in range(2))


def tau_phi(W, M_phi):
    """Phase-field relaxation time from the scaled mobility M_phi = W^2 / tau_phi (Section 2.2)."""
    return W ** 2 / M_phi


def source_phi(phi, mu, prm):
    """Phase-field source term, Eq. SourceTerm_Phi:
    S = -(1/tau_phi) omega_dw'(phi) + (lambda / tau_phi) p'(phi) Delta omega(mu)."""
    tp = tau_phi(prm.W, prm.M_phi)
    return -domega_dw(phi) / tp + (prm.lam / tp) * dp(phi) * delta_omega(mu, prm.c_eq)


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
    s = sum((c_eq[0][a] - c_eq[1][a]) ** 2 / M_alpha[a] for a in range(2))
    return (2.0 / 3.0) / (M_phi * (19.0 / 120.0) * s)


def capillary_length(W, lam):
    """delta = (2/3) W / lambda, Eq. Delta (Section 2.4)."""
    return (2.0 / 3.0) * W / lam

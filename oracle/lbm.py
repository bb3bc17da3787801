"""The discrete lattice-Boltzmann map of the paper, written plainly (test infrastructure only).

One time step, Section 3 of the paper, in this order:

  pass 1, every node (Eqs. Moment0_c_alpha, Moment0_Phi, PotChem, SourceTerm_Phi)
      c^alpha = sum_k h_k^alpha
      phi*    = sum_k g_k
      phi     = phi* + S(phi*, mu(c, phi*)) / 2          (one predictor step, see below)
      mu      = mu(c, phi),   S = S(phi, mu)
  pass 2, every node, flow only (Eqs. DerivDirec_Grad ... Laplacian, SurfaceTension_Force,
      HydroPressure, Velocity)
      grad phi, lap phi on the fluid lattice from the pass-1 phi field
      F   = (phi - phi_ref) drho g + (3/2) sigma W [omega_dw'(phi)/W^2 - lap phi] grad phi
      p_h = sum_k f_k,   rho0 u = (1/c_s^2) sum_k f_k e_k + F/2
  collision (Eqs. LBE_FluidFlow, ForcingTerm, GammaFunction, Feq, LBE_Phi, Geq,
      Source_LBE_Phi, LBE_c_alpha, Heq), BGK with rate 1/(tau + 1/2) and D = tau c_s^2
  streaming: X_k(x + e_k) <- X*_k(x); across a wall the population returns to its own
      node in the opposite direction (half-way bounce-back, Section 4.2.4).

Readings of points the paper leaves open (each is also a field of ``Params``):
  * phi = sum g + S/2 is implicit in phi (S depends on phi).  It is resolved by one
    predictor step: S is first evaluated at phi* = sum g, then at the corrected phi.
  * All moments of step n come from the populations of step n; nothing is lagged.
  * The grad/Laplacian stencil always uses the fluid lattice (D2Q9 in 2D, D3Q19 in 3D)
    with the factor 3 = 1/c_s^2 of that lattice; walls use mirror ghosts
    phi(-1) = phi(0), phi(N) = phi(N-1) (zero normal gradient at a half-way wall).
  * nu(phi) is interpolated linearly (see ``model.viscosity``).
  * The gravity force uses (phi - phi_ref) drho g.  phi_ref = 0 (the paper's form)
    unless ``gravity_mean_subtract`` is set, for fully periodic boxes, where
    phi_ref is the domain mean of phi of the previous step (of phi_0 at step 0).
  * The scalar lattices D2Q5 / D3Q7 use their own c_s^2 (1/3, 1/4) in the rates and
    in the c_k.u / c_s^2 terms of g^eq and h^eq.

Arrays are indexed [k][z][y][x] (2D grids have nz = 1).
"""

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

from . import geometry, model
from .lattices import BY_NAME, D2Q9, D3Q19, moment_basis


@dataclass
class Params:
    nx: int
    ny: int
    nz: int = 1
    fluid: Optional[str] = None          # None, "D2Q9" or "D3Q19"
    scalar: str = "D2Q5"                 # "D2Q5", "D3Q7" or the paper's "D2Q9", "D3Q19"
    bc: Tuple[str, str, str] = ("periodic", "periodic", "periodic")   # per axis x, y, z
    W: float = 4.0
    lam: float = 1.0
    M_phi: float = 0.1
    M_A: Tuple[float, float] = (0.1, 0.1)      # (phase 0, phase 1)
    M_B: Tuple[float, float] = (0.1, 0.1)
    c_eq: Tuple[Tuple[float, float], Tuple[float, float]] = ((0.2, 0.1), (0.6, 0.3))  # [phase][A, B]
    rho0: float = 1.0
    drho: float = 0.0
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    sigma: float = 0.0
    nu: Tuple[float, float] = (0.1, 0.1)       # (phase 0, phase 1)
    gravity_mean_subtract: bool = False
    collision: str = "BGK"                      # "BGK" (the paper's), "TRT" or "MRT"
    # MRT rates of the moments the transport coefficients leave free: f (bulk, third
    # order, fourth order); g, h^A, h^B (second, third, fourth order)
    mrt_rates: Tuple[Tuple[float, float, float], Tuple[float, float, float]] = ((1.2, 1.1, 1.2), (1.1, 1.0, 1.2))
    variable_density: bool = False              # False: Boussinesq (the paper's); True: rho(phi)
    # general curvatures: ((k_AA, k_AB, k_BB) of phase 0, same of phase 1) = K (K_pi)^-1;
    # None is the paper's K_pi = K identity
    kappa: Optional[Tuple[Tuple[float, float, float], Tuple[float, float, float]]] = None
    trt_magic: Tuple[float, float] = (3.0 / 16.0, 0.25)   # TRT Lambda of (f, the scalar lattices)
    # N components (the conclusion's extension, same quadratic free energies): mobilities
    # (phase 0, phase 1) of the compositions beyond A and B, named C, D, ...; c_eq then
    # lists 2 + len(M_x) compositions per phase
    M_x: Tuple[Tuple[float, float], ...] = ()

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncomp(self):
        """Number of independent compositions (2 for the ternary fluid)."""
        return 2 + len(self.M_x)

    @property
    def dim(self):
        return BY_NAME[self.scalar].dim

    @property
    def slat(self):
        return BY_NAME[self.scalar]

    @property
    def flat(self):
        return BY_NAME[self.fluid] if self.fluid else None

    @property
    def stencil_lattice(self):
        return D2Q9 if self.dim == 2 else D3Q19

    def with_(self, **kw):
        return replace(self, **kw)


@dataclass
class State:
    g: np.ndarray                 # [Qs][z][y][x]
    hA: np.ndarray
    hB: np.ndarray
    f: Optional[np.ndarray] = None  # [Qf][z][y][x] or None without flow
    phi_ref: complex = 0.0
    step: int = 0
    hx: Tuple[np.ndarray, ...] = ()  # compositions beyond A, B (C, D, ...)

    def copy(self):
        return State(self.g.copy(), self.hA.copy(), self.hB.copy(),
                     None if self.f is None else self.f.copy(), self.phi_ref, self.step,
                     tuple(h.copy() for h in self.hx))


# ----------------------------------------------------------------------------------------
# neighbour access and streaming

def _padded(field, bc):
    """Pad a [z][y][x] field by one node per side: periodic axes wrap, wall axes repeat
    the edge value (mirror ghost of a half-way wall)."""
    out = field
    for ax, b in ((0, bc[2]), (1, bc[1]), (2, bc[0])):
        pw = [(0, 0)] * 3
        pw[ax] = (1, 1)
        out = np.pad(out, pw, mode="wrap" if b == "periodic" else "edge")
    return out


def neighbour(field, e, bc):
    """Value of ``field`` at x + e for every node x (|e_i| <= 1)."""
    P = _padded(field, bc)
    nz, ny, nx = field.shape
    ex, ey, ez = (int(v) for v in e)
    return P[1 + ez:1 + ez + nz, 1 + ey:1 + ey + ny, 1 + ex:1 + ex + nx]


def _outside_mask(shape, e, bc):
    """True where x - e lies outside the domain across a wall axis."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape, dtype=bool)
    for coord, n, comp, b in ((x, nx, e[0], bc[0]), (y, ny, e[1], bc[1]), (z, nz, e[2], bc[2])):
        if b == "walls" and comp != 0:
            src = coord - comp
            out |= (src < 0) | (src >= n)
    return out


def stream(post, lat, bc):
    """Streaming of post-collision populations ``post[k]`` (LBE left-hand sides):
    X_k(x) = X*_k(x - e_k) when x - e_k is inside the domain (periodic axes wrap),
    otherwise X*_opp(k)(x): the population that left x towards the wall comes back
    reversed (half-way bounce-back with a wall at rest)."""
    new = np.empty_like(post)
    for k in range(lat.Q):
        e = lat.e[k]
        rolled = np.roll(post[k], shift=(int(e[2]), int(e[1]), int(e[0])), axis=(0, 1, 2))
        mask = _outside_mask(post.shape[1:], e, bc)
        new[k] = np.where(mask, post[lat.opp[k]], rolled)
    return new


# ----------------------------------------------------------------------------------------
# finite-difference stencils of Section 3.1

def gradient(phi, bc, lat):
    """Isotropic gradient, Eqs. DerivDirec_Grad and Grad:
    e_k . grad phi = [phi(x + e_k) - phi(x - e_k)] / 2,
    grad phi = 3 sum_k w_k e_k (e_k . grad phi)."""
    grad = [np.zeros_like(phi) for _ in range(3)]
    for k in range(lat.Q):
        e = lat.e[k]
        d = 0.5 * (neighbour(phi, e, bc) - neighbour(phi, -e, bc))
        for a in range(3):
            if e[a] != 0:
                grad[a] = grad[a] + 3.0 * lat.w[k] * e[a] * d
    return grad


def laplacian(phi, bc, lat):
    """Isotropic Laplacian, Eqs. DerivDirect_Laplacian and Laplacian:
    lap phi = 3 sum_{k != 0} w_k [phi(x + e_k) - 2 phi(x) + phi(x - e_k)]."""
    lap = np.zeros_like(phi)
    for k in range(1, lat.Q):
        e = lat.e[k]
        lap = lap + 3.0 * lat.w[k] * (neighbour(phi, e, bc) - 2.0 * phi + neighbour(phi, -e, bc))
    return lap


# ----------------------------------------------------------------------------------------
# equilibria and forcing of Section 3

def _edot(e, vec):
    return e[0] * vec[0] + e[1] * vec[1] + e[2] * vec[2]


def gamma_k(lat, k, u):
    """Eq. GammaFunction."""
    eu = _edot(lat.e[k], u)
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    cs2 = lat.cs2
    return lat.w[k] * (1.0 + eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2))


def forcing_k(lat, k, u, F):
    """He-Shan-Doolen forcing population, Eq. ForcingTerm: F_k = Gamma_k (c_k - u) . F."""
    e = lat.e[k]
    return gamma_k(lat, k, u) * ((e[0] - u[0]) * F[0] + (e[1] - u[1]) * F[1] + (e[2] - u[2]) * F[2])


def f_equilibrium_k(lat, k, p_h, u, rho0, Fk):
    """He-Luo incompressible equilibrium with the forcing shift, Eq. Feq."""
    eu = _edot(lat.e[k], u)
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    cs2 = lat.cs2
    return lat.w[k] * (p_h + rho0 * cs2 * (eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2))) - 0.5 * Fk


def g_equilibrium_k(lat, k, phi, u, Gk):
    """Phase-field equilibrium, Eq. Geq: w_k phi (1 + c_k.u / c_s^2) - G_k / 2."""
    return lat.w[k] * phi * (1.0 + _edot(lat.e[k], u) / lat.cs2) - 0.5 * Gk


def h_equilibrium_k(lat, k, c, mu, u):
    """Composition equilibrium, Eq. Heq: c - (1 - w_0) mu for k = 0,
    w_k mu + w_k c (c_k.u) / c_s^2 otherwise."""
    if k == 0:
        return c - (1.0 - lat.w[0]) * mu
    return lat.w[k] * mu + lat.w[k] * c * _edot(lat.e[k], u) / lat.cs2


def rate(D, cs2):
    """BGK rate 1/(tau + 1/2) with the transport coefficient D = tau c_s^2 (delta t = 1)."""
    return 1.0 / (D / cs2 + 0.5)


def trt_partner_rate(w, magic):
    """Two-relaxation-time collision (the TRT operator the paper names as an alternative
    to BGK in Section 3; Ginzburg's form): the rate that the transport coefficient does
    not fix follows from the magic parameter Lambda = (1/w+ - 1/2)(1/w- - 1/2)."""
    return 1.0 / (0.5 + magic / (1.0 / w - 0.5))


_BASES = {}


def _basis(lat):
    if lat.name not in _BASES:
        rows, orders = moment_basis(lat)
        M = np.array([[float(a) for a in r] for r in rows])
        D = np.array([float(sum(w * a * a for w, a in zip(lat.w_exact, r))) for r in rows])
        _BASES[lat.name] = (M, D, orders)
    return _BASES[lat.name]


def mrt_collide(X, eqs, src, lat, rates):
    """Multiple-relaxation-time collision (the MRT alternative the paper names in
    Section 3): the non-equilibrium part n = X - eqs (shifted equilibria, as in BGK)
    is taken to the weighted-orthogonal moment basis M of lattices.moment_basis, moment
    i is relaxed at rates[i] (a scalar or a field), and the result is taken back:
        X*_k = X_k - sum_i (w_k M_ik / <M_i, M_i>) rates_i (M n)_i + src_k.
    Equal rates give the BGK collision; even/odd-order rates w+ / w- give TRT."""
    M, D, _ = _basis(lat)
    n = [X[k] - eqs[k] for k in range(lat.Q)]
    m = [sum(M[i, k] * n[k] for k in range(lat.Q) if M[i, k] != 0.0) * rates[i] / D[i] for i in range(lat.Q)]
    return np.stack([X[k] - lat.w[k] * sum(M[i, k] * m[i] for i in range(lat.Q) if M[i, k] != 0.0) + src[k]
                     for k in range(lat.Q)])


def mrt_rates(lat, transport_rate, free, fluid):
    """Rate of each row of the moment basis.  Orders 0 and 1 of f are conserved by the
    collision (their n moments vanish; rate 1).  f: the traceless second order relaxes
    at the viscous rate, the trace at free[0], third and fourth orders at free[1],
    free[2].  g, h: the first order (the diffusive flux) at the mobility rate, second,
    third and fourth orders at free[0], free[1], free[2]; order 0 with the other even
    orders at free[0] (it is conserved for h; for g the phi predictor leaves a small
    S difference, which BGK and TRT relax with the even rate too)."""
    _, _, orders = _basis(lat)
    rates, first2 = [], True
    for o in orders:
        if fluid:
            if o <= 1:
                rates.append(1.0)
            elif o == 2:
                rates.append(free[0] if first2 else transport_rate)
                first2 = False
            else:
                rates.append(free[1] if o == 3 else free[2])
        else:
            rates.append(free[0] if o == 0 else transport_rate if o == 1 else free[o - 2])
    return rates


def trt_collide(X, eqs, src, lat, w_sym, w_anti):
    """Post-collision populations of a TRT collision: the non-equilibrium part
    n_k = X_k - eqs_k (eqs: the shifted equilibrium of the BGK form) is split into its
    symmetric and antisymmetric parts over the pair (k, opp(k)), relaxed at w_sym and
    w_anti, and the source src_k is added:
        X*_k = X_k - w_sym (n_k + n_opp)/2 - w_anti (n_k - n_opp)/2 + src_k.
    With w_sym = w_anti this is the BGK collision X_k - w n_k + src_k."""
    n = [X[k] - eqs[k] for k in range(lat.Q)]
    out = []
    for k in range(lat.Q):
        o = lat.opp[k]
        out.append(X[k] - w_sym * 0.5 * (n[k] + n[o]) - w_anti * 0.5 * (n[k] - n[o]) + src[k])
    return np.stack(out)


# ----------------------------------------------------------------------------------------
# moments

COMP_NAMES = "ABCDEFGH"   # compositions in order: A, B (the ternary fluid), then C, D, ...


def scalar_moments(st, prm):
    """Pass 1: compositions, phase field (with the predictor), potentials and source."""
    c = tuple(h.sum(axis=0) for h in (st.hA, st.hB) + tuple(st.hx))   # Eq. Moment0_c_alpha
    phi_star = st.g.sum(axis=0)                          # sum_k g_k
    mu_star = model.closure_mu(c, phi_star, prm.c_eq, prm.kappa)
    S_star = model.source_phi(phi_star, mu_star, prm)
    phi = phi_star + 0.5 * S_star                        # Eq. Moment0_Phi (predictor)
    mu = model.closure_mu(c, phi, prm.c_eq, prm.kappa)   # Eq. PotChem
    S = model.source_phi(phi, mu, prm)                   # Eq. SourceTerm_Phi
    out = dict(phi=phi, phi_star=phi_star, S=S)
    for a in range(len(c)):
        out["c" + COMP_NAMES[a]] = c[a]
        out["mu" + COMP_NAMES[a]] = mu[a]
    return out


def force(phi, prm, phi_ref):
    """Total force of Eq. QDM: buoyancy plus capillary force Eq. SurfaceTension_Force."""
    lat = prm.stencil_lattice
    grad = gradient(phi, prm.bc, lat)
    lap = laplacian(phi, prm.bc, lat)
    bracket = model.domega_dw(phi) / prm.W ** 2 - lap
    cap = 1.5 * prm.sigma * prm.W
    return [(phi - phi_ref) * prm.drho * prm.g[a] + cap * bracket * grad[a] for a in range(3)]


def flow_moments(f, F, prm):
    """Eqs. HydroPressure and Velocity."""
    lat = prm.flat
    p_h = f.sum(axis=0)
    u = []
    for a in range(3):
        m = np.zeros_like(p_h)
        for k in range(lat.Q):
            if lat.e[k][a] != 0:
                m = m + f[k] * lat.e[k][a]
        u.append((m / lat.cs2 + 0.5 * F[a]) / prm.rho0)
    return p_h, u


def density(phi, prm):
    """rho(phi) of the variable-density model: rho0 in phase 0, rho0 + drho in phase 1,
    interpolated linearly like the viscosity (the paper interpolates the bulk densities
    without giving the law)."""
    return prm.rho0 + prm.drho * phi


def flow_moments_variable(f, phi, F_sb, prm):
    """Variable-density flow moments (the alternative of Section 3 after Eq. Velocity:
    the equilibrium carries the dimensionless pressure p* = p_h / (rho(phi) c_s^2), and
    the pressure and viscous forces join the total force).  Reading:
    f holds dimensionless populations, p* = sum_k f_k, p_h = rho c_s^2 p*;
    F_p = -p* c_s^2 grad rho;
    u* = sum_k f_k c_k + (F_sb + F_p) / (2 rho);
    F_mu,i = -(nu w+ / c_s^2) Pi_ij d_j rho, Pi = sum_k c_k c_k (f_k - f^eq_k(p*, u*)) with
    the unshifted equilibrium, w+ the rate of the viscous stress (nu(phi) / c_s^2 + 1/2)^-1;
    u = u* + F_mu / (2 rho).  Returns p_h, u and the total force."""
    lat = prm.flat
    cs2 = lat.cs2
    rho = density(phi, prm)
    grad = gradient(phi, prm.bc, prm.stencil_lattice)
    grho = [prm.drho * g for g in grad]
    p_star = f.sum(axis=0)
    F_p = [-p_star * cs2 * grho[a] for a in range(3)]
    u_star = []
    for a in range(3):
        m = np.zeros_like(p_star)
        for k in range(lat.Q):
            if lat.e[k][a] != 0:
                m = m + f[k] * lat.e[k][a]
        u_star.append(m + 0.5 * (F_sb[a] + F_p[a]) / rho)
    zero = np.zeros_like(p_star)
    Pi = [[zero, zero, zero], [zero, zero, zero], [zero, zero, zero]]
    for k in range(lat.Q):
        n = f[k] - f_equilibrium_k(lat, k, p_star, u_star, 1.0 / cs2, 0.0)
        e = lat.e[k]
        for i in range(3):
            for j in range(3):
                if e[i] != 0 and e[j] != 0:
                    Pi[i][j] = Pi[i][j] + e[i] * e[j] * n
    w_plus = rate(model.viscosity(phi, prm.nu), cs2)
    F_mu = [-(model.viscosity(phi, prm.nu) * w_plus / cs2) * sum(Pi[i][j] * grho[j] for j in range(3))
            for i in range(3)]
    u = [u_star[a] + 0.5 * F_mu[a] / rho for a in range(3)]
    F = [F_sb[a] + F_p[a] + F_mu[a] for a in range(3)]
    return rho * cs2 * p_star, u, F


def _flow(f, phi, prm, phi_ref):
    """p_h, u, total force and the forcing populations of the current state (either
    density model).  The forcing populations are in the units of f: F_k for the
    Boussinesq model, F_k / (rho c_s^2) for the variable-density one."""
    F = force(phi, prm, phi_ref)
    flat = prm.flat
    if not prm.variable_density:
        p_h, u = flow_moments(f, F, prm)
        return p_h, u, F, [forcing_k(flat, k, u, F) for k in range(flat.Q)]
    p_h, u, F = flow_moments_variable(f, phi, F, prm)
    scale = 1.0 / (density(phi, prm) * flat.cs2)
    return p_h, u, F, [forcing_k(flat, k, u, F) * scale for k in range(flat.Q)]


def moments(st, prm):
    """All macroscopic fields of the current state: phi, c, mu, S, p_h, u, F."""
    m = scalar_moments(st, prm)
    zero = np.zeros_like(m["phi"])
    if prm.fluid:
        p_h, u, F, _ = _flow(st.f, m["phi"], prm, st.phi_ref)
    else:
        F = [zero, zero, zero]
        p_h, u = zero, [zero, zero, zero]
    m.update(p=p_h, ux=u[0], uy=u[1], uz=u[2], F=F)
    return m


# ----------------------------------------------------------------------------------------
# init and step

def init(phi0, muA0, muB0, prm, phi_ref=None, c0=None, mu_x0=()):
    """Populations at rest from (phi_0, mu_0), with u = 0 and p_h = 0 (Section 4.2.1):
    c from the closure Eq. species_closure, every population set to its equilibrium
    including the -G_k/2 and -F_k/2 shifts, so that the moments of Eqs. Moment0_Phi
    and Velocity give back phi_0 + O(S) and u = 0.  c0 = (c^A, c^B) gives the
    compositions instead of the closure (the paper's own initial condition, Eq.
    Compos_Init with mu = 0, is not in equilibrium with the closure).  mu_x0 holds the
    initial potentials of the compositions beyond A and B (N components); c0 then lists
    every composition."""
    phi0 = np.asarray(phi0)
    shape = prm.shape
    phi0 = phi0.reshape(shape)
    mu0 = (np.asarray(muA0).reshape(shape), np.asarray(muB0).reshape(shape)) + tuple(
        np.asarray(m).reshape(shape) for m in mu_x0)
    if len(mu0) != prm.ncomp:
        raise ValueError(f"{prm.ncomp} compositions need {prm.ncomp} initial potentials")
    if c0 is None:
        c = model.closure_c(mu0, phi0, prm.c_eq, prm.kappa)
    else:
        c = tuple(np.asarray(ci).reshape(shape) for ci in c0)
    S0 = model.source_phi(phi0, mu0, prm)
    zero = np.zeros_like(phi0 * S0)
    u0 = [zero, zero, zero]
    slat = prm.slat
    g = np.stack([g_equilibrium_k(slat, k, phi0, u0, slat.w[k] * S0) for k in range(slat.Q)])
    hs = [np.stack([h_equilibrium_k(slat, k, c[a], mu0[a], u0) + zero for k in range(slat.Q)])
          for a in range(prm.ncomp)]
    hA, hB = hs[0], hs[1]
    if phi_ref is None:  # buoyancy reference of the initial force (given for a window of a larger box)
        phi_ref = phi0.mean() if prm.gravity_mean_subtract else 0.0
    f = None
    if prm.fluid:
        flat = prm.flat
        F0 = force(phi0, prm, phi_ref)
        if not prm.variable_density:
            f = np.stack([f_equilibrium_k(flat, k, zero, u0, prm.rho0, forcing_k(flat, k, u0, F0))
                          for k in range(flat.Q)])
        else:  # dimensionless populations; at rest with p* = 0 the pressure and viscous forces vanish
            scale = 1.0 / (density(phi0, prm) * flat.cs2)
            f = np.stack([f_equilibrium_k(flat, k, zero, u0, 1.0 / flat.cs2, forcing_k(flat, k, u0, F0) * scale)
                          for k in range(flat.Q)])
    return State(g=g, hA=hA, hB=hB, f=f, phi_ref=phi_ref, step=0, hx=tuple(hs[2:]))


def step(st, prm):
    """One time step P^n -> P^(n+1) (see the module docstring for the order)."""
    slat = prm.slat
    m = scalar_moments(st, prm)
    phi, S = m["phi"], m["S"]
    zero = np.zeros_like(phi)
    if prm.fluid:
        flat = prm.flat
        p_h, u, F, Fk = _flow(st.f, phi, prm, st.phi_ref)
        # pressure variable and inertia of the equilibrium (Eq. Feq, or its dimensionless form)
        p_eq, rho_eq = (p_h, prm.rho0) if not prm.variable_density else (st.f.sum(axis=0), 1.0 / flat.cs2)
    else:
        u = [zero, zero, zero]

    trt = prm.collision == "TRT"
    mrt = prm.collision == "MRT"
    lam_f, lam_s = prm.trt_magic

    # g: Eqs. LBE_Phi, Geq, Source_LBE_Phi
    wg = rate(prm.M_phi, slat.cs2)
    if mrt:
        Gk = [slat.w[k] * S for k in range(slat.Q)]
        g_post = mrt_collide(st.g, [g_equilibrium_k(slat, k, phi, u, Gk[k]) for k in range(slat.Q)], Gk, slat,
                             mrt_rates(slat, wg, prm.mrt_rates[1], False))
    elif not trt:
        g_post = np.stack([st.g[k] - wg * (st.g[k] - g_equilibrium_k(slat, k, phi, u, slat.w[k] * S))
                           + slat.w[k] * S for k in range(slat.Q)])
    else:  # the diffusive flux is the antisymmetric part: M_phi sets w-
        Gk = [slat.w[k] * S for k in range(slat.Q)]
        g_post = trt_collide(st.g, [g_equilibrium_k(slat, k, phi, u, Gk[k]) for k in range(slat.Q)], Gk, slat,
                             trt_partner_rate(wg, lam_s), wg)

    # h^alpha: Eqs. LBE_c_alpha, Heq with the phase-dependent mobility
    h_post = []
    fields = [(st.hA, m["cA"], m["muA"], prm.M_A), (st.hB, m["cB"], m["muB"], prm.M_B)]
    for a, (h, Mpair) in enumerate(zip(st.hx, prm.M_x)):
        name = COMP_NAMES[2 + a]
        fields.append((h, m["c" + name], m["mu" + name], Mpair))
    for h, c, mu, Mpair in fields:
        wh = rate(model.mobility(phi, Mpair), slat.cs2)
        if mrt:
            h_post.append(mrt_collide(h, [h_equilibrium_k(slat, k, c, mu, u) for k in range(slat.Q)],
                                      [0.0] * slat.Q, slat, mrt_rates(slat, wh, prm.mrt_rates[1], False)))
        elif not trt:
            h_post.append(np.stack([h[k] - wh * (h[k] - h_equilibrium_k(slat, k, c, mu, u))
                                    for k in range(slat.Q)]))
        else:
            h_post.append(trt_collide(h, [h_equilibrium_k(slat, k, c, mu, u) for k in range(slat.Q)],
                                      [0.0] * slat.Q, slat, trt_partner_rate(wh, lam_s), wh))

    f_new = None
    if prm.fluid:
        # f: Eqs. LBE_FluidFlow, ForcingTerm, GammaFunction, Feq
        wf = rate(model.viscosity(phi, prm.nu), flat.cs2)
        if mrt:
            f_post = mrt_collide(st.f, [f_equilibrium_k(flat, k, p_eq, u, rho_eq, Fk[k]) for k in range(flat.Q)],
                                 Fk, flat, mrt_rates(flat, wf, prm.mrt_rates[0], True))
        elif not trt:
            f_post = np.stack([st.f[k] - wf * (st.f[k] - f_equilibrium_k(flat, k, p_eq, u, rho_eq, Fk[k]))
                               + Fk[k] for k in range(flat.Q)])
        else:  # the viscous stress is the symmetric part: nu sets w+
            f_post = trt_collide(st.f, [f_equilibrium_k(flat, k, p_eq, u, rho_eq, Fk[k]) for k in range(flat.Q)],
                                 Fk, flat, wf, trt_partner_rate(wf, lam_f))
        f_new = stream(f_post, flat, prm.bc)

    phi_ref = phi.mean() if prm.gravity_mean_subtract else st.phi_ref
    return State(g=stream(g_post, slat, prm.bc), hA=stream(h_post[0], slat, prm.bc),
                 hB=stream(h_post[1], slat, prm.bc), f=f_new, phi_ref=phi_ref, step=st.step + 1,
                 hx=tuple(stream(h, slat, prm.bc) for h in h_post[2:]))


def run(st, prm, nsteps):
    for _ in range(nsteps):
        st = step(st, prm)
    return st


# ----------------------------------------------------------------------------------------
# diagnostics

DIAG_NAMES = ("sum_cA", "sum_cB", "sum_phi", "kinetic_energy", "max_u",
              "interface_measure", "free_energy", "nan_count", "droplets", "mean_radius")


def diagnostics(st, prm):
    """Global reductions of the current state:
    sums of c^A, c^B and phi; kinetic energy sum rho |u|^2 / 2 (rho0, or rho(phi) with
    variable density); max |u|;
    interface measure sum (4/W) phi (1 - phi) (the integrand of Eq. Rmoy_2D);
    free energy sum [W^2/2 |grad phi|^2 + omega_dw(phi) + lambda/2 (mu_A^2 + mu_B^2)],
    which is the functional of Eq. functional in units of H after the Legendre
    transform with the parabolic wells (bulk free energy density = |mu|^2 / 2 in
    units of K, lambda = K/H); gradient on the dimension's fluid lattice;
    count of nodes whose phi, c^A or c^B is not finite; droplet count N and mean
    radius <R> of Section 4.2.2 (geometry module, on the real part of phi)."""
    m = moments(st, prm)
    phi = m["phi"]
    u2 = m["ux"] ** 2 + m["uy"] ** 2 + m["uz"] ** 2
    grad = gradient(phi, prm.bc, prm.stencil_lattice)
    g2 = grad[0] ** 2 + grad[1] ** 2 + grad[2] ** 2
    names = COMP_NAMES[:prm.ncomp]
    fe = 0.5 * prm.W ** 2 * g2 + model.omega_dw(phi) + prm.lam * model.bulk_free_energy(
        tuple(m["mu" + a] for a in names), phi, prm.kappa)
    bad = ~np.isfinite(phi)
    for a in names:
        bad |= ~np.isfinite(m["c" + a])
    n_drops = geometry.euler_characteristic(phi.real, prm.bc)
    extra = {"sum_c" + a: m["c" + a].sum() for a in names[2:]}
    return dict(sum_cA=m["cA"].sum(), sum_cB=m["cB"].sum(), sum_phi=phi.sum(), **extra,
                kinetic_energy=(0.5 * (density(phi, prm) if prm.variable_density else prm.rho0) * u2).sum(),
                max_u=np.sqrt(u2.real).max(),
                interface_measure=((4.0 / prm.W) * phi * (1.0 - phi)).sum(),
                free_energy=fe.sum(), nan_count=int(bad.sum()),
                droplets=n_drops, mean_radius=geometry.mean_radius(phi.real, prm.W, n_drops))

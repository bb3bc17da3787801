"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: values printed in
the paper (tests/golden/paper_printed_values.json), moment identities the paper states
for its equilibria, exact conservation laws of the discrete map, closed-form solutions
(diffusion, tanh interface, curvature-driven shrinkage, diffusion couple, Poiseuille,
Laplace), and exact rational arithmetic for the lattice tables.
"""

import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import analytic, lattices, lbm, model

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_printed_values.json")))

ALL_LATTICES = [lattices.D2Q5, lattices.D2Q9, lattices.D3Q7, lattices.D3Q19]


# ----------------------------------------------------------------------------------------
# lattice tables (exact rational arithmetic)

@pytest.mark.parametrize("lat", ALL_LATTICES, ids=lambda l: l.name)
def test_lattice_moments_exact(lat):
    w, e = lat.w_exact, lat.e
    assert sum(w) == 1
    for a in range(3):
        assert sum(wk * int(ek[a]) for wk, ek in zip(w, e)) == 0
    cs2 = {"D2Q5": Fr(1, 3), "D2Q9": Fr(1, 3), "D3Q7": Fr(1, 4), "D3Q19": Fr(1, 3)}[lat.name]
    assert lat.cs2_exact == cs2
    for a in range(lat.dim):
        for b in range(lat.dim):
            m2 = sum(wk * int(ek[a]) * int(ek[b]) for wk, ek in zip(w, e))
            assert m2 == (cs2 if a == b else 0)
            for c in range(lat.dim):
                assert sum(wk * int(ek[a]) * int(ek[b]) * int(ek[c]) for wk, ek in zip(w, e)) == 0
    for k in range(lat.Q):
        assert (lat.e[lat.opp[k]] == -lat.e[k]).all()
        assert lat.w_exact[lat.opp[k]] == lat.w_exact[k]


@pytest.mark.parametrize("lat", [lattices.D2Q9, lattices.D3Q19], ids=lambda l: l.name)
def test_fluid_lattice_fourth_moment_isotropic(lat):
    """D2Q9 / D3Q19 carry the isotropic fourth moment c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    that the He-Luo equilibrium (Eq. Feq) relies on."""
    w, e = lat.w_exact, lat.e
    cs4 = Fr(1, 9)
    D = range(lat.dim)
    for a in D:
        for b in D:
            for c in D:
                for d in D:
                    m4 = sum(wk * int(ek[a]) * int(ek[b]) * int(ek[c]) * int(ek[d]) for wk, ek in zip(w, e))
                    iso = cs4 * ((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c))
                    assert m4 == iso


def test_paper_table_orderings():
    """Tables tab:D2Q9 and tab:D3Q19: first vectors and weights in the printed order."""
    assert [tuple(v[:2]) for v in lattices.D2Q9.e[:5]] == [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)]
    assert tuple(lattices.D2Q9.e[6][:2]) == (-1, 1)
    assert lattices.D2Q9.w_exact[0] == Fr(4, 9) and lattices.D2Q9.w_exact[5] == Fr(1, 36)
    assert tuple(lattices.D3Q19.e[9]) == (1, 0, 1) and tuple(lattices.D3Q19.e[18]) == (0, -1, 1)
    assert lattices.D3Q19.w_exact[6] == Fr(1, 18) and lattices.D3Q19.w_exact[7] == Fr(1, 36)


# ----------------------------------------------------------------------------------------
# thermodynamics

def test_interpolation_and_double_well_properties():
    """p(0)=0, p(1)=1, p'(0)=p'(1)=0 (Section 2.2); p(1 - phi) = 1 - p(phi)."""
    phi = np.linspace(-0.3, 1.3, 33)
    assert model.p(0.0) == 0.0 and model.p(1.0) == 1.0
    assert model.dp(0.0) == 0.0 and model.dp(1.0) == 0.0
    np.testing.assert_allclose(model.p(1.0 - phi), 1.0 - model.p(phi), atol=1e-14)
    h = 1e-6
    np.testing.assert_allclose((model.p(phi + h) - model.p(phi - h)) / (2 * h), model.dp(phi), atol=1e-8)
    np.testing.assert_allclose((model.omega_dw(phi + h) - model.omega_dw(phi - h)) / (2 * h),
                               model.domega_dw(phi), atol=1e-7)


def test_tanh_profile_is_equilibrium_and_surface_tension():
    """Eq. tanh solves W^2 phi'' = omega_dw'(phi); the excess grand potential of the
    profile, int [W^2/2 phi'^2 + omega_dw] dx in units of H, is sigma/H = 2W/3."""
    W = 3.7
    x = np.linspace(-12 * W, 12 * W, 200001)
    dx = x[1] - x[0]
    phi = analytic.tanh_profile(x, W)
    d1 = np.gradient(phi, dx)
    d2 = np.gradient(d1, dx)
    inner = slice(100, -100)
    np.testing.assert_allclose(W ** 2 * d2[inner], model.domega_dw(phi)[inner], atol=1e-6)
    excess = np.trapezoid(0.5 * W ** 2 * d1 ** 2 + model.omega_dw(phi), x)
    assert abs(excess - 2.0 * W / 3.0) < 1e-6


def test_lambda_star_printed():
    dcp = GOLD["diffusion_couple"]
    c_eq = (tuple(dcp["c_eq_phase0"]), tuple(dcp["c_eq_phase1"]))
    lam = model.lambda_star(1.0, dcp["M_phi"], dcp["M_alpha"], c_eq)
    assert abs(lam - dcp["lambda_star"]) < 5e-9
    # the value does not depend on W (beta and delta both scale with W)
    assert abs(model.lambda_star(7.0, dcp["M_phi"], dcp["M_alpha"], c_eq) - lam) < 1e-12


def test_far_field_potentials_printed():
    """Caption of tab:Parameters_Diffusion-Couple: the far-field compositions are
    equivalent to the printed potentials (phase 0 on the left, phase 1 on the right)."""
    dcp = GOLD["diffusion_couple"]
    c_eq = (tuple(dcp["c_eq_phase0"]), tuple(dcp["c_eq_phase1"]))
    mu_l = model.closure_mu(tuple(dcp["c_minus_inf"]), 0.0, c_eq)
    mu_r = model.closure_mu(tuple(dcp["c_plus_inf"]), 1.0, c_eq)
    np.testing.assert_allclose(mu_l, dcp["mu_minus_inf"], atol=1e-15)
    np.testing.assert_allclose(mu_r, dcp["mu_plus_inf"], atol=1e-15)
    # the forward closure inverts the backward one at any phi
    for phi in (0.0, 0.3, 0.5, 1.0):
        mu = model.closure_mu((0.31, 0.27), phi, c_eq)
        np.testing.assert_allclose(model.closure_c(mu, phi, c_eq), (0.31, 0.27), atol=1e-15)


def test_delta_omega_closed_form_and_coexistence():
    """Delta omega = -sum mu (c_0 - c_1) (Section 2.2); it vanishes on the coexistence
    line, and c = -d omega / d mu gives back the closure compositions (Eq. species_closure)."""
    c_eq = ((0.3, 0.3), (0.4, 0.4))
    rng = np.random.default_rng(1)
    mu = rng.normal(size=(2, 10))
    d = model.delta_omega(mu, c_eq)
    np.testing.assert_allclose(d, -(mu[0] * (0.3 - 0.4) + mu[1] * (0.3 - 0.4)), atol=1e-15)
    assert abs(model.delta_omega((0.05, -0.05), c_eq)) < 1e-16
    h = 1e-6
    for pi in range(2):
        for a in range(2):
            mp = [mu[0].copy(), mu[1].copy()]
            mm = [mu[0].copy(), mu[1].copy()]
            mp[a] += h
            mm[a] -= h
            dw = (model.grand_potential(mp, c_eq[pi]) - model.grand_potential(mm, c_eq[pi])) / (2 * h)
            np.testing.assert_allclose(-dw, mu[a] + c_eq[pi][a], atol=1e-8)


def test_ostwald_collision_rates_printed():
    """Caption of tab:Parameters_Ostwald-Ripening: the listed rates are tau + 1/2 of a
    D2Q9 lattice with D = tau c_s^2 dt/dx^2 - this pins the oracle's rate convention.
    The printed figures are the values cut after four decimals (0.81468 -> 0.8146)."""
    o = GOLD["ostwald_2d"]
    s = o["dt"] / o["dx"] ** 2
    cs2 = lattices.D2Q9.cs2
    for D, printed in ((o["M_phi"], o["tau_g"]), (o["M_alpha"][0], o["tau_hA"]), (o["M_alpha"][1], o["tau_hB"])):
        assert 0.0 <= 1.0 / lbm.rate(D * s, cs2) - printed < 1e-4


# ----------------------------------------------------------------------------------------
# equilibrium moments stated in Section 3

@pytest.mark.parametrize("slat,flat", [(lattices.D2Q5, lattices.D2Q9), (lattices.D3Q7, lattices.D3Q19),
                                       (lattices.D2Q9, lattices.D2Q9), (lattices.D3Q19, lattices.D3Q19)],
                         ids=["2D", "3D", "2D-paper-scalars", "3D-paper-scalars"])
def test_equilibrium_moments(slat, flat):
    rng = np.random.default_rng(7)
    n = 17
    phi, c, mu, p_h, S = (rng.uniform(-1, 1, n) for _ in range(5))
    u = [rng.uniform(-0.1, 0.1, n) for _ in range(3)]
    F = [rng.uniform(-0.01, 0.01, n) for _ in range(3)]
    if slat.dim == 2:
        u[2] = np.zeros(n)
        F[2] = np.zeros(n)
    rho0 = 1.3
    heq = [lbm.h_equilibrium_k(slat, k, c, mu, u) for k in range(slat.Q)]
    Gk = [slat.w[k] * S for k in range(slat.Q)]
    geq = [lbm.g_equilibrium_k(slat, k, phi, u, Gk[k]) for k in range(slat.Q)]
    Fk = [lbm.forcing_k(flat, k, u, F) for k in range(flat.Q)]
    feq = [lbm.f_equilibrium_k(flat, k, p_h, u, rho0, Fk[k]) for k in range(flat.Q)]
    tol = dict(atol=1e-14, rtol=0)
    # Eq. Heq: zeroth moment c, first moment c u, second moment c_s^2 mu I
    np.testing.assert_allclose(sum(heq), c, **tol)
    for a in range(slat.dim):
        np.testing.assert_allclose(sum(heq[k] * slat.e[k][a] for k in range(slat.Q)), c * u[a], **tol)
        for b in range(slat.dim):
            m2 = sum(heq[k] * slat.e[k][a] * slat.e[k][b] for k in range(slat.Q))
            np.testing.assert_allclose(m2, slat.cs2 * mu * (a == b), **tol)
    # Eqs. Geq, Source_LBE_Phi: sum G = S, sum g^eq = phi - S/2, first moment phi u
    np.testing.assert_allclose(sum(Gk), S, **tol)
    np.testing.assert_allclose(sum(geq), phi - 0.5 * S, **tol)
    for a in range(slat.dim):
        np.testing.assert_allclose(sum(geq[k] * slat.e[k][a] for k in range(slat.Q)), phi * u[a], **tol)
    # Eq. ForcingTerm: sum F_k = 0, sum F_k c_k = c_s^2 F (the form Eq. Velocity needs)
    np.testing.assert_allclose(sum(Fk), 0.0, **tol)
    for a in range(flat.dim):
        np.testing.assert_allclose(sum(Fk[k] * flat.e[k][a] for k in range(flat.Q)), flat.cs2 * F[a], **tol)
    # Eq. Feq: sum f^eq = p_h; (1/c_s^2) sum f^eq c_k + F/2 = rho0 u (Eq. Velocity)
    np.testing.assert_allclose(sum(feq), p_h, **tol)
    for a in range(flat.dim):
        m1 = sum(feq[k] * flat.e[k][a] for k in range(flat.Q))
        np.testing.assert_allclose(m1 / flat.cs2 + 0.5 * F[a], rho0 * u[a], **tol)


# ----------------------------------------------------------------------------------------
# exact conservation of the discrete map

def _droplet_fields(shape, centres, radii, W, rng, noise=1e-3):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = np.zeros(shape)
    for c, R in zip(centres, radii):
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        phi = np.maximum(phi, analytic.tanh_profile(R - r, W))
    mu = rng.normal(0.0, noise, (2,) + shape)
    return phi, mu[0], mu[1]


@pytest.mark.parametrize("case", ["2d_noflow_walls", "2d_flow_walls", "3d_flow_walls", "3d_flow_periodic_g",
                                  "2d_paper_scalars_flow_walls", "3d_paper_scalars_flow_walls"])
def test_mass_conservation_exact(case):
    rng = np.random.default_rng(3)
    if case == "2d_noflow_walls":
        prm = lbm.Params(nx=40, ny=24, bc=("walls", "periodic", "periodic"), W=3.0, lam=21.05)
        fields = _droplet_fields(prm.shape, [(10, 12, 0), (28, 8, 0)], [6, 5], 3.0, rng)
        nsteps = 150
    elif case == "2d_flow_walls":
        prm = lbm.Params(nx=32, ny=28, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05,
                         drho=0.5, g=(0, -1e-4, 0), sigma=1e-3, nu=(0.1, 0.05))
        fields = _droplet_fields(prm.shape, [(16, 14, 0)], [7], 4.0, rng)
        nsteps = 100
    elif case == "3d_flow_walls":
        prm = lbm.Params(nx=14, ny=12, nz=16, fluid="D3Q19", scalar="D3Q7", bc=("periodic", "periodic", "walls"),
                         W=4.0, lam=21.05, drho=0.5, g=(0, 0, -1e-4), sigma=1e-3, nu=(0.1, 0.05))
        fields = _droplet_fields(prm.shape, [(7, 6, 8)], [4.5], 4.0, rng)
        nsteps = 30
    elif case == "2d_paper_scalars_flow_walls":
        prm = lbm.Params(nx=30, ny=26, fluid="D2Q9", scalar="D2Q9", bc=("walls", "walls", "periodic"), W=4.0,
                         lam=21.05, drho=0.5, g=(0, -1e-4, 0), sigma=1e-3, nu=(0.1, 0.05))
        fields = _droplet_fields(prm.shape, [(15, 13, 0)], [6], 4.0, rng)
        nsteps = 80
    elif case == "3d_paper_scalars_flow_walls":
        prm = lbm.Params(nx=12, ny=10, nz=14, fluid="D3Q19", scalar="D3Q19", bc=("periodic", "walls", "walls"),
                         W=4.0, lam=21.05, drho=0.5, g=(0, 0, -1e-4), sigma=1e-3, nu=(0.1, 0.05))
        fields = _droplet_fields(prm.shape, [(6, 5, 7)], [4.0], 4.0, rng)
        nsteps = 20
    else:
        prm = lbm.Params(nx=12, ny=12, nz=12, fluid="D3Q19", scalar="D3Q7", W=4.0, lam=21.05,
                         drho=0.5, g=(0, 0, -1e-4), sigma=1e-3, nu=(0.1, 0.05), gravity_mean_subtract=True)
        fields = _droplet_fields(prm.shape, [(6, 6, 6)], [4.0], 4.0, rng)
        nsteps = 30
    st = lbm.init(*fields, prm)
    d0 = lbm.diagnostics(st, prm)
    p0 = st.f.sum() if st.f is not None else 0.0
    st = lbm.run(st, prm, nsteps)
    d1 = lbm.diagnostics(st, prm)
    for key in ("sum_cA", "sum_cB"):
        assert abs(d1[key] - d0[key]) <= 1e-12 * abs(d0[key]), key
    if st.f is not None:
        # sum_k F_k = 0 and sum_k f^eq_k = p_h make sum_x p_h invariant as well
        assert abs(st.f.sum() - p0) <= 1e-12 * max(1.0, abs(d0["sum_phi"]))
    assert d1["nan_count"] == 0


def test_momentum_balance_periodic():
    """Fully periodic flow: total momentum changes by exactly the total force each step
    (sum_k F_k c_k = c_s^2 F and the half-force shift of Eq. Velocity)."""
    rng = np.random.default_rng(5)
    prm = lbm.Params(nx=20, ny=18, fluid="D2Q9", W=4.0, lam=21.05, drho=0.5, g=(2e-4, -1e-4, 0),
                     sigma=1e-3, nu=(0.1, 0.05))
    st = lbm.init(*_droplet_fields(prm.shape, [(10, 9, 0)], [5], 4.0, rng), prm)
    for _ in range(5):
        m = lbm.moments(st, prm)
        mom_a = [(prm.rho0 * m[u]).sum() - 0.5 * m["F"][a].sum() for a, u in enumerate(("ux", "uy"))]
        st2 = lbm.step(st, prm)
        m2 = lbm.moments(st2, prm)
        mom_b = [(prm.rho0 * m2[u]).sum() - 0.5 * m2["F"][a].sum() for a, u in enumerate(("ux", "uy"))]
        for a in range(2):
            assert abs(mom_b[a] - mom_a[a] - m["F"][a].sum()) < 1e-15 * prm.nx * prm.ny + 1e-14
        st = st2


# ----------------------------------------------------------------------------------------
# diffusion of the composition lattice: Fourier-mode decay against exp(-M k^2 t)

@pytest.mark.parametrize("scalar,axis", [("D2Q5", 0), ("D2Q5", 1), ("D3Q7", 2), ("D2Q9", 0), ("D2Q9", 1),
                                         ("D3Q19", 2)])
def test_fourier_mode_diffusivity(scalar, axis):
    """phi = 0 everywhere stays 0 (omega_dw'(0) = p'(0) = 0), so c^A obeys
    dc/dt = M lap mu with mu = c - c_0 (Eq. Compos, bulk phase 0).  A sine mode decays
    as exp(-M k^2 t) up to O(k^4); the measured rate must approach M k^2 with an error
    that falls like k^2."""
    errs = []
    for N in (16, 32):
        shape = [1, 1, 1] if scalar == "D3Q7" else [1, 1, 1]
        shape[2 - axis] = N
        nz, ny, nx = shape
        M = 0.15
        prm = lbm.Params(nx=nx, ny=ny, nz=nz, scalar=scalar, W=4.0, lam=10.0, M_phi=0.1,
                         M_A=(M, M), M_B=(M, M), c_eq=((0.2, 0.1), (0.6, 0.3)))
        coord = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")[2 - axis]
        kw = 2 * math.pi / N
        eps = 1e-3
        mu0 = eps * np.sin(kw * coord)
        st = lbm.init(np.zeros(prm.shape), mu0, 0 * mu0, prm)
        t0, t1 = 40, 40 + int(2.0 / (M * kw * kw))
        st = lbm.run(st, prm, t0)
        a0 = (lbm.moments(st, prm)["muA"] * np.sin(kw * coord)).sum()
        st = lbm.run(st, prm, t1 - t0)
        m = lbm.moments(st, prm)
        assert np.abs(m["phi"]).max() == 0.0
        a1 = (m["muA"] * np.sin(kw * coord)).sum()
        rate_meas = -math.log(a1 / a0) / (t1 - t0)
        errs.append(abs(rate_meas / (M * kw * kw) - 1.0))
    assert errs[1] < 0.02
    assert errs[0] / errs[1] > 3.0   # O(k^2) relative error


@pytest.mark.parametrize("scalar", ["D2Q5", "D3Q7", "D2Q9"])
@pytest.mark.parametrize("phase", [0, 1])
def test_fourier_mode_per_phase_mobility(scalar, phase):
    """The species mobility depends on the phase (Section 2.3): M(phi) = M_0 (1 - phi)
    + M_1 phi.  In bulk phase pi (phi = pi everywhere: omega_dw'(pi) = p'(pi) = 0, so
    S = 0 and phi stays pi up to the rounding of sum_k w_k) c = mu + c_pi,eq and a Fourier mode of each component
    decays at M_pi k^2.  Unequal mobilities per phase and per component tell the phases
    and the components apart: with them exchanged the rates would be off by 4x."""
    N = 32
    shape = [1, 1, 1]
    axis = 2 if scalar == "D3Q7" else 0
    shape[2 - axis] = N
    nz, ny, nx = shape
    M_A, M_B = (0.05, 0.2), (0.2, 0.05)
    prm = lbm.Params(nx=nx, ny=ny, nz=nz, scalar=scalar, W=4.0, lam=10.0, M_phi=0.1,
                     M_A=M_A, M_B=M_B, c_eq=((0.2, 0.1), (0.6, 0.3)))
    coord = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")[2 - axis]
    kw = 2 * math.pi / N
    mode = np.sin(kw * coord)
    st = lbm.init(np.full(prm.shape, float(phase)), 1e-3 * mode, -2e-3 * mode, prm)
    t0 = 40
    t1 = t0 + int(1.5 / (min(M_A[phase], M_B[phase]) * kw * kw))
    st = lbm.run(st, prm, t0)
    m0 = lbm.moments(st, prm)
    st = lbm.run(st, prm, t1 - t0)
    m1 = lbm.moments(st, prm)
    assert np.abs(m1["phi"] - float(phase)).max() < 1e-12
    for key, M in (("muA", M_A), ("muB", M_B)):
        a0, a1 = (m0[key] * mode).sum(), (m1[key] * mode).sum()
        rate_meas = -math.log(a1 / a0) / (t1 - t0)
        assert abs(rate_meas / (M[phase] * kw * kw) - 1.0) < 0.02, (key, rate_meas / (M[phase] * kw * kw))


@pytest.mark.parametrize("scalar", ["D2Q5", "D2Q9", "D3Q7", "D3Q19"])
def test_fourier_mode_diagonal(scalar):
    """Isotropy of the composition lattice: a mode along a lattice diagonal decays at
    M |k|^2 as well (to O(k^2) relative error)."""
    N = 24
    three = scalar in ("D3Q7", "D3Q19")
    nz, ny, nx = (1, N, N) if not three else (N, N, 1)
    M = 0.15
    prm = lbm.Params(nx=nx, ny=ny, nz=nz, scalar=scalar, W=4.0, lam=10.0, M_phi=0.1,
                     M_A=(M, M), M_B=(M, M), c_eq=((0.2, 0.1), (0.6, 0.3)))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kw = 2 * math.pi / N
    arg = kw * (y + z) if three else kw * (x + y)
    mu0 = 1e-3 * np.sin(arg)
    st = lbm.run(lbm.init(np.zeros(prm.shape), mu0, 0 * mu0, prm), prm, 30)
    a0 = (lbm.moments(st, prm)["muA"] * np.sin(arg)).sum()
    T = int(1.0 / (M * 2 * kw * kw))
    st = lbm.run(st, prm, T)
    a1 = (lbm.moments(st, prm)["muA"] * np.sin(arg)).sum()
    rate = -math.log(a1 / a0) / T
    assert abs(rate / (M * 2 * kw * kw) - 1.0) < 0.03


def test_init_given_compositions():
    """The paper's initial condition gives c and mu separately.  With c equal to the
    closure the populations equal those of the ordinary initialisation; with mu = 0
    the h populations are c at rest (h_0 = c, h_k = 0) and g does not depend on c."""
    rng = np.random.default_rng(21)
    prm = lbm.Params(nx=18, ny=14, fluid="D2Q9", scalar="D2Q9", W=3.0, lam=21.05, drho=0.5,
                     g=(0, -1e-4, 0), sigma=1e-3, nu=(0.1, 0.05))
    phi, muA, muB = _droplet_fields(prm.shape, [(9, 7, 0)], [4.0], 3.0, rng)
    a = lbm.init(phi, muA, muB, prm)
    c = model.closure_c((muA, muB), phi, prm.c_eq)
    b = lbm.init(phi, muA, muB, prm, c0=c)
    for k in ("g", "hA", "hB", "f"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    cA = np.where(phi >= 0.5, 0.6, 0.21)
    cB = np.where(phi >= 0.5, 0.3, 0.11)
    z = np.zeros_like(phi)
    st = lbm.init(phi, z, z, prm, c0=(cA, cB))
    assert np.array_equal(st.hA[0], cA) and np.array_equal(st.hB[0], cB)
    assert np.abs(st.hA[1:]).max() == 0.0 and np.abs(st.hB[1:]).max() == 0.0
    assert np.array_equal(st.g, lbm.init(phi, z, z, prm).g)


# ----------------------------------------------------------------------------------------
# Allen-Cahn dynamics of the g lattice (Delta omega = 0 by equal phase compositions)

@pytest.mark.slow
def test_flat_tanh_interface_is_stationary():
    errs = []
    for W in (4.0, 8.0):
        N = int(16 * W)
        prm = lbm.Params(nx=N, ny=1, bc=("walls", "periodic", "periodic"), W=W, lam=21.05, M_phi=0.1,
                         c_eq=((0.3, 0.3), (0.3, 0.3)))
        x = np.arange(N) - (N - 1) / 2.0
        phi0 = analytic.tanh_profile(x, W).reshape(prm.shape)
        st = lbm.run(lbm.init(phi0, 0 * phi0, 0 * phi0, prm), prm, int(4 * W * W / prm.M_phi))
        phi = lbm.moments(st, prm)["phi"].ravel()
        errs.append(np.abs(phi - analytic.tanh_profile(x, W)).max())
    assert errs[0] < 2e-2
    assert errs[0] / errs[1] > 3.0   # O(W^-2)


@pytest.mark.slow
def test_disk_shrinks_by_curvature():
    """Delta omega = 0: V = -M_phi kappa, so R^2 = R0^2 - 2 M_phi t in 2D."""
    N, W, R0, Mphi = 96, 4.0, 30.0, 0.1
    prm = lbm.Params(nx=N, ny=N, W=W, lam=21.05, M_phi=Mphi, c_eq=((0.3, 0.3), (0.3, 0.3)))
    z, y, x = np.meshgrid(np.arange(1), np.arange(N), np.arange(N), indexing="ij")
    r = np.sqrt((x - N / 2 + 0.5) ** 2 + (y - N / 2 + 0.5) ** 2)
    phi0 = analytic.tanh_profile(R0 - r, W)
    st = lbm.init(phi0, 0 * phi0, 0 * phi0, prm)
    st = lbm.run(st, prm, 200)
    r2a = lbm.moments(st, prm)["phi"].sum() / math.pi
    T = 1500
    st = lbm.run(st, prm, T)
    r2b = lbm.moments(st, prm)["phi"].sum() / math.pi
    slope = (r2b - r2a) / T
    assert abs(slope / (-2.0 * Mphi) - 1.0) < 0.05


# ----------------------------------------------------------------------------------------
# ternary diffusion couple (Section 4.1)

def test_diffusion_couple_printed_parameters_root():
    """With the printed table the similarity equation has the single root xi = 0 in
    [-4, 4] and mu_int = (mu_-inf + mu_+inf)/2 (the printed xi = -0.269824 does not
    follow from the printed parameters)."""
    dcp = GOLD["diffusion_couple"]
    dc = [a - b for a, b in zip(dcp["c_eq_phase0"], dcp["c_eq_phase1"])]
    roots = analytic.dc_roots(dcp["mu_minus_inf"], dcp["mu_plus_inf"], dc, dcp["M_alpha"])
    assert len(roots) == 1 and abs(roots[0]) < 1e-12
    for a in range(2):
        mi = analytic.dc_interface_mu(roots[0], dcp["mu_minus_inf"][a], dcp["mu_plus_inf"][a], dc[a], dcp["M_alpha"][a])
        assert abs(mi - 0.5 * (dcp["mu_minus_inf"][a] + dcp["mu_plus_inf"][a])) < 1e-14


def _interface_position(phi, x):
    i = np.nonzero((phi[:-1] - 0.5) * (phi[1:] - 0.5) <= 0)[0][0]
    return x[i] + (0.5 - phi[i]) / (phi[i + 1] - phi[i]) * (x[i + 1] - x[i])


def _run_couple(mu_l, mu_r, c_eq, M, Mphi, W, N, T, snaps):
    """M[alpha]: the mobility of component alpha, one number or the pair (phase 0,
    phase 1); lambda = lambda* of the phase-averaged mobilities."""
    dc = [c_eq[0][a] - c_eq[1][a] for a in range(2)]
    pairs = [(m, m) if np.ndim(m) == 0 else tuple(m) for m in M]
    lam = model.lambda_star(W, Mphi, [0.5 * (p[0] + p[1]) for p in pairs], c_eq)
    prm = lbm.Params(nx=N, ny=1, bc=("walls", "periodic", "periodic"), W=W, lam=lam, M_phi=Mphi,
                     M_A=pairs[0], M_B=pairs[1], c_eq=c_eq)
    x = np.arange(N) - (N - 1) / 2.0
    phi0 = analytic.tanh_profile(x, W)
    muA0 = np.where(x < 0, mu_l[0], mu_r[0])
    muB0 = np.where(x < 0, mu_l[1], mu_r[1])
    st = lbm.init(phi0.reshape(prm.shape), muA0.reshape(prm.shape), muB0.reshape(prm.shape), prm)
    out = {}
    t = 0
    for s in snaps:
        st = lbm.run(st, prm, s - t)
        t = s
        m = lbm.moments(st, prm)
        out[s] = dict(xI=_interface_position(m["phi"].ravel(), x), muA=m["muA"].ravel(), muB=m["muB"].ravel())
    return x, dc, out


@pytest.mark.slow
def test_diffusion_couple_printed_parameters_profiles():
    """Paper's couple in lattice units (mobilities x 0.1, W = 4): the interface stays at
    x = 0 and the potentials follow the erfc solution with mu_int = (-0.0375, 0.0375)."""
    dcp = GOLD["diffusion_couple"]
    c_eq = (tuple(dcp["c_eq_phase0"]), tuple(dcp["c_eq_phase1"]))
    M = [0.1 * m for m in dcp["M_alpha"]]
    T = 2000
    x, dc, out = _run_couple(dcp["mu_minus_inf"], dcp["mu_plus_inf"], c_eq, M, 0.12, 4.0, 512, T, [T])
    assert abs(out[T]["xI"]) < 0.05
    for a, key in enumerate(("muA", "muB")):
        ref = analytic.dc_mu_profile(x, T, 0.0, dcp["mu_minus_inf"][a], dcp["mu_plus_inf"][a], dc[a], M[a])
        assert np.abs(out[T][key] - ref).max() < 0.01 * abs(dcp["mu_plus_inf"][a] - dcp["mu_minus_inf"][a])


@pytest.mark.slow
def test_diffusion_couple_moving_interface():
    """A couple whose far fields are not symmetric about the coexistence line moves as
    x_I = xi sqrt(t) with xi from the similarity equation; the phase-field interface must
    follow it (pins the sign and size of the coupling lambda p' Delta omega, the closure
    and the interface mass balance together)."""
    c_eq = ((0.3, 0.3), (0.4, 0.4))
    M = [0.1, 0.08]
    mu_l, mu_r = (0.1, 0.05), (-0.02, 0.0)
    dc = [c_eq[0][a] - c_eq[1][a] for a in range(2)]
    roots = analytic.dc_roots(mu_l, mu_r, dc, M)
    assert len(roots) == 1
    xi = roots[0]
    assert xi < -0.4     # phase 1 grows to the left
    snaps = [1000, 4000]
    x, _, out = _run_couple(mu_l, mu_r, c_eq, M, 0.12, 4.0, 512, snaps[-1], snaps)
    # the velocity is checked through the displacement between two times, which cancels the
    # initial transient offset of the diffuse interface
    xi_meas = (out[snaps[1]]["xI"] - out[snaps[0]]["xI"]) / (math.sqrt(snaps[1]) - math.sqrt(snaps[0]))
    assert abs(xi_meas / xi - 1.0) < 0.05
    for a, key in enumerate(("muA", "muB")):
        ref = analytic.dc_mu_profile(x, snaps[1], xi, mu_l[a], mu_r[a], dc[a], M[a])
        far = np.abs(x - out[snaps[1]]["xI"]) > 3 * 4.0
        assert np.abs(out[snaps[1]][key] - ref)[far].max() < 0.05 * abs(mu_l[a] - mu_r[a])


@pytest.mark.slow
def test_diffusion_couple_per_phase_mobilities():
    """A moving couple with different mobilities in the two phases (Section 2.3):
    phase 0 (left) diffuses with M_0, phase 1 (right) with M_1, and the similarity
    solution of Eqs. Stefan ... Solution_Mu with per-side diffusivities fixes the
    interface velocity xi.  The measured xi must match it within 5%; with the phases'
    mobilities exchanged the same couple moves at xi = -0.229 instead of -0.580."""
    c_eq = ((0.3, 0.3), (0.4, 0.4))
    M_A, M_B = (0.1, 0.025), (0.08, 0.02)
    mu_l, mu_r = (0.1, 0.05), (-0.02, 0.0)
    dc = [c_eq[0][a] - c_eq[1][a] for a in range(2)]
    roots = analytic.dc_roots(mu_l, mu_r, dc, [M_A, M_B])
    assert len(roots) == 1
    xi = roots[0]
    swapped = analytic.dc_roots(mu_l, mu_r, dc, [M_A[::-1], M_B[::-1]])
    assert len(swapped) == 1 and abs(swapped[0] / xi - 1.0) > 0.5
    snaps = [1000, 4000]
    x, _, out = _run_couple(mu_l, mu_r, c_eq, (M_A, M_B), 0.12, 4.0, 512, snaps[-1], snaps)
    xi_meas = (out[snaps[1]]["xI"] - out[snaps[0]]["xI"]) / (math.sqrt(snaps[1]) - math.sqrt(snaps[0]))
    assert abs(xi_meas / xi - 1.0) < 0.05, (xi_meas, xi)


# ----------------------------------------------------------------------------------------
# the whole discrete map against exact rational arithmetic

def _exact_case(name):
    """Parameters (binary fractions, so both sides start from identical values) and step
    count.  Unequal mobilities and viscosities per phase, capillary force, buoyancy."""
    base = dict(W=4.0, lam=21.5, M_phi=0.125, M_A=(0.125, 0.0625), M_B=(0.09375, 0.15625),
                c_eq=((0.25, 0.125), (0.625, 0.3125)), rho0=1.0, drho=0.5, sigma=1.0 / 16, nu=(0.125, 0.0625))
    cases = {
        "2d_noflow_walls": dict(nx=3, ny=3, nz=1, fluid=None, scalar="D2Q5", bc=("walls", "periodic", "periodic")),
        "2d_flow_walls": dict(nx=3, ny=3, nz=1, fluid="D2Q9", scalar="D2Q5", bc=("periodic", "walls", "periodic"),
                              g=(0.0, -1.0 / 4096, 0.0)),
        "2d_paper_periodic_mean": dict(nx=3, ny=3, nz=1, fluid="D2Q9", scalar="D2Q9", bc=("periodic",) * 3,
                                       g=(1.0 / 8192, -1.0 / 4096, 0.0), gravity_mean_subtract=True),
        "3d_flow_walls": dict(nx=3, ny=3, nz=3, fluid="D3Q19", scalar="D3Q7", bc=("walls", "periodic", "walls"),
                              g=(0.0, 0.0, -1.0 / 4096)),
    }
    return dict(base, **cases[name])


@pytest.mark.parametrize("name", ["2d_noflow_walls", "2d_flow_walls", "2d_paper_periodic_mean", "3d_flow_walls"])
def test_whole_map_matches_exact_rational_arithmetic(name):
    """Every operation of the step (moments, closure with the predictor, source, stencil,
    force, flow moments, the three collisions with rational rates, streaming with walls) is
    +, -, x or /.  On random dyadic-rational populations the independent Fraction
    reference of tests/exact_map.py is exact; two oracle steps must match it to 1e-14 of
    each field's largest population (measured: <= 7e-16).  More steps are impractical: the
    exact denominators reach 2e4 bits after two steps and 5e5 bits after three."""
    import exact_map
    p = _exact_case(name)
    shape = (p["nz"], p["ny"], p["nx"])
    nodes = [(x, y, z) for z in range(shape[0]) for y in range(shape[1]) for x in range(shape[2])]
    rng = np.random.default_rng(5)

    def dyadic(lo, hi, den=4096):
        return Fr(int(rng.integers(int(lo * den), int(hi * den) + 1)), den)

    _, sw = exact_map.LATTICES[p["scalar"]]
    phi = {x: dyadic(0.05, 0.95) for x in nodes}
    cA = {x: dyadic(0.2, 0.6) for x in nodes}
    cB = {x: dyadic(0.1, 0.3) for x in nodes}
    st = {"phi_ref": dyadic(0.3, 0.7) if p.get("gravity_mean_subtract") else Fr(0)}
    st["g"] = [{x: sw[k] * phi[x] + dyadic(-0.01, 0.01) for x in nodes} for k in range(len(sw))]
    st["hA"] = [{x: (cA[x] if k == 0 else 0) + dyadic(-0.01, 0.01) for x in nodes} for k in range(len(sw))]
    st["hB"] = [{x: (cB[x] if k == 0 else 0) + dyadic(-0.01, 0.01) for x in nodes} for k in range(len(sw))]
    if p["fluid"]:
        _, fw = exact_map.LATTICES[p["fluid"]]
        st["f"] = [{x: fw[k] * dyadic(-0.01, 0.01) + dyadic(-0.001, 0.001) for x in nodes} for k in range(len(fw))]

    def arr(pops):
        a = np.zeros((len(pops),) + shape)
        for k, d in enumerate(pops):
            for (x, y, z), v in d.items():
                a[k, z, y, x] = float(v)
        return a

    exact_prm = {k: Fr(v) for k, v in p.items() if isinstance(v, float)}
    exact_prm.update(shape=shape, bc=p["bc"], scalar=p["scalar"], fluid=p["fluid"],
                     gravity_mean_subtract=p.get("gravity_mean_subtract", False),
                     M_A=tuple(map(Fr, p["M_A"])), M_B=tuple(map(Fr, p["M_B"])), nu=tuple(map(Fr, p["nu"])),
                     g=tuple(map(Fr, p.get("g", (0.0, 0.0, 0.0)))),
                     c_eq=tuple(tuple(map(Fr, r)) for r in p["c_eq"]))
    prm = lbm.Params(**p)
    ost = lbm.State(g=arr(st["g"]), hA=arr(st["hA"]), hB=arr(st["hB"]), f=arr(st["f"]) if p["fluid"] else None,
                    phi_ref=float(st["phi_ref"]))
    for _ in range(2):
        st = exact_map.step(st, exact_prm)
        ost = lbm.step(ost, prm)
        for key in ("g", "hA", "hB") + (("f",) if p["fluid"] else ()):
            ex = arr(st[key])
            assert np.abs(getattr(ost, key) - ex).max() <= 1e-14 * np.abs(ex).max(), key
        assert abs(ost.phi_ref - float(st["phi_ref"])) <= 1e-15


# ----------------------------------------------------------------------------------------
# N components: the conclusion's extension to more than three components, with the
# quadratic free energies of Eq. Taylor (unit curvatures) for every independent
# composition.  Three compositions A, B, C (a quaternary fluid) below.

C_EQ3 = ((0.2, 0.1, 0.15), (0.6, 0.3, 0.05))


def _ncomp_case(c_eq=C_EQ3, M_x=((0.08, 0.06),), nx=40, ny=30, seed=41):
    prm = lbm.Params(nx=nx, ny=ny, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=12.0,
                     M_phi=0.1, M_A=(0.1, 0.07), M_B=(0.05, 0.09), M_x=M_x, c_eq=c_eq, drho=0.5,
                     g=(0.0, -1e-4, 0.0), sigma=2e-3, nu=(0.1, 0.05))
    phi0 = _droplet_fields((1, ny, nx), [(20.0, 14.0, 0.0), (8.0, 22.0, 0.0)], [7.0, 4.5], 4.0,
                           np.random.default_rng(seed))[0]
    rng = np.random.default_rng(seed + 1)
    mu = [1e-3 * rng.standard_normal(prm.shape) for _ in range(prm.ncomp)]
    return prm, phi0, mu


def test_ncomp_absent_component_reproduces_ternary():
    """A fourth component that is absent (zero equilibrium compositions and zero initial
    potential) stays absent and leaves the ternary run unchanged."""
    prm3, phi0, mu = _ncomp_case(c_eq=((0.2, 0.1, 0.0), (0.6, 0.3, 0.0)))
    tern = prm3.with_(M_x=(), c_eq=((0.2, 0.1), (0.6, 0.3)))
    a = lbm.run(lbm.init(phi0, mu[0], mu[1], tern), tern, 60)
    b = lbm.run(lbm.init(phi0, mu[0], mu[1], prm3, mu_x0=(0 * mu[2],)), prm3, 60)
    assert np.all(b.hx[0] == 0.0)
    for key in ("g", "hA", "hB", "f"):
        assert np.abs(getattr(a, key) - getattr(b, key)).max() <= 1e-15 * np.abs(getattr(a, key)).max(), key


def test_ncomp_relabelling_permutes_the_run():
    """The model treats every composition alike: relabelling (A, B, C) -> (B, C, A) in the
    equilibrium compositions, mobilities and initial potentials relabels the run."""
    prm, phi0, mu = _ncomp_case()
    st = lbm.run(lbm.init(phi0, mu[0], mu[1], prm, mu_x0=(mu[2],)), prm, 60)
    perm = (1, 2, 0)
    mob = (prm.M_A, prm.M_B) + prm.M_x
    q = prm.with_(c_eq=tuple(tuple(row[i] for i in perm) for row in prm.c_eq), M_A=mob[perm[0]],
                  M_B=mob[perm[1]], M_x=(mob[perm[2]],))
    sq = lbm.run(lbm.init(phi0, mu[perm[0]], mu[perm[1]], q, mu_x0=(mu[perm[2]],)), q, 60)
    h = (st.hA, st.hB, st.hx[0])
    hq = (sq.hA, sq.hB, sq.hx[0])
    for j, i in enumerate(perm):
        assert np.abs(hq[j] - h[i]).max() <= 1e-13 * np.abs(h[i]).max()
    for key in ("g", "f"):
        assert np.abs(getattr(sq, key) - getattr(st, key)).max() <= 1e-13 * np.abs(getattr(st, key)).max()


def test_ncomp_conserves_every_composition():
    """Streaming and bounce-back permute populations and every h collision conserves
    its zeroth moment, so each composition's total is invariant."""
    prm, phi0, mu = _ncomp_case()
    st = lbm.init(phi0, mu[0], mu[1], prm, mu_x0=(mu[2],))
    d0 = lbm.diagnostics(st, prm)
    st = lbm.run(st, prm, 200)
    d1 = lbm.diagnostics(st, prm)
    for k in ("sum_cA", "sum_cB", "sum_cC"):
        assert abs(d1[k] - d0[k]) <= 1e-12 * abs(d0[k]), k
    assert d1["nan_count"] == 0


def test_ncomp_flat_interface_coexistence():
    """Three compositions: a flat interface with uniform potentials on the coexistence
    plane Delta omega = -sum_alpha mu_alpha (c_0 - c_1)_alpha = 0 stays put (all three
    potentials nonzero); shifted off the plane, phase 1 grows when Delta omega > 0 and
    shrinks when < 0."""
    dc = [C_EQ3[0][a] - C_EQ3[1][a] for a in range(3)]
    muB, muC = 0.01, -0.02
    muA = -(muB * dc[1] + muC * dc[2]) / dc[0]
    assert abs(model.delta_omega((muA, muB, muC), C_EQ3)) < 1e-17
    nx = 48
    x = np.arange(nx) - (nx - 1) / 2.0
    phi0 = (0.5 * (1.0 + np.tanh(2.0 * x / 4.0))).reshape(1, 1, nx)
    prm = lbm.Params(nx=nx, ny=1, bc=("walls", "periodic", "periodic"), W=4.0, lam=2.0, M_phi=0.1,
                     M_A=(0.1, 0.1), M_B=(0.1, 0.1), M_x=((0.1, 0.1),), c_eq=C_EQ3)
    moved = {}
    for shift in (0.0, 0.01, -0.01):
        st = lbm.init(phi0, np.full_like(phi0, muA + shift), np.full_like(phi0, muB), prm,
                      mu_x0=(np.full_like(phi0, muC),))
        s0 = lbm.diagnostics(st, prm)["sum_phi"]
        st = lbm.run(st, prm, 300)
        moved[shift] = lbm.diagnostics(st, prm)["sum_phi"] - s0
    d_plus = model.delta_omega((muA + 0.01, muB, muC), C_EQ3)
    assert abs(moved[0.0]) < 1e-9
    assert np.sign(moved[0.01]) == np.sign(d_plus) and abs(moved[0.01]) > 1e3 * abs(moved[0.0]) + 1e-6
    assert np.sign(moved[-0.01]) == -np.sign(d_plus) and abs(moved[-0.01]) > 1e-6


def test_ncomp_whole_map_matches_exact_rational_arithmetic():
    """The exact rational reference with three compositions: two oracle steps of a 3 x 3
    grid with flow and walls match it to 1e-14 of each field's largest population."""
    import exact_map
    p = _exact_case("2d_flow_walls")
    p.update(c_eq=((0.25, 0.125, 0.1875), (0.625, 0.3125, 0.0625)), M_x=((0.0625, 0.125),))
    shape = (p["nz"], p["ny"], p["nx"])
    nodes = [(x, y, z) for z in range(shape[0]) for y in range(shape[1]) for x in range(shape[2])]
    rng = np.random.default_rng(6)

    def dyadic(lo, hi, den=4096):
        return Fr(int(rng.integers(int(lo * den), int(hi * den) + 1)), den)

    _, sw = exact_map.LATTICES[p["scalar"]]
    _, fw = exact_map.LATTICES[p["fluid"]]
    phi = {x: dyadic(0.05, 0.95) for x in nodes}
    st = {"phi_ref": Fr(0)}
    st["g"] = [{x: sw[k] * phi[x] + dyadic(-0.01, 0.01) for x in nodes} for k in range(len(sw))]
    cs = [{x: dyadic(lo, hi) for x in nodes} for lo, hi in ((0.2, 0.6), (0.1, 0.3), (0.05, 0.2))]
    hs = [[{x: (c[x] if k == 0 else 0) + dyadic(-0.01, 0.01) for x in nodes} for k in range(len(sw))] for c in cs]
    st["hA"], st["hB"], st["hx"] = hs[0], hs[1], [hs[2]]
    st["f"] = [{x: fw[k] * dyadic(-0.01, 0.01) + dyadic(-0.001, 0.001) for x in nodes} for k in range(len(fw))]

    def arr(pops):
        a = np.zeros((len(pops),) + shape)
        for k, d in enumerate(pops):
            for (x, y, z), v in d.items():
                a[k, z, y, x] = float(v)
        return a

    exact_prm = {k: Fr(v) for k, v in p.items() if isinstance(v, float)}
    exact_prm.update(shape=shape, bc=p["bc"], scalar=p["scalar"], fluid=p["fluid"],
                     M_A=tuple(map(Fr, p["M_A"])), M_B=tuple(map(Fr, p["M_B"])), nu=tuple(map(Fr, p["nu"])),
                     M_x=[tuple(map(Fr, m)) for m in p["M_x"]], g=tuple(map(Fr, p["g"])),
                     c_eq=tuple(tuple(map(Fr, r)) for r in p["c_eq"]))
    prm = lbm.Params(**p)
    ost = lbm.State(g=arr(st["g"]), hA=arr(st["hA"]), hB=arr(st["hB"]), f=arr(st["f"]), phi_ref=0.0,
                    hx=(arr(st["hx"][0]),))
    for _ in range(2):
        st = exact_map.step(st, exact_prm)
        ost = lbm.step(ost, prm)
        for got, ex in ((ost.g, st["g"]), (ost.hA, st["hA"]), (ost.hB, st["hB"]), (ost.hx[0], st["hx"][0]),
                        (ost.f, st["f"])):
            e = arr(ex)
            assert np.abs(got - e).max() <= 1e-14 * np.abs(e).max()


# ----------------------------------------------------------------------------------------
# flow

@pytest.mark.slow
def test_poiseuille_between_walls():
    """phi = 1 everywhere: no capillary force, buoyancy is a uniform body force drho g;
    the steady profile between half-way bounce-back walls is the parabola."""
    N, nu = 16, 0.1
    prm = lbm.Params(nx=2, ny=N, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05,
                     drho=1.0, g=(1e-6, 0, 0), sigma=1e-3, nu=(nu, nu))
    phi0 = np.ones(prm.shape)
    st = lbm.run(lbm.init(phi0, 0 * phi0, 0 * phi0, prm), prm, 6000)
    ux = lbm.moments(st, prm)["ux"][0, :, 0]
    ref = analytic.poiseuille(np.arange(N), N, 1e-6, prm.rho0, nu)
    assert np.abs(ux - ref).max() < 0.01 * ref.max()


# ----------------------------------------------------------------------------------------
# TRT collision (the two-relaxation-time alternative to BGK named in Section 3)

@pytest.mark.parametrize("nu,steps", [(0.5, 1000), (0.2, 2200)])
def test_trt_poiseuille_exact(nu, steps):
    """With the magic parameter 3/16 the half-way bounce-back wall sits exactly at
    -1/2 and N - 1/2 for any viscosity: the steady TRT profile is the parabola to
    rounding, where BGK leaves a viscosity-dependent slip."""
    N = 12
    ref = analytic.poiseuille(np.arange(N), N, 1e-6, 1.0, nu)
    errs = {}
    for coll in ("TRT", "BGK"):
        prm = lbm.Params(nx=2, ny=N, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05,
                         drho=1.0, g=(1e-6, 0, 0), sigma=1e-3, nu=(nu, nu), collision=coll,
                         trt_magic=(3.0 / 16.0, 0.25))
        if coll == "BGK" and nu != 0.5:
            continue
        phi0 = np.ones(prm.shape)
        st = lbm.run(lbm.init(phi0, 0 * phi0, 0 * phi0, prm), prm, steps)
        ux = lbm.moments(st, prm)["ux"][0, :, 0]
        errs[coll] = np.abs(ux - ref).max() / ref.max()
    assert errs["TRT"] < 1e-9, errs
    if "BGK" in errs:
        assert errs["BGK"] > 1e-2, errs


def test_trt_equals_bgk_when_rates_coincide():
    """With one rate per lattice and Lambda = tau^2 (tau = 1/w - 1/2) both TRT rates are
    the BGK rate: the two collisions agree to rounding, flow, walls and sources included."""
    rng = np.random.default_rng(8)
    M, nu = 0.1, 0.08
    cs2 = 1.0 / 3.0
    common = dict(nx=26, ny=22, fluid="D2Q9", scalar="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0,
                  lam=21.05, M_phi=M, M_A=(M, M), M_B=(M, M), drho=0.5, g=(0, -1e-4, 0), sigma=1e-3,
                  nu=(nu, nu))
    fields = _droplet_fields((1, 22, 26), [(13, 11, 0)], [5], 4.0, rng)
    a = lbm.run(lbm.init(*fields, lbm.Params(**common)), lbm.Params(**common), 25)
    trt = lbm.Params(**common, collision="TRT", trt_magic=((nu / cs2) ** 2, (M / cs2) ** 2))
    b = lbm.run(lbm.init(*fields, trt), trt, 25)
    for k in ("f", "g", "hA", "hB"):
        assert np.abs(getattr(a, k) - getattr(b, k)).max() < 1e-14, k


@pytest.mark.parametrize("magic", [0.25, 1.0 / 12.0])
def test_trt_fourier_mode_diffusivity(magic):
    """The TRT diffusivity is set by the antisymmetric rate alone: D = c_s^2 (1/w- - 1/2)
    whatever Lambda (to the O(k^2) error of the scheme)."""
    errs = []
    for N in (16, 32):
        M = 0.15
        prm = lbm.Params(nx=N, ny=1, scalar="D2Q9", W=4.0, lam=10.0, M_phi=0.1, M_A=(M, M), M_B=(M, M),
                         c_eq=((0.2, 0.1), (0.6, 0.3)), collision="TRT", trt_magic=(0.25, magic))
        x = np.arange(N)[None, None, :] * np.ones(prm.shape)
        kw = 2 * math.pi / N
        mu0 = 1e-3 * np.sin(kw * x)
        st = lbm.run(lbm.init(np.zeros(prm.shape), mu0, 0 * mu0, prm), prm, 40)
        a0 = (lbm.moments(st, prm)["muA"] * np.sin(kw * x)).sum()
        T = int(2.0 / (M * kw * kw))
        st = lbm.run(st, prm, T)
        a1 = (lbm.moments(st, prm)["muA"] * np.sin(kw * x)).sum()
        errs.append(abs(-math.log(a1 / a0) / T / (M * kw * kw) - 1.0))
    assert errs[1] < 0.02
    assert errs[0] / errs[1] > 3.0


def test_trt_conserves_mass_and_pressure_sum():
    rng = np.random.default_rng(9)
    prm = lbm.Params(nx=24, ny=20, fluid="D2Q9", bc=("walls", "walls", "periodic"), W=4.0, lam=21.05,
                     M_A=(0.1, 0.05), M_B=(0.08, 0.12), drho=0.5, g=(0, -1e-4, 0), sigma=1e-3, nu=(0.1, 0.05),
                     collision="TRT", trt_magic=(3.0 / 16.0, 0.25))
    st = lbm.init(*_droplet_fields(prm.shape, [(12, 10, 0)], [5], 4.0, rng), prm)
    d0, p0 = lbm.diagnostics(st, prm), st.f.sum()
    st = lbm.run(st, prm, 60)
    d1 = lbm.diagnostics(st, prm)
    for key in ("sum_cA", "sum_cB"):
        assert abs(d1[key] - d0[key]) <= 1e-12 * abs(d0[key]), key
    assert abs(st.f.sum() - p0) <= 1e-12 * max(1.0, abs(d0["sum_phi"]))
    assert d1["nan_count"] == 0


# ----------------------------------------------------------------------------------------
# MRT collision (the multiple-relaxation-time alternative named in Section 3)

@pytest.mark.parametrize("lat", [lattices.D2Q5, lattices.D2Q9, lattices.D3Q7, lattices.D3Q19], ids=lambda l: l.name)
def test_moment_basis_exact(lat):
    """Weighted-orthogonal rows, exact inverse M^-1_{k i} = w_k M_ik / <M_i, M_i>, the
    first rows are 1 and c, and the orders run 0, 1, 2 (, 3, 4)."""
    rows, orders = lattices.moment_basis(lat)
    Q = lat.Q
    D = [sum(w * a * a for w, a in zip(lat.w_exact, r)) for r in rows]
    for i in range(Q):
        for j in range(Q):
            dot = sum(w * a * b for w, a, b in zip(lat.w_exact, rows[i], rows[j]))
            assert dot == (D[i] if i == j else 0)
    for k in range(Q):       # (M^-1 M)_{kl} = delta_kl, exactly
        for l in range(Q):
            assert sum(lat.w_exact[k] * rows[i][k] / D[i] * rows[i][l] for i in range(Q)) == (1 if k == l else 0)
    assert all(a == 1 for a in rows[0])
    for a in range(lat.dim):
        assert [int(v) for v in rows[1 + a]] == [int(e[a]) for e in lat.e]
    assert orders == sorted(orders) and orders[:lat.dim + 1] == [0] + [1] * lat.dim


def test_moment_basis_matches_the_classical_d2q9_moments():
    """The classical D2Q9 moment set (density, energy, energy square, momentum, heat
    flux, stresses; orthogonal without weights) and the weighted Gram-Schmidt basis
    span the same spaces order by order: span(rows of order <= k) agree for k = 0..4,
    so the rates given per order act on the same physical moments."""
    rows, orders = lattices.moment_basis(lattices.D2Q9)
    M = np.array([[float(a) for a in r] for r in rows])
    classical = {  # rows in the table order 0, +x, +y, -x, -y, ++, -+, --, +-
        0: [[1, 1, 1, 1, 1, 1, 1, 1, 1]],
        1: [[0, 1, 0, -1, 0, 1, -1, -1, 1], [0, 0, 1, 0, -1, 1, 1, -1, -1]],
        2: [[-4, -1, -1, -1, -1, 2, 2, 2, 2], [0, 1, -1, 1, -1, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1, -1, 1, -1]],
        3: [[0, -2, 0, 2, 0, 1, -1, -1, 1], [0, 0, -2, 0, 2, 1, 1, -1, -1]],
        4: [[4, -2, -2, -2, -2, 1, 1, 1, 1]],
    }
    for k in range(5):
        ours = M[[i for i, o in enumerate(orders) if o <= k]]
        theirs = np.array([r for j in range(k + 1) for r in classical[j]], dtype=float)
        both = np.vstack([ours, theirs])
        assert np.linalg.matrix_rank(ours) == np.linalg.matrix_rank(theirs) == np.linalg.matrix_rank(both), k


@pytest.mark.parametrize("scalar", ["D2Q5", "D2Q9"])
def test_mrt_reduces_to_bgk_and_trt(scalar):
    """Uniform rates: MRT with every free rate equal to the BGK rate is BGK, and with
    even / odd orders at w+ / w- it is TRT (to rounding)."""
    rng = np.random.default_rng(17)
    M, nu, cs2 = 0.1, 0.08, 1.0 / 3.0
    wv, wm = lbm.rate(nu, cs2), lbm.rate(M, cs2)
    common = dict(nx=26, ny=22, fluid="D2Q9", scalar=scalar, bc=("periodic", "walls", "periodic"), W=4.0,
                  lam=21.05, M_phi=M, M_A=(M, M), M_B=(M, M), drho=0.5, g=(0, -1e-4, 0), sigma=1e-3,
                  nu=(nu, nu))
    fields = _droplet_fields((1, 22, 26), [(13, 11, 0)], [5], 4.0, rng)
    run = lambda prm: lbm.run(lbm.init(*fields, prm), prm, 20)
    a = run(lbm.Params(**common))
    b = run(lbm.Params(**common, collision="MRT", mrt_rates=((wv, wv, wv), (wm, wm, wm))))
    lf, ls = 3.0 / 16.0, 0.25
    c = run(lbm.Params(**common, collision="TRT", trt_magic=(lf, ls)))
    wmf, wps = lbm.trt_partner_rate(wv, lf), lbm.trt_partner_rate(wm, ls)
    d = run(lbm.Params(**common, collision="MRT", mrt_rates=((wv, wmf, wv), (wps, wm, wps))))
    for k in ("f", "g", "hA", "hB"):
        assert np.abs(getattr(a, k) - getattr(b, k)).max() < 1e-14, k
        assert np.abs(getattr(c, k) - getattr(d, k)).max() < 1e-14, k


def test_mrt_poiseuille_exact():
    """The wall position depends on the shear and third-order rates only: with
    (1/s_nu - 1/2)(1/s_3 - 1/2) = 3/16 the profile is the parabola whatever the bulk and
    fourth-order rates."""
    N, nu = 12, 0.5
    s3 = lbm.trt_partner_rate(lbm.rate(nu, 1.0 / 3.0), 3.0 / 16.0)
    prm = lbm.Params(nx=2, ny=N, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05, drho=1.0,
                     g=(1e-6, 0, 0), sigma=1e-3, nu=(nu, nu), collision="MRT", mrt_rates=((1.1, s3, 1.3), (1, 1, 1)))
    phi0 = np.ones(prm.shape)
    st = lbm.run(lbm.init(phi0, 0 * phi0, 0 * phi0, prm), prm, 1000)
    ux = lbm.moments(st, prm)["ux"][0, :, 0]
    ref = analytic.poiseuille(np.arange(N), N, 1e-6, 1.0, nu)
    assert np.abs(ux - ref).max() < 1e-9 * ref.max()


def test_mrt_conserves_mass():
    rng = np.random.default_rng(18)
    prm = lbm.Params(nx=24, ny=20, fluid="D2Q9", scalar="D2Q9", bc=("walls", "walls", "periodic"), W=4.0,
                     lam=21.05, M_A=(0.1, 0.05), M_B=(0.08, 0.12), drho=0.5, g=(0, -1e-4, 0), sigma=1e-3,
                     nu=(0.1, 0.05), collision="MRT")
    st = lbm.init(*_droplet_fields(prm.shape, [(12, 10, 0)], [5], 4.0, rng), prm)
    d0, p0 = lbm.diagnostics(st, prm), st.f.sum()
    st = lbm.run(st, prm, 60)
    d1 = lbm.diagnostics(st, prm)
    for key in ("sum_cA", "sum_cB"):
        assert abs(d1[key] - d0[key]) <= 1e-12 * abs(d0[key]), key
    assert abs(st.f.sum() - p0) <= 1e-12 * max(1.0, abs(d0["sum_phi"]))


# ----------------------------------------------------------------------------------------
# variable-density flow (the rho(phi) alternative to Boussinesq named after Eq. Velocity)

def test_variable_density_reduces_to_boussinesq():
    """With equal densities the pressure and viscous forces vanish and the dimensionless
    populations are the Boussinesq ones divided by rho0 c_s^2: same state to rounding."""
    rng = np.random.default_rng(12)
    common = dict(nx=30, ny=24, fluid="D2Q9", bc=("walls", "walls", "periodic"), W=4.0, lam=21.05,
                  rho0=1.7, drho=0.0, g=(0, -1e-4, 0), sigma=2e-3, nu=(0.1, 0.05))
    fields = _droplet_fields((1, 24, 30), [(15, 12, 0)], [6], 4.0, rng)
    pb, pv = lbm.Params(**common), lbm.Params(**common, variable_density=True)
    a = lbm.run(lbm.init(*fields, pb), pb, 40)
    b = lbm.run(lbm.init(*fields, pv), pv, 40)
    assert np.abs(b.f * (1.7 / 3.0) - a.f).max() < 1e-14
    for k in ("g", "hA", "hB"):
        assert np.abs(getattr(a, k) - getattr(b, k)).max() < 1e-14, k
    ma, mb = lbm.moments(a, pb), lbm.moments(b, pv)
    for k in ("p", "ux", "uy"):
        assert np.abs(ma[k] - mb[k]).max() < 1e-14, k
    assert np.abs(ma["ux"]).max() > 1e-6   # the capillary force drives a flow


def _layered_channel_ode(N, W, phi_of, b_of, mu_of):
    """Steady u_x(y) of d/dy (mu(y) du/dy) = -b(y) between walls at -1/2 and N - 1/2
    (trapezoidal quadrature of the closed form on a fine grid)."""
    ys = np.linspace(-0.5, N - 0.5, 100001)
    ph = phi_of(ys)
    b, inv = b_of(ph), 1.0 / mu_of(ph)
    cum = lambda v: np.concatenate([[0.0], np.cumsum(0.5 * (v[1:] + v[:-1]) * np.diff(ys))])
    B = cum(b)
    I1, I2 = cum(inv), cum(B * inv)
    u = I2[-1] / I1[-1] * I1 - I2
    return np.interp(np.arange(N), ys, u)


def test_boussinesq_layered_channel_per_phase_viscosity():
    """The viscosity of Eq. QDM depends on the phase; the reading taken is
    nu(phi) = nu_0 (1 - phi) + nu_1 phi.  Two layers between walls (phase 1 in the lower
    half), driven along them by the buoyancy phi drho g of the Boussinesq model: the
    steady profile solves d/dy (rho0 nu(phi) du/dy) = -phi drho g.  With the phases'
    viscosities exchanged the profile is far off."""
    N, W, drho, nu, g = 24, 4.0, 1.0, (0.2, 0.05), 1e-6
    y0 = N / 2 - 0.5
    phi_of = lambda y: 0.5 * (1.0 + np.tanh(2.0 * (y0 - y) / W))
    prm = lbm.Params(nx=2, ny=N, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=W, lam=21.05,
                     drho=drho, g=(g, 0, 0), sigma=1e-3, nu=nu)
    phi0 = np.repeat(phi_of(np.arange(N))[None, :, None], 2, axis=2)
    z = np.zeros_like(phi0)
    st = lbm.run(lbm.init(phi0, z, z, prm), prm, 4000)
    ux = lbm.moments(st, prm)["ux"][0, :, 0]
    ref = _layered_channel_ode(N, W, phi_of, lambda p: p * drho * g, lambda p: nu[0] * (1 - p) + nu[1] * p)
    swapped = _layered_channel_ode(N, W, phi_of, lambda p: p * drho * g, lambda p: nu[1] * (1 - p) + nu[0] * p)
    assert np.abs(ux - ref).max() < 0.02 * ref.max()
    assert np.abs(swapped - ref).max() > 0.3 * ref.max()


def test_variable_density_layered_channel():
    """Two layers (density ratio 4, viscosity ratio 1/2) between walls, driven along the
    layers by the buoyancy of the dense one: the steady profile solves
    d/dy (rho nu du/dy) = -b with the dynamic viscosity rho(phi) nu(phi), which needs the
    viscous force; the Boussinesq model's rho0 nu(phi) profile is far off."""
    N, W, drho, nu, g = 24, 4.0, 3.0, (0.2, 0.1), 1e-6
    y0 = N / 2 - 0.5
    phi_of = lambda y: 0.5 * (1.0 + np.tanh(2.0 * (y0 - y) / W))
    prm = lbm.Params(nx=2, ny=N, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=W, lam=21.05,
                     drho=drho, g=(g, 0, 0), sigma=1e-3, nu=nu, variable_density=True)
    phi0 = np.repeat(phi_of(np.arange(N))[None, :, None], 2, axis=2)
    z = np.zeros_like(phi0)
    st = lbm.run(lbm.init(phi0, z, z, prm), prm, 3000)
    ux = lbm.moments(st, prm)["ux"][0, :, 0]
    visc = lambda p: nu[0] * (1 - p) + nu[1] * p
    ref = _layered_channel_ode(N, W, phi_of, lambda p: p * drho * g, lambda p: (1.0 + drho * p) * visc(p))
    bous = _layered_channel_ode(N, W, phi_of, lambda p: p * drho * g, lambda p: 1.0 * visc(p))
    assert np.abs(ux - ref).max() < 0.02 * ref.max()
    assert np.abs(ux - bous).max() > 0.3 * bous.max()


def test_variable_density_conserves_mass():
    rng = np.random.default_rng(13)
    prm = lbm.Params(nx=26, ny=22, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05,
                     drho=2.0, g=(0, -1e-5, 0), sigma=1e-3, nu=(0.1, 0.05), variable_density=True,
                     collision="TRT")
    st = lbm.init(*_droplet_fields(prm.shape, [(13, 11, 0)], [5], 4.0, rng), prm)
    d0 = lbm.diagnostics(st, prm)
    st = lbm.run(st, prm, 60)
    d1 = lbm.diagnostics(st, prm)
    for key in ("sum_cA", "sum_cB"):
        assert abs(d1[key] - d0[key]) <= 1e-12 * abs(d0[key]), key
    assert d1["nan_count"] == 0 and d1["max_u"] > 0


# ----------------------------------------------------------------------------------------
# general curvature matrices K_pi (Eq. Taylor with a full matrix; the paper's model has
# K_pi = K identity)

KAPPA = ((1.0, 0.1, 0.9), (0.95, -0.05, 1.2))   # (k_AA, k_AB, k_BB) of phases 0 and 1
C_EQ = ((0.2, 0.1), (0.6, 0.3))


def _legendre_numeric(mu, c_eq_pi, kappa_pi):
    """omega(mu) = min_c [f(c) - mu . c] with f(c) = 1/2 (c - c_eq) . K^-1 (c - c_eq),
    by numerical minimisation (independent of the closed form)."""
    from scipy.optimize import minimize
    kAA, kAB, kBB = kappa_pi
    Kinv = np.linalg.inv(np.array([[kAA, kAB], [kAB, kBB]]))
    ce = np.array(c_eq_pi)
    fun = lambda c: 0.5 * (c - ce) @ Kinv @ (c - ce) - np.dot(mu, c)
    r = minimize(fun, ce, method="BFGS", options=dict(gtol=1e-13))
    return r.fun, r.x


def test_general_curvature_grand_potential_is_the_legendre_transform():
    rng = np.random.default_rng(14)
    for _ in range(5):
        mu = rng.uniform(-0.1, 0.1, 2)
        for pi in range(2):
            w_num, c_num = _legendre_numeric(mu, C_EQ[pi], KAPPA[pi])
            assert abs(model.grand_potential(tuple(mu), C_EQ[pi], KAPPA[pi]) - w_num) < 1e-12
            c = model.closure_c(tuple(mu), float(pi), C_EQ, KAPPA)  # phi = 0 or 1: the pure phase
            np.testing.assert_allclose(c, c_num, atol=1e-7)


def test_general_curvature_closure():
    """c = -d omega / d mu of the interpolated grand potential (complex step), and
    closure_mu inverts closure_c; identity curvatures give the paper's closure."""
    rng = np.random.default_rng(15)
    phi = rng.uniform(0, 1, 6)
    mu = (rng.uniform(-0.1, 0.1, 6), rng.uniform(-0.1, 0.1, 6))
    c = model.closure_c(mu, phi, C_EQ, KAPPA)
    h = 1e-30
    for a in range(2):
        mp = [mu[0] + 0j, mu[1] + 0j]
        mp[a] = mp[a] + 1j * h
        om = (1 - model.p(phi)) * model.grand_potential(mp, C_EQ[0], KAPPA[0]) + \
            model.p(phi) * model.grand_potential(mp, C_EQ[1], KAPPA[1])
        np.testing.assert_allclose(-om.imag / h, c[a], rtol=1e-13)
    back = model.closure_mu(c, phi, C_EQ, KAPPA)
    np.testing.assert_allclose(back[0], mu[0], atol=1e-15)
    np.testing.assert_allclose(back[1], mu[1], atol=1e-15)
    ident = ((1.0, 0.0, 1.0), (1.0, 0.0, 1.0))
    np.testing.assert_allclose(model.closure_mu(c, phi, C_EQ, ident), model.closure_mu(c, phi, C_EQ), atol=1e-15)
    np.testing.assert_allclose(model.delta_omega(mu, C_EQ, ident), model.delta_omega(mu, C_EQ), atol=1e-16)


def test_general_curvature_flat_interface_coexistence():
    """A flat interface with uniform mu on the coexistence line Delta omega(mu) = 0 stays
    put; shifted off it, phase 1 grows when Delta omega > 0 and shrinks when < 0."""
    from scipy.optimize import brentq
    muB = 0.02
    muA = brentq(lambda a: model.delta_omega((a, muB), C_EQ, KAPPA), -0.2, 0.2)
    nx = 48
    x = np.arange(nx) - (nx - 1) / 2.0
    phi0 = (0.5 * (1.0 + np.tanh(2.0 * x / 4.0))).reshape(1, 1, nx)
    prm = lbm.Params(nx=nx, ny=1, bc=("walls", "periodic", "periodic"), W=4.0, lam=2.0, M_phi=0.1,
                     M_A=(0.1, 0.1), M_B=(0.1, 0.1), c_eq=C_EQ, kappa=KAPPA)
    moved = {}
    for shift in (0.0, 0.01, -0.01):
        m0 = np.full_like(phi0, muA + shift)
        st = lbm.init(phi0, m0, np.full_like(phi0, muB), prm)
        s0 = lbm.diagnostics(st, prm)["sum_phi"]
        st = lbm.run(st, prm, 300)
        moved[shift] = lbm.diagnostics(st, prm)["sum_phi"] - s0
    d_plus = model.delta_omega((muA + 0.01, muB), C_EQ, KAPPA)
    # at coexistence only the start-up transient moves the interface (unequal
    # curvatures make it asymmetric): 2% of the motion off coexistence
    assert abs(moved[0.0]) < 5e-3
    assert np.sign(moved[0.01]) == np.sign(d_plus) and abs(moved[0.01]) > 20 * abs(moved[0.0])
    assert np.sign(moved[-0.01]) == -np.sign(d_plus) and abs(moved[-0.01]) > 20 * abs(moved[0.0])


@pytest.mark.parametrize("scalar,stable,unstable", [("D2Q5", 0.70, 0.65), ("D2Q9", 0.5, None)])
def test_general_curvature_lattice_stability(scalar, stable, unstable):
    """The composition lattice relaxes h towards w_k mu with mu = kappa^-1 (c - c^eq):
    on D2Q5 a checkerboard mode grows once the smallest eigenvalue of kappa drops below
    1 - w_0 = 2/3 (the limit the library enforces); D2Q9 stays stable further down."""
    def growth(k):
        prm = lbm.Params(nx=32, ny=32, scalar=scalar, W=3.0, lam=2.0, kappa=((k, 0.0, k), (k, 0.0, k)))
        mu = 1e-6 * np.random.default_rng(1).standard_normal((2,) + prm.shape)
        st = lbm.run(lbm.init(np.zeros(prm.shape), mu[0], mu[1], prm), prm, 200)
        return np.abs(lbm.moments(st, prm)["muA"]).max() / np.abs(mu[0]).max()
    assert growth(stable) < 1.0
    if unstable is not None:
        assert growth(unstable) > 1e3


def test_general_curvature_run_conserves_and_matches_identity():
    rng = np.random.default_rng(16)
    common = dict(nx=28, ny=22, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05,
                  drho=0.5, g=(0, -1e-4, 0), sigma=1e-3, nu=(0.1, 0.05))
    fields = _droplet_fields((1, 22, 28), [(14, 11, 0)], [6], 4.0, rng)
    a = lbm.Params(**common)
    b = lbm.Params(**common, kappa=((1.0, 0.0, 1.0), (1.0, 0.0, 1.0)))
    sa = lbm.run(lbm.init(*fields, a), a, 30)
    sb = lbm.run(lbm.init(*fields, b), b, 30)
    for k in ("f", "g", "hA", "hB"):
        assert np.abs(getattr(sa, k) - getattr(sb, k)).max() < 1e-13, k
    c = lbm.Params(**common, kappa=KAPPA)
    st = lbm.init(*fields, c)
    d0 = lbm.diagnostics(st, c)
    st = lbm.run(st, c, 40)
    d1 = lbm.diagnostics(st, c)
    for key in ("sum_cA", "sum_cB"):
        assert abs(d1[key] - d0[key]) <= 1e-12 * abs(d0[key]), key


@pytest.mark.slow
def test_laplace_pressure_jump():
    """Static 2D drop with no driving force: p_in - p_out = sigma / R (within the spurious
    current error of the diffuse-interface force Eq. SurfaceTension_Force)."""
    N, W, R, sigma = 64, 4.0, 16.0, 1e-3
    prm = lbm.Params(nx=N, ny=N, fluid="D2Q9", W=W, lam=21.05, M_phi=0.002, c_eq=((0.3, 0.3), (0.3, 0.3)),
                     drho=0.0, sigma=sigma, nu=(0.2, 0.2))
    z, y, x = np.meshgrid(np.arange(1), np.arange(N), np.arange(N), indexing="ij")
    r = np.sqrt((x - N / 2 + 0.5) ** 2 + (y - N / 2 + 0.5) ** 2)
    phi0 = analytic.tanh_profile(R - r, W)
    st = lbm.run(lbm.init(phi0, 0 * phi0, 0 * phi0, prm), prm, 1500)
    m = lbm.moments(st, prm)
    R_now = math.sqrt(m["phi"].sum() / math.pi)
    dp = m["p"][r < R - 2 * W].mean() - m["p"][r > R + 2 * W].mean()
    assert abs(dp / analytic.laplace_jump(sigma, R_now) - 1.0) < 0.05


# ----------------------------------------------------------------------------------------
# free-energy decrease without flow

def test_free_energy_decreases_without_flow():
    rng = np.random.default_rng(11)
    prm = lbm.Params(nx=48, ny=40, W=3.0, lam=21.05, M_phi=0.1, M_A=(0.1, 0.1), M_B=(0.1, 0.1))
    st = lbm.init(*_droplet_fields(prm.shape, [(12, 12, 0), (32, 26, 0), (36, 8, 0)], [7, 5, 4], 3.0, rng,
                                   noise=2e-3), prm)
    F = [lbm.diagnostics(st, prm)["free_energy"]]
    for _ in range(8):
        st = lbm.run(st, prm, 25)
        F.append(lbm.diagnostics(st, prm)["free_energy"])
    assert all(b < a for a, b in zip(F, F[1:]))


# ----------------------------------------------------------------------------------------
# complex-step derivatives of the oracle against central differences

def test_complex_step_matches_central_difference():
    rng = np.random.default_rng(2)
    base = lbm.Params(nx=16, ny=14, fluid="D2Q9", bc=("periodic", "walls", "periodic"), W=4.0, lam=21.05,
                      M_phi=0.1, M_A=(0.1, 0.1), M_B=(0.1, 0.1), drho=0.5, g=(0, -1e-4, 0), sigma=1e-3,
                      nu=(0.1, 0.05))
    phi0, muA, muB = _droplet_fields(base.shape, [(8, 7, 0)], [4.5], 4.0, rng)

    def loss(M, W, dphi=0.0):
        prm = base.with_(M_phi=M, M_A=(M, M), M_B=(M, M), W=W)
        st = lbm.run(lbm.init(phi0 + dphi, muA, muB, prm), prm, 12)
        return (lbm.moments(st, prm)["phi"] ** 2).sum()

    h = 1e-30
    dM_cs = loss(0.1 + 1j * h, 4.0).imag / h
    dW_cs = loss(0.1, 4.0 + 1j * h).imag / h
    v = rng.normal(size=phi0.shape)
    dv_cs = loss(0.1, 4.0, 1j * h * v).imag / h
    e = 1e-5
    dM_fd = (loss(0.1 + e, 4.0) - loss(0.1 - e, 4.0)) / (2 * e)
    dW_fd = (loss(0.1, 4.0 + e) - loss(0.1, 4.0 - e)) / (2 * e)
    dv_fd = (loss(0.1, 4.0, e * v) - loss(0.1, 4.0, -e * v)) / (2 * e)
    for a, b in ((dM_cs, dM_fd), (dW_cs, dW_fd), (dv_cs, dv_fd)):
        assert abs(a - b) <= 1e-6 * max(abs(a), 1e-3)

"""Exact rational arithmetic reference of the discrete map (test infrastructure only).

A second, independent statement of one time step of the coupled lattice-Boltzmann
scheme of Section 3, written node by node with Python fractions.  Every operation of
the step is +, -, x or / (the rates 1 / (D / c_s^2 + 1/2) included), so on rational
inputs this reference is exact.  It shares no code with the FP64 oracle (`oracle/`):
its lattice tables are typed from Tables tab:D2Q9 and tab:D3Q19 (and the reduced
scalar lattices of the workloads: D2Q5 with w = 1/3, 1/6 ordered 0, +x, +y, -x, -y;
D3Q7 with w = 1/4, 1/8 ordered 0, +x, -x, +y, -y, +z, -z), its formulas are written
in the form of the paper's equations rather than the oracle's, and it walks the
nodes one at a time.  It serves to pin the whole oracle step to rounding error.

One step, in the paper's order:
  moments and closure   c = sum h (Eq. Moment0_c_alpha), phi* = sum g, one predictor
                        evaluation of the source (Eqs. Moment0_Phi, SourceTerm_Phi,
                        PotChem), then mu and S at the corrected phi;
  phase-field stencil   Eqs. DerivDirec_Grad, Grad, DerivDirect_Laplacian, Laplacian on
                        the fluid lattice, mirror ghosts beyond half-way walls;
  force and flow        buoyancy (phi - phi_ref) drho g and Eq. SurfaceTension_Force;
                        Eqs. HydroPressure and Velocity;
  collisions            Eqs. LBE_FluidFlow, ForcingTerm, GammaFunction, Feq (f);
                        LBE_Phi, Geq, Source_LBE_Phi (g); LBE_c_alpha, Heq (h^A, h^B);
                        mobility and viscosity interpolated linearly in phi;
  streaming             periodic, or half-way bounce-back across a wall (Section 4.2.4).
With gravity_mean_subtract the buoyancy reference of the next step is the mean of phi.
"""

from fractions import Fraction as Fr

# ---- velocity sets ---------------------------------------------------------------------

LATTICES = {
    # Table tab:D2Q9
    "D2Q9": ([(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
              (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)],
             [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4),
    # Table tab:D3Q19
    "D3Q19": ([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
               (1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1),
               (1, -1, 0), (-1, 1, 0), (1, 0, -1), (-1, 0, 1), (0, 1, -1), (0, -1, 1)],
              [Fr(1, 3)] + [Fr(1, 18)] * 6 + [Fr(1, 36)] * 12),
    "D2Q5": ([(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0)],
             [Fr(1, 3)] + [Fr(1, 6)] * 4),
    "D3Q7": ([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
             [Fr(1, 4)] + [Fr(1, 8)] * 6),
}


def sound_speed2(name):
    """c_s^2 = sum_k w_k e_kx^2."""
    e, w = LATTICES[name]
    return sum(wk * ek[0] * ek[0] for ek, wk in zip(e, w))


def opposite(name, k):
    e, _ = LATTICES[name]
    return e.index(tuple(-c for c in e[k]))


# ---- thermodynamics of Section 2 ------------------------------------------------------

def interp(phi):
    """p(phi) = 3 phi^2 - 2 phi^3."""
    return 3 * phi * phi - 2 * phi * phi * phi


def interp_d(phi):
    """p'(phi) = 6 phi - 6 phi^2."""
    return 6 * phi - 6 * phi * phi


def double_well_d(phi):
    """d/dphi of 8 phi^2 (1 - phi)^2, by the product rule."""
    return 16 * phi * (1 - phi) * (1 - phi) - 16 * phi * phi * (1 - phi)


def potentials(c, phi, prm):
    """Eq. PotChem with p(1 - phi) = 1 - p(phi), for every composition."""
    q = interp(phi)
    return [c[a] - (1 - q) * prm["c_eq"][0][a] - q * prm["c_eq"][1][a] for a in range(len(c))]


def grand_potential(mu, c_eq_pi):
    """Eq. dimless_grand_potentials: -1/2 sum (mu^2 + 2 mu c_eq)."""
    return -Fr(1, 2) * sum(mu[a] * mu[a] + 2 * mu[a] * c_eq_pi[a] for a in range(len(mu)))


def source(phi, mu, prm):
    """Eq. SourceTerm_Phi with 1 / tau_phi = M_phi / W^2."""
    inv_tau = prm["M_phi"] / (prm["W"] * prm["W"])
    d_omega = grand_potential(mu, prm["c_eq"][0]) - grand_potential(mu, prm["c_eq"][1])
    return inv_tau * (-double_well_d(phi) + prm["lam"] * interp_d(phi) * d_omega)


# ---- the step -------------------------------------------------------------------------

def _nodes(shape):
    nz, ny, nx = shape
    return [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]


def _shift(node, e, shape, bc, mirror):
    """Node node + e: periodic wrap; across a wall either the node itself (mirror ghost,
    when `mirror`) or None."""
    n = (shape[2], shape[1], shape[0])
    out = []
    for a in range(3):
        c = node[a] + e[a]
        if 0 <= c < n[a]:
            out.append(c)
        elif bc[a] == "periodic":
            out.append(c % n[a])
        elif mirror:
            out.append(node[a])
        else:
            return None
    return tuple(out)


def step(state, prm):
    """One step of the map on exact rationals.

    state: dict with 'g', 'hA', 'hB' (and 'f' with flow; 'hx', a list, for compositions
    beyond A and B) mapping to lists over k of dicts node (x, y, z) -> Fraction, and
    'phi_ref'.  prm: dict of Fractions and names (see the keys used below; 'M_x' the
    mobility pairs of the extra compositions).  Returns the new state."""
    shape = prm["shape"]
    bc = prm["bc"]
    nodes = _nodes(shape)
    sname, fname = prm["scalar"], prm["fluid"]
    se, sw = LATTICES[sname]
    cs2_s = sound_speed2(sname)
    dim = 2 if sname in ("D2Q5", "D2Q9") else 3
    stencil = "D2Q9" if dim == 2 else "D3Q19"

    # moments, closure, predictor
    hfields = [state["hA"], state["hB"]] + list(state.get("hx", []))
    mobil = [prm["M_A"], prm["M_B"]] + list(prm.get("M_x", []))
    mom = {}
    for x in nodes:
        c = [sum(h[k][x] for k in range(len(sw))) for h in hfields]
        phi_s = sum(state["g"][k][x] for k in range(len(sw)))
        s_star = source(phi_s, potentials(c, phi_s, prm), prm)
        phi = phi_s + s_star / 2
        mu = potentials(c, phi, prm)
        mom[x] = dict(c=c, phi=phi, mu=mu, S=source(phi, mu, prm))

    # phase-field stencil, force and flow moments
    u = {x: [Fr(0)] * 3 for x in nodes}
    F = {x: [Fr(0)] * 3 for x in nodes}
    p_h = {}
    if fname:
        te, tw = LATTICES[stencil]
        fe, fw = LATTICES[fname]
        cs2_f = sound_speed2(fname)
        for x in nodes:
            phi = mom[x]["phi"]
            grad = [Fr(0)] * 3
            lap = Fr(0)
            for k in range(1, len(tw)):
                fwd = mom[_shift(x, te[k], shape, bc, True)]["phi"]
                bwd = mom[_shift(x, tuple(-c for c in te[k]), shape, bc, True)]["phi"]
                directional = (fwd - bwd) / 2                      # Eq. DerivDirec_Grad
                for a in range(3):
                    grad[a] += 3 * tw[k] * te[k][a] * directional   # Eq. Grad
                lap += 3 * tw[k] * (fwd - 2 * phi + bwd)             # Eqs. DerivDirect_Laplacian, Laplacian
            bracket = Fr(3, 2) * prm["sigma"] * prm["W"] * (double_well_d(phi) / (prm["W"] * prm["W"]) - lap)
            F[x] = [(phi - state["phi_ref"]) * prm["drho"] * prm["g"][a] + bracket * grad[a] for a in range(3)]
            p_h[x] = sum(state["f"][k][x] for k in range(len(fw)))
            u[x] = [(sum(state["f"][k][x] * fe[k][a] for k in range(len(fw))) / cs2_f + F[x][a] / 2) / prm["rho0"]
                    for a in range(3)]

    def dot(e, v):
        return e[0] * v[0] + e[1] * v[1] + e[2] * v[2]

    post = {key: [dict() for _ in range(len(sw))] for key in ("g",)}
    post["h"] = [[dict() for _ in range(len(sw))] for _ in hfields]
    rate_g = 1 / (prm["M_phi"] / cs2_s + Fr(1, 2))
    for x in nodes:
        phi, S, vel = mom[x]["phi"], mom[x]["S"], u[x]
        for k in range(len(sw)):
            Gk = sw[k] * S                                                   # Eq. Source_LBE_Phi
            geq = sw[k] * phi * (1 + dot(se[k], vel) / cs2_s) - Gk / 2       # Eq. Geq
            gk = state["g"][k][x]
            post["g"][k][x] = gk - rate_g * (gk - geq) + Gk                  # Eq. LBE_Phi
        for a, (hf, Mpair) in enumerate(zip(hfields, mobil)):
            M = Mpair[0] * (1 - phi) + Mpair[1] * phi
            rate_h = 1 / (M / cs2_s + Fr(1, 2))
            c, mu = mom[x]["c"][a], mom[x]["mu"][a]
            for k in range(len(sw)):
                if k == 0:
                    heq = c - (1 - sw[0]) * mu                               # Eq. Heq
                else:
                    heq = sw[k] * mu + sw[k] * c * dot(se[k], vel) / cs2_s
                hk = hf[k][x]
                post["h"][a][k][x] = hk - rate_h * (hk - heq)                # Eq. LBE_c_alpha
    if fname:
        post["f"] = [dict() for _ in range(len(fw))]
        for x in nodes:
            phi, vel, Ft = mom[x]["phi"], u[x], F[x]
            nu = prm["nu"][0] * (1 - phi) + prm["nu"][1] * phi
            rate_f = 1 / (nu / cs2_f + Fr(1, 2))
            uu = dot(vel, vel)
            for k in range(len(fw)):
                eu = dot(fe[k], vel)
                gamma = fw[k] * (1 + eu / cs2_f + eu * eu / (2 * cs2_f * cs2_f) - uu / (2 * cs2_f))  # Eq. GammaFunction
                Fk = gamma * sum((fe[k][a] - vel[a]) * Ft[a] for a in range(3))                      # Eq. ForcingTerm
                feq = fw[k] * (p_h[x] + prm["rho0"] * cs2_f * (eu / cs2_f + eu * eu / (2 * cs2_f * cs2_f)
                                                                - uu / (2 * cs2_f))) - Fk / 2          # Eq. Feq
                fk = state["f"][k][x]
                post["f"][k][x] = fk - rate_f * (fk - feq) + Fk                                        # Eq. LBE_FluidFlow

    # streaming: X_k(x + e_k) <- X*_k(x), or back into X_opp(k)(x) across a wall
    def streamed(pops, name):
        e, _ = LATTICES[name]
        out = [dict() for _ in range(len(e))]
        for x in nodes:
            for k in range(len(e)):
                dest = _shift(x, e[k], shape, bc, False)
                if dest is None:
                    out[opposite(name, k)][x] = pops[k][x]
                else:
                    out[k][dest] = pops[k][x]
        return out

    new = {"g": streamed(post["g"], sname)}
    hs = [streamed(h, sname) for h in post["h"]]
    new["hA"], new["hB"] = hs[0], hs[1]
    if len(hs) > 2:
        new["hx"] = hs[2:]
    if fname:
        new["f"] = streamed(post["f"], fname)
    new["phi_ref"] = (sum(mom[x]["phi"] for x in nodes) / len(nodes) if prm.get("gravity_mean_subtract")
                      else state["phi_ref"])
    return new

"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws initial fields and holds the workload recipes (grid,
lattices, boundaries, parameters, step counts).  It contains none of the
method's arithmetic: the compositions, sources and populations are derived from
(phi_0, mu_0) inside each implementation.  The one exception is an input by
definition: the paper's own initial condition (Section 4.2.1) prescribes the
compositions directly (Eq. Compos_Init, with mu_0 = 0), and its recipe (droplet
placement by phase fraction, lever rule, supersaturation offset) lives here.
Both the GPU library's callers and the oracle-based tests take their inputs
from here.

Initial phase field: circular / spherical droplets with the equilibrium
profile of Eq. tanh, phi = (1 + tanh(2 (R - r) / W)) / 2, r the minimum-image
distance to the droplet centre, combined by taking the largest value (the
profile of the droplet whose surface is closest, Section 4.2.1).
"""

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

SEED = 240903401

# coupling constant that cancels the kinetic coefficient (Eq. KineticCoeff) for
# equal mobilities and the tie line c_0 = (0.2, 0.1), c_1 = (0.6, 0.3):
# 80 / (19 * sum (c_0 - c_1)^2) = 80 / (19 * 0.2)
LAMBDA_TIE = 80.0 / (19.0 * 0.2)
# the paper's diffusion-couple value (Table tab:Parameters_Diffusion-Couple)
LAMBDA_PAPER = 155.94541910
TIE_LINE = ((0.2, 0.1), (0.6, 0.3))


def rng_for(i: int) -> np.random.Generator:
    """Independent stream number i (child i of SeedSequence(SEED))."""
    return np.random.default_rng(np.random.SeedSequence(SEED).spawn(i + 1)[i])


def place_droplets(shape, n, rmin, rmax, W, rng, wall_axes=(), max_tries=200000):
    """Random non-overlapping droplets: radius ~ U[rmin, rmax], centre uniform; a
    candidate is rejected when its minimum-image distance to an accepted droplet is
    below R_i + R_j + W, or when it comes closer than R + W/2 to a wall (the
    clearances of Fig. initialization_flowchart).  Returns [(centre_xyz, R)]."""
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    ndim = 3 if nz > 1 else 2
    drops = []
    tries = 0
    while len(drops) < n and tries < max_tries:
        tries += 1
        R = rng.uniform(rmin, rmax)
        c = [rng.uniform(0, dims[a]) if a < ndim else 0.0 for a in range(3)]
        ok = True
        for a in wall_axes:
            if c[a] < R + W / 2 or c[a] > dims[a] - 1 - R - W / 2:
                ok = False
        if not ok:
            continue
        for (c2, R2) in drops:
            d2 = 0.0
            for a in range(ndim):
                d = abs(c[a] - c2[a])
                if a not in wall_axes:
                    d = min(d, dims[a] - d)
                d2 += d * d
            if d2 < (R + R2 + W) ** 2:
                ok = False
                break
        if ok:
            drops.append((tuple(c), R))
    return drops


def droplet_field(shape, drops, W, wall_axes=()):
    """phi_0 on [z][y][x] from a droplet list (profile of Eq. tanh, max over droplets)."""
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    ndim = 3 if nz > 1 else 2
    phi = np.zeros(shape)
    reach = 3.0 * W
    for (c, R) in drops:
        # index ranges covering the droplet plus the tanh tail, with periodic images
        sl = []
        coords = []
        for a in range(3):
            if a >= ndim:
                coords.append(np.zeros(1))
                sl.append(np.zeros(1, dtype=np.int64))
                continue
            lo = int(math.floor(c[a] - R - reach))
            hi = int(math.ceil(c[a] + R + reach))
            idx = np.arange(lo, hi + 1)
            if a in wall_axes:
                idx = idx[(idx >= 0) & (idx < dims[a])]
                coords.append(idx.astype(float))
                sl.append(idx)
            else:
                if hi - lo + 1 >= dims[a]:
                    idx = np.arange(dims[a])
                    d = idx - c[a]
                    d = d - dims[a] * np.round(d / dims[a])
                    coords.append(c[a] + d)
                    sl.append(idx)
                else:
                    coords.append(idx.astype(float))
                    sl.append(np.mod(idx, dims[a]))
        X, Y, Z = np.meshgrid(coords[0], coords[1], coords[2], indexing="ij")
        r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        prof = 0.5 * (1.0 + np.tanh(2.0 * (R - r) / W))   # Eq. tanh
        zi, yi, xi = np.ix_(sl[2], sl[1], sl[0])
        blk = np.transpose(prof, (2, 1, 0))
        phi[zi, yi, xi] = np.maximum(phi[zi, yi, xi], blk)
    return phi


# ----------------------------------------------------------------------------------------
# the paper's initial condition (Section 4.2.1)

def lever_rule_fraction(cg, c0, c1):
    """Eq. phi_glob_eq: equilibrium phase fraction of the inventory cg on the tie line
    from c0 (phase 0) to c1 (phase 1)."""
    return float(np.linalg.norm(np.subtract(c0, cg)) / np.linalg.norm(np.subtract(c0, c1)))


def supersaturation_offset(phi_eq, phi_frac):
    """Eq. Delta-1: delta = (Phi_eq - Phi) / (1 - Phi)."""
    return (phi_eq - phi_frac) / (1.0 - phi_frac)


def stepped_composition(phi, c_eq, cg):
    """Eq. Compos_Init: c = c_1 where phi >= 1/2, c = (1 - delta) c_0 + delta c_1
    elsewhere, delta from Eqs. phi_glob_eq and Delta-1.  Readings: Phi is the fraction
    of nodes with phi >= 1/2, so that the mean composition is cg exactly; the matrix
    offset is + delta (c_1 - c_0), as in Eq. Compos_Init and the inventory balance
    (Eq. Init_c0 prints the opposite sign).  Returns (cA, cB) and the recipe values."""
    phi = np.asarray(phi)
    c0, c1 = np.asarray(c_eq[0], float), np.asarray(c_eq[1], float)
    inside = phi >= 0.5
    frac = float(inside.mean())
    phi_eq = lever_rule_fraction(cg, c0, c1)
    delta = supersaturation_offset(phi_eq, frac)
    matrix = (1.0 - delta) * c0 + delta * c1
    cA = np.where(inside, c1[0], matrix[0])
    cB = np.where(inside, c1[1], matrix[1])
    return (cA, cB), dict(phase_fraction=frac, phi_eq=phi_eq, delta=delta, matrix=tuple(matrix))


def place_droplets_by_fraction(shape, s, vmin, vmax, W, rng, max_tries=2_000_000):
    """Droplet ensemble of Fig. initialization_flowchart: volume (area in 2D) V ~ U[vmin,
    vmax], centre uniform in the box.  A candidate is discarded when its centre lies
    within R_max + W/2 of a domain bound or within 2 (R_max + W/2) of an accepted
    centre, R_max the radius of volume vmax.  Droplets are added until their volumes
    reach s times the domain volume (reading: the last accepted droplet may pass it).
    Returns [(centre_xyz, R)]."""
    nz, ny, nx = shape
    dims = np.array([nx, ny, nz], float)
    ndim = 3 if nz > 1 else 2
    radius = (lambda V: math.sqrt(V / math.pi)) if ndim == 2 else (lambda V: (3.0 * V / (4.0 * math.pi)) ** (1 / 3))
    clear = radius(vmax) + W / 2
    target = s * float(np.prod(dims[:ndim]))
    centres = np.zeros((0, ndim))
    drops, total, tries = [], 0.0, 0
    while total < target and tries < max_tries:
        tries += 1
        V = rng.uniform(vmin, vmax)
        c = rng.uniform(0.0, 1.0, ndim) * dims[:ndim]
        if np.any(c < clear) or np.any(c > dims[:ndim] - clear):
            continue
        if len(centres) and np.min(np.sum((centres - c) ** 2, axis=1)) < (2 * clear) ** 2:
            continue
        centres = np.vstack([centres, c])
        drops.append((tuple(c) + (0.0,) * (3 - ndim), radius(V)))
        total += V
    return drops


@dataclass
class Workload:
    name: str
    params: Dict            # shared parameter set (LBMConfig / oracle Params field names)
    precision: str
    steps: int
    phi0: np.ndarray
    muA0: np.ndarray
    muB0: np.ndarray
    note: str = ""
    drops: Optional[List] = None
    c0: Optional[Tuple[np.ndarray, np.ndarray]] = None   # given compositions (paper's initial condition)

    @property
    def nodes(self):
        return int(np.prod(self.phi0.shape))


def _base(nx, ny, nz, **kw):
    p = dict(nx=nx, ny=ny, nz=nz, W=4.0, lam=LAMBDA_TIE, M_phi=0.1, M_A=(0.1, 0.1), M_B=(0.1, 0.1),
             c_eq=TIE_LINE, rho0=1.0, drho=0.0, g=(0.0, 0.0, 0.0), sigma=0.0, nu=(0.1, 0.1),
             fluid=None, scalar="D2Q5" if nz == 1 else "D3Q7",
             bc=("periodic", "periodic", "periodic"), gravity_mean_subtract=False)
    p.update(kw)
    return p


def diffusion_couple_tie(nx=512):
    """C1a: quasi-1D couple on the tie line, both halves at equilibrium; FP64, walls in x."""
    p = _base(nx, 1, 1, bc=("walls", "periodic", "periodic"))
    x = np.arange(nx) - (nx - 1) / 2.0
    phi0 = 0.5 * (1.0 + np.tanh(2.0 * x / p["W"]))
    z = np.zeros((1, 1, nx))
    return Workload("diffusion_couple_512_fp64", p, "fp64", 2000, phi0.reshape(1, 1, nx), z, z.copy(),
                    note="left phase 0 (0.2, 0.1), right phase 1 (0.6, 0.3), mu_0 = 0")


def diffusion_couple_paper(nx=512):
    """C1b: the paper's couple (Table tab:Parameters_Diffusion-Couple) in lattice units:
    mobilities scaled by 0.1, W = 4, far-field potentials as printed."""
    p = _base(nx, 1, 1, bc=("walls", "periodic", "periodic"), lam=LAMBDA_PAPER, M_phi=0.12,
              M_A=(0.1, 0.1), M_B=(0.08, 0.08), c_eq=((0.3, 0.3), (0.4, 0.4)))
    x = np.arange(nx) - (nx - 1) / 2.0
    phi0 = 0.5 * (1.0 + np.tanh(2.0 * x / p["W"]))
    muA0 = np.where(x < 0, 0.1, -0.175)
    muB0 = np.where(x < 0, -0.125, 0.2)
    return Workload("diffusion_couple_paper_512_fp64", p, "fp64", 2000, phi0.reshape(1, 1, nx),
                    muA0.reshape(1, 1, nx), muB0.reshape(1, 1, nx))


def ostwald_2d(n=1024, ndrops=400, precision="fp32", rng_index=1):
    """C2: 2D ripening without flow, periodic, 400 disks R ~ U[6, 14], W = 3."""
    p = _base(n, n, 1, W=3.0)
    rng = rng_for(rng_index)
    drops = place_droplets((1, n, n), ndrops, 6.0, 14.0, p["W"], rng)
    phi0 = droplet_field((1, n, n), drops, p["W"])
    mu = rng.normal(0.0, 1e-3, (2, 1, n, n))
    return Workload(f"ostwald_2d_{n}_{precision}", p, precision, 20000, phi0, mu[0], mu[1], drops=drops)


def sediment_3d(n=256, ndrops=64, rmin=10.0, rmax=18.0, precision="fp32", rng_index=2, nz=None, ny=None,
                phi_eq=None):
    """C3: 3D droplets sedimenting between walls at z = 0, n - 1, D3Q19 + 3 x D3Q7.
    phi_eq: use the paper's initial condition (Section 4.2.1) instead of mu_0 = 0 with
    the closure: compositions stepped at phi = 1/2 for the inventory whose equilibrium
    phase fraction is phi_eq (a supersaturated matrix when phi_eq exceeds the droplets'
    fraction), mu_0 = 0."""
    nz = nz or n
    ny = ny or n
    p = _base(n, ny, nz, fluid="D3Q19", bc=("periodic", "periodic", "walls"), drho=0.5,
              g=(0.0, 0.0, -1e-5), sigma=1e-4, nu=(0.1, 0.05))
    rng = rng_for(rng_index)
    drops = place_droplets((nz, ny, n), ndrops, rmin, rmax, p["W"], rng, wall_axes=(2,))
    phi0 = droplet_field((nz, ny, n), drops, p["W"], wall_axes=(2,))
    z = np.zeros((nz, ny, n))
    c0 = None
    if phi_eq is not None:
        c_eq = p["c_eq"]
        cg = tuple(c_eq[0][a] + phi_eq * (c_eq[1][a] - c_eq[0][a]) for a in range(2))
        c0, _ = stepped_composition(phi0, c_eq, cg)
    return Workload(f"sediment_3d_{n}_{precision}", p, precision, 10000, phi0, z, z.copy(), drops=drops, c0=c0)


def single_drop_2d(n=512, R=40.0, centre=None, precision="fp32"):
    """C4: one 2D drop sedimenting between walls at y = 0, n - 1, D2Q9 + 3 x D2Q5."""
    p = _base(n, n, 1, fluid="D2Q9", bc=("periodic", "walls", "periodic"), drho=0.5,
              g=(0.0, -1e-5, 0.0), sigma=1e-4, nu=(0.1, 0.05))
    c = centre or (n / 2, 0.75 * n, 0.0)
    phi0 = droplet_field((1, n, n), [(c, R)], p["W"], wall_axes=(1,))
    z = np.zeros((1, n, n))
    return Workload(f"single_drop_2d_{n}_{precision}", p, precision, 4096, phi0, z, z.copy())


def spinodal_3d(n=512, precision="bf16", rng_index=4):
    """C5: periodic box, phi_0 = 1/2 + U(-0.05, 0.05) per node, mu_0 = 0 (mean composition
    (0.4, 0.2), the tie-line midpoint), gravity with the mean subtracted."""
    p = _base(n, n, n, fluid="D3Q19", drho=0.5, g=(0.0, 0.0, -5e-6), sigma=1e-4, nu=(0.1, 0.05),
              gravity_mean_subtract=True)
    rng = rng_for(rng_index)
    phi0 = 0.5 + rng.uniform(-0.05, 0.05, (n, n, n))
    z = np.zeros((n, n, n))
    return Workload(f"spinodal_3d_{n}_{precision}", p, precision, 50000, phi0, z, z.copy())


# the paper's 2D ripening run (Table tab:Parameters_Ostwald-Ripening) in lattice units
OSTWALD_PAPER_DX = 4.882e-4
OSTWALD_PAPER_DT = 2.5e-8


def ostwald_paper_2d(n=4096, precision="fp32", rng_index=5):
    """E2 of the paper in lattice units, with the paper's discretisation (D2Q9 for every
    equation) and initial condition (Section 4.2.1).  Mobilities M dt / dx^2 from the
    table (collision rates 0.8776, 0.8146, 0.7517), W = 3, lambda = 155.95, tie line
    (0.3, 0.3) - (0.4, 0.4); droplet areas U[S_avg - dS, S_avg + dS] / dx^2 placed to the
    phase fraction 0.08; compositions stepped at phi = 1/2 for the inventory (0.31, 0.31)
    with mu_0 = 0.  n = 4096 is the paper's box; smaller n keep dx (a crop)."""
    k = OSTWALD_PAPER_DT / OSTWALD_PAPER_DX ** 2
    c_eq = ((0.3, 0.3), (0.4, 0.4))
    p = _base(n, n, 1, W=3.0, lam=155.95, M_phi=1.2 * k, M_A=(1.0 * k, 1.0 * k), M_B=(0.8 * k, 0.8 * k),
              c_eq=c_eq, scalar="D2Q9")
    rng = rng_for(rng_index)
    a2 = OSTWALD_PAPER_DX ** 2
    drops = place_droplets_by_fraction((1, n, n), 0.08, (1.02e-4 - 0.957e-4) / a2, (1.02e-4 + 0.957e-4) / a2,
                                       p["W"], rng)
    phi0 = droplet_field((1, n, n), drops, p["W"])
    c0, info = stepped_composition(phi0, c_eq, (0.31, 0.31))
    z = np.zeros((1, n, n))
    return Workload(f"ostwald_paper_2d_{n}_{precision}", p, precision, 20000, phi0, z, z.copy(), drops=drops,
                    c0=c0, note=f"{len(drops)} droplets, phase fraction {info['phase_fraction']:.4f}, "
                                f"delta {info['delta']:.5f}")


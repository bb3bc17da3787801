"""CPU pins of the paper's initial-condition recipe (Section 4.2.1) in inputs.py.

- Eq. phi_glob_eq with the printed ripening inventory: c_g = (0.31, 0.31) on the tie
  line (0.3, 0.3) - (0.4, 0.4) gives Phi_eq = 0.1; Eq. Delta-1 with the printed
  Phi = 0.08 gives delta = 0.02 / 0.92.
- Eq. Global_Compos (the inventory balance): the stepped compositions of Eq.
  Compos_Init have mean c_g exactly, whatever the droplet field.
- The placement of Fig. initialization_flowchart: every accepted droplet keeps the
  clearances of the caption, and the accepted volume just reaches the target.
- The stored oracle run from a supersaturated start (tests/golden/ripening64_oracle.npz):
  its droplets survive and grow.
"""

import math

import numpy as np
import pytest

from paper_2409_03401_amd import inputs

C_EQ = ((0.3, 0.3), (0.4, 0.4))


def test_lever_rule_and_offset_printed_values():
    phi_eq = inputs.lever_rule_fraction((0.31, 0.31), C_EQ[0], C_EQ[1])
    assert abs(phi_eq - 0.1) < 1e-14
    assert abs(inputs.supersaturation_offset(0.1, 0.08) - 0.02 / 0.92) < 1e-15
    # Phi = Phi_eq: no offset; Phi = 0: the whole inventory in the matrix
    assert inputs.supersaturation_offset(0.1, 0.1) == 0.0
    assert abs(inputs.supersaturation_offset(0.1, 0.0) - 0.1) < 1e-15


@pytest.mark.parametrize("shape,seed", [((1, 96, 128), 0), ((24, 20, 30), 1)])
def test_stepped_composition_inventory(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    vol = (8.0, 80.0) if nz == 1 else (30.0, 200.0)
    drops = inputs.place_droplets_by_fraction(shape, 0.06, vol[0], vol[1], 3.0, rng, max_tries=20000)
    phi = inputs.droplet_field(shape, drops, 3.0)
    cg = (0.31, 0.31)
    (cA, cB), info = inputs.stepped_composition(phi, C_EQ, cg)
    # inventory balance, Eq. Global_Compos
    assert abs(cA.mean() - cg[0]) < 1e-14 and abs(cB.mean() - cg[1]) < 1e-14
    inside = phi >= 0.5
    assert np.all(cA[inside] == 0.4) and np.all(cB[inside] == 0.4)
    # the matrix is supersaturated along the tie line (delta > 0 when Phi < Phi_eq)
    assert info["phase_fraction"] < info["phi_eq"] and info["delta"] > 0
    m = cA[~inside]
    assert np.all(m == m[0]) and 0.3 < m[0] < 0.4
    assert abs((m[0] - 0.3) / 0.1 - info["delta"]) < 1e-12


@pytest.mark.parametrize("shape", [(1, 300, 256), (40, 36, 48)])
def test_flowchart_placement_rules(shape):
    rng = np.random.default_rng(7)
    nz, ny, nx = shape
    two = nz == 1
    vmin, vmax = (30.0, 400.0) if two else (30.0, 150.0)
    W, s = 3.0, (0.07 if two else 0.03)
    drops = inputs.place_droplets_by_fraction(shape, s, vmin, vmax, W, rng)
    ndim = 2 if two else 3
    rad = (lambda V: math.sqrt(V / math.pi)) if two else (lambda V: (3 * V / (4 * math.pi)) ** (1 / 3))
    vol = (lambda R: math.pi * R * R) if two else (lambda R: 4 / 3 * math.pi * R ** 3)
    clear = rad(vmax) + W / 2
    dims = (nx, ny, nz)[:ndim]
    C = np.array([d[0][:ndim] for d in drops])
    for (c, R) in drops:
        assert rad(vmin) - 1e-9 <= R <= rad(vmax) + 1e-9
        for a in range(ndim):
            assert clear <= c[a] <= dims[a] - clear
    d2 = np.sum((C[:, None, :] - C[None, :, :]) ** 2, axis=-1) + np.eye(len(C)) * 1e30
    assert d2.min() >= (2 * clear) ** 2
    V = [vol(R) for _, R in drops]
    target = s * np.prod(dims)
    assert sum(V) >= target and sum(V) - V[-1] < target


def test_paper_ripening_workload_recipe():
    """The lattice-unit workload of Table tab:Parameters_Ostwald-Ripening: collision
    rates of the caption, phase fraction near 0.08, mean composition (0.31, 0.31)."""
    w = inputs.ostwald_paper_2d(n=512)
    p = w.params
    for D, printed in ((p["M_phi"], 0.8776), (p["M_A"][0], 0.8146), (p["M_B"][0], 0.7517)):
        assert 0.0 <= D / (1 / 3) + 0.5 - printed < 1e-4   # tau + 1/2, printed to four decimals
    assert p["scalar"] == "D2Q9"
    assert abs(w.c0[0].mean() - 0.31) < 1e-14 and abs(w.c0[1].mean() - 0.31) < 1e-14
    assert 0.07 < float((w.phi0 >= 0.5).mean()) < 0.09
    assert np.all(w.muA0 == 0) and np.all(w.muB0 == 0)


def test_stored_supersaturated_run_grows_its_droplets():
    """The oracle run stored for the long-horizon GPU test: droplets present at every
    stored step, no non-finite node, and a mean radius that grows out of the
    supersaturated matrix (later steps above the first)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ripening64_oracle.npz")
    g = np.load(path)
    names = ("sum_cA", "sum_cB", "sum_phi", "kinetic_energy", "max_u", "interface_measure", "free_energy",
             "nan_count", "droplets", "mean_radius")
    steps = [int(s) for s in g["steps"] if f"diag_{int(s)}" in g]
    assert steps
    d = [dict(zip(names, g[f"diag_{s}"])) for s in steps]
    assert all(x["droplets"] > 0 and x["nan_count"] == 0 for x in d)
    assert all(x["mean_radius"] > d[0]["mean_radius"] for x in d[1:])

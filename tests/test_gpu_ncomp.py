"""A third independent composition on the GPU (N components, the conclusion's
extension with the quadratic free energies of Eq. Taylor), against the FP64 oracle
(oracle/lbm.py with three compositions) on the same seeded inputs.

Bars as for the ternary fluid: FP64 populations within 1e-12 and diagnostics within
1e-11; FP32 relative L2 within 1e-5 on phi, the compositions and the populations;
16-bit storage within 1e-3 on the compositions and 1e-2 on phi.  Structural checks:
an absent third composition reproduces the ternary kernels, relabelling A and C
permutes the run, and every composition is conserved.
"""

import functools

import numpy as np
import pytest

from helpers import gpu_config, max_abs, rel_l2
from oracle import lbm as olbm
from paper_2409_03401_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# equilibrium compositions (A, B, C) per phase and the mobilities of C
C_EQ3 = ((0.2, 0.1, 0.15), (0.6, 0.3, 0.05))
M_C = (0.12, 0.07)
NAMES3 = ("phi", "cA", "cB", "cC", "muA", "muB", "muC", "p", "ux", "uy", "uz")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _drops(shape, n, rmin, rmax, W, seed, wall_axes=()):
    rng = np.random.default_rng(seed)
    drops = inputs.place_droplets(shape, n, rmin, rmax, W, rng, wall_axes=wall_axes)
    phi = inputs.droplet_field(shape, drops, W, wall_axes=wall_axes)
    mu = rng.normal(0.0, 5e-3, (3,) + shape)
    return phi, mu[0], mu[1], mu[2]


@functools.lru_cache(maxsize=None)
def case(name):
    """(common parameters, phi0, muA0, muB0, muC0, steps)"""
    flow2 = dict(fluid="D2Q9", drho=0.5, g=(0.0, -1e-4, 0.0), sigma=1e-3, nu=(0.1, 0.05))
    flow3 = dict(fluid="D3Q19", drho=0.5, g=(0.0, 0.0, -1e-4), sigma=1e-3, nu=(0.1, 0.05))
    common = dict(c_eq=C_EQ3, M_A=(0.1, 0.08), M_B=(0.09, 0.11))
    if name == "2d_noflow":
        p = inputs._base(75, 41, 1, W=3.0, **common)
        return (p, *_drops((1, 41, 75), 5, 3.0, 7.0, 3.0, 81), 40)
    if name == "2d_flow_walls":
        p = inputs._base(66, 48, 1, W=4.0, bc=("periodic", "walls", "periodic"), **common, **flow2)
        return (p, *_drops((1, 48, 66), 3, 4.0, 8.0, 4.0, 82, (1,)), 40)
    if name == "3d_flow_walls":
        p = inputs._base(21, 18, 20, W=4.0, bc=("periodic", "periodic", "walls"), **common, **flow3)
        return (p, *_drops((20, 18, 21), 1, 4.0, 5.0, 4.0, 83, (2,)), 12)
    if name == "3d_noflow_xy_walls":
        # x and y walls (the fix-up kernel), ragged tiles (70 = 64 + 6, 13 = 3 x 4 + 1)
        p = inputs._base(70, 13, 17, W=3.0, bc=("walls", "walls", "periodic"), **common)
        return (p, *_drops((17, 13, 70), 2, 3.0, 3.5, 3.0, 84, (0, 1)), 10)
    raise KeyError(name)


CASES = ["2d_noflow", "2d_flow_walls", "3d_flow_walls", "3d_noflow_xy_walls"]


def _oracle_params(p):
    return olbm.Params(**dict(p, M_x=(M_C,)))


@functools.lru_cache(maxsize=None)
def oracle_case(name):
    p, phi0, muA0, muB0, muC0, steps = case(name)
    prm = _oracle_params(p)
    st = olbm.run(olbm.init(phi0, muA0, muB0, prm, mu_x0=(muC0,)), prm, steps)
    m = olbm.moments(st, prm)
    mom = {k: np.asarray(m[k]) for k in NAMES3}
    parts = ([st.f] if st.f is not None else []) + [st.g, st.hA, st.hB, *st.hx]
    return mom, np.concatenate(parts, axis=0), olbm.diagnostics(st, prm)


def _sim(p, precision, phi0, muA0, muB0, muC0, c_eq=C_EQ3, m_c=M_C):
    from paper_2409_03401_amd.lbm import Simulation
    return Simulation(gpu_config(dict(p, c_eq=c_eq), precision, M_C=m_c), phi0, muA0, muB0, mu_x0=(muC0,))


def _gpu(name, precision):
    p, phi0, muA0, muB0, muC0, steps = case(name)
    print(f"[three compositions] {name} shape={phi0.shape} {precision} steps={steps}", flush=True)
    sim = _sim(p, precision, phi0, muA0, muB0, muC0)
    sim.step(steps)
    mom = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    return mom, sim.populations().cpu().numpy(), sim.diagnostics()


@pytest.mark.parametrize("name", CASES)
def test_nc3_parity_fp64(name):
    _require_gpu()
    mom, pops, diag = _gpu(name, "fp64")
    ora_m, ora_p, ora_d = oracle_case(name)
    assert set(mom) == set(NAMES3)
    err = max_abs(pops, ora_p)
    assert err <= 1e-12, err
    for k in NAMES3:
        assert max_abs(mom[k], ora_m[k]) <= 1e-12 * max(1.0, np.abs(ora_m[k]).max()), k
    for k in ("sum_cA", "sum_cB", "sum_cC", "sum_phi", "free_energy", "kinetic_energy", "interface_measure"):
        assert abs(diag[k] - ora_d[k]) <= 1e-11 * max(1.0, abs(ora_d[k])), (k, diag[k], ora_d[k])
    assert abs(diag["max_u"] - ora_d["max_u"]) <= 1e-12
    assert diag["nan_count"] == 0 and diag["droplets"] == ora_d["droplets"]


@pytest.mark.parametrize("name", CASES)
def test_nc3_parity_fp32(name):
    _require_gpu()
    mom, pops, _ = _gpu(name, "fp32")
    ora_m, ora_p, _ = oracle_case(name)
    errs = {k: rel_l2(mom[k], ora_m[k]) for k in ("phi", "cA", "cB", "cC")}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    assert rel_l2(pops, ora_p) <= 1e-5


@pytest.mark.parametrize("name", ["2d_flow_walls", "3d_flow_walls", "3d_noflow_xy_walls"])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_nc3_parity_16bit(name, prec):
    """16-bit storage (FP32 rest populations and arithmetic; h^C takes reference 0 and,
    in FP16, its own shift)."""
    _require_gpu()
    mom, _, diag = _gpu(name, prec)
    ora_m, _, ora_d = oracle_case(name)
    errs = {k: rel_l2(mom[k], ora_m[k]) for k in ("phi", "cA", "cB", "cC")}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k in ("cA", "cB", "cC"):
        assert errs[k] <= 1e-3, (k, errs[k])
    assert errs["phi"] <= 1e-2
    # the residue feedback keeps each composition's total to FP32 rounding
    for k in ("sum_cA", "sum_cB", "sum_cC"):
        assert abs(diag[k] - ora_d[k]) <= 1e-5 * abs(ora_d[k]), (k, diag[k], ora_d[k])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_nc3_absent_component_reproduces_ternary(prec):
    """c^C_eq = 0 in both phases and mu^C_0 = 0: h^C stays zero and every other field
    follows the ternary kernels."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation
    p, phi0, muA0, muB0, _, steps = case("2d_flow_walls")
    ternary = dict(p, c_eq=tuple(c[:2] for c in C_EQ3))
    absent = tuple(c[:2] + (0.0,) for c in C_EQ3)
    a = Simulation(gpu_config(ternary, prec), phi0, muA0, muB0)
    b = _sim(p, prec, phi0, muA0, muB0, np.zeros_like(muA0), c_eq=absent)
    a.step(steps)
    b.step(steps)
    pa, pb = a.populations(), b.populations()
    n2 = pa.shape[0]
    tol = 1e-14 if prec == "fp64" else 1e-6
    assert (pa - pb[:n2]).abs().max().item() <= tol
    assert pb[n2:].abs().max().item() == 0.0
    ma, mb = a.moments(), b.moments()
    for k in ("phi", "cA", "cB", "muA", "muB", "ux", "uy"):
        assert (ma[k] - mb[k]).abs().max().item() <= tol * max(1.0, ma[k].abs().max().item()), k
    assert mb["cC"].abs().max().item() == 0.0 and mb["muC"].abs().max().item() == 0.0
    da, db = a.diagnostics(), b.diagnostics()
    assert db["sum_cC"] == 0.0 and "sum_cC" not in da
    assert abs(da["free_energy"] - db["free_energy"]) <= tol * abs(da["free_energy"])


def test_nc3_relabelling_permutes_the_run():
    """Swapping the labels A and C (equilibria, mobilities, initial potentials) swaps
    their fields and leaves phi and the flow unchanged (FP64, up to the order of the
    sum in Delta omega)."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation
    p, phi0, muA0, muB0, muC0, steps = case("2d_flow_walls")
    a = _sim(p, "fp64", phi0, muA0, muB0, muC0)
    swapped = tuple((c[2], c[1], c[0]) for c in C_EQ3)
    q = dict(p, M_A=M_C)
    b = Simulation(gpu_config(dict(q, c_eq=swapped), "fp64", M_C=p["M_A"]), phi0, muC0, muB0, mu_x0=(muA0,))
    a.step(steps)
    b.step(steps)
    ma, mb = a.moments(), b.moments()
    for ka, kb in (("phi", "phi"), ("cA", "cC"), ("cC", "cA"), ("cB", "cB"), ("muA", "muC"), ("ux", "ux"),
                   ("uy", "uy"), ("p", "p")):
        assert (ma[ka] - mb[kb]).abs().max().item() <= 1e-13 * max(1.0, ma[ka].abs().max().item()), ka


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_nc3_conserves_every_composition(prec):
    """Closed box (walls in y, periodic x) with flow: sum c^A, c^B, c^C stay at their
    initial values over 300 steps, to FP64 rounding, and to FP32 rounding of the rest
    populations with 16-bit storage."""
    _require_gpu()
    p, phi0, muA0, muB0, muC0, _ = case("2d_flow_walls")
    sim = _sim(p, prec, phi0, muA0, muB0, muC0)
    series = sim.run_series(300, 100)
    assert set(series) >= {"sum_cA", "sum_cB", "sum_cC"}
    tol = 1e-12 if prec == "fp64" else 2e-6
    for k in ("sum_cA", "sum_cB", "sum_cC"):
        s = series[k]
        assert np.all(np.abs(s - s[0]) <= tol * abs(s[0])), (k, s)
    assert np.all(series["nan_count"] == 0)


def test_nc3_population_round_trip_and_errors():
    """get / set populations over Q_f + 4 Q_s slots (FP64: bitwise); the third
    composition's moments are refused on a ternary run; no adjoint."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import LBM_EINVAL, LBM_EUNSUPPORTED, LBMError, Simulation, adjoint_bytes
    p, phi0, muA0, muB0, muC0, _ = case("2d_flow_walls")
    sim = _sim(p, "fp64", phi0, muA0, muB0, muC0)
    sim.step(3)
    pops = sim.populations()
    assert pops.shape[0] == 9 + 4 * 5
    ref = sim.moments()
    sim.set_populations(pops)
    assert torch.equal(sim.populations(), pops)
    again = sim.moments()
    for k in ref:
        assert torch.equal(ref[k], again[k]), k
    ternary = Simulation(gpu_config(dict(p, c_eq=tuple(c[:2] for c in C_EQ3)), "fp64"), phi0, muA0, muB0)
    with pytest.raises(LBMError) as e:
        ternary.moments(["cC"])
    assert e.value.code == LBM_EINVAL
    cfg = gpu_config(dict(p, c_eq=C_EQ3), "fp64", M_C=M_C)
    work = torch.zeros(adjoint_bytes(cfg), dtype=torch.uint8, device="cuda")
    with pytest.raises(LBMError) as e:
        sim.adjoint_seed(sim.save(), torch.zeros(cfg.nodes, dtype=torch.float64, device="cuda"), work)
    assert e.value.code == LBM_EUNSUPPORTED

"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Both sides start from the same seeded inputs (paper_2409_03401_amd.inputs) and run
the same number of steps; fields and populations are compared element by element.

Bars:
  fp64 storage  : populations and fields agree to 1e-12 (rounding order only)
  fp32 storage  : relative L2 error <= 1e-5 on c^A, c^B and phi; potentials, pressure
                  and velocity within 1e-5 of the field's own scale
  fp16 / bf16   : relative L2 error <= 1e-3 on c^A, c^B (stated per field otherwise)
"""

import functools
import math

import numpy as np
import pytest

from helpers import (MOMENT_NAMES, field_errors, gpu_config, max_abs, oracle_moments, oracle_populations,
                     oracle_run, rel_l2)
from paper_2409_03401_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(p, precision, phi0, muA0, muB0):
    from paper_2409_03401_amd.lbm import Simulation
    return Simulation(gpu_config(p, precision), phi0, muA0, muB0)


def _gpu_run(p, precision, phi0, muA0, muB0, steps):
    sim = _sim(p, precision, phi0, muA0, muB0)
    sim.step(steps)
    mom = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    pops = sim.populations().cpu().numpy()
    diag = sim.diagnostics()
    return sim, mom, pops, diag


# ----------------------------------------------------------------------------------------
# small cases the oracle finishes in seconds; 3D sizes are ragged with respect to the
# 64 x 4 work-group tiles (2D cases wider than one 256-node row segment are in
# test_gpu_2d_tiles.py)

def _drops2d(shape, n, rmin, rmax, W, seed, wall_axes=()):
    rng = np.random.default_rng(seed)
    drops = inputs.place_droplets(shape, n, rmin, rmax, W, rng, wall_axes=wall_axes)
    return inputs.droplet_field(shape, drops, W, wall_axes=wall_axes), rng


@functools.lru_cache(maxsize=None)
def case(name):
    """Returns (params, phi0, muA0, muB0, steps) for a named small case."""
    if name == "c1a_couple_fp64":
        w = inputs.diffusion_couple_tie()
        return w.params, w.phi0, w.muA0, w.muB0, 400
    if name == "c1b_couple_paper_fp64":
        w = inputs.diffusion_couple_paper()
        return w.params, w.phi0, w.muA0, w.muB0, 400
    if name == "noflow_2d":
        p = inputs._base(150, 77, 1, W=3.0)
        phi0, rng = _drops2d((1, 77, 150), 12, 5.0, 10.0, 3.0, 11)
        mu = rng.normal(0.0, 1e-3, (2, 1, 77, 150))
        return p, phi0, mu[0], mu[1], 120
    if name == "flow_2d_walls":
        p = inputs._base(130, 90, 1, fluid="D2Q9", bc=("periodic", "walls", "periodic"), drho=0.5,
                         g=(0.0, -1e-4, 0.0), sigma=1e-3, nu=(0.1, 0.05))
        phi0, rng = _drops2d((1, 90, 130), 4, 8.0, 14.0, 4.0, 12, wall_axes=(1,))
        mu = rng.normal(0.0, 5e-4, (2, 1, 90, 130))
        return p, phi0, mu[0], mu[1], 150
    if name == "noflow_3d":
        p = inputs._base(45, 30, 21, W=3.0, bc=("periodic", "walls", "periodic"))
        phi0, rng = _drops2d((21, 30, 45), 4, 4.0, 7.0, 3.0, 13, wall_axes=(1,))
        mu = rng.normal(0.0, 1e-3, (2, 21, 30, 45))
        return p, phi0, mu[0], mu[1], 40
    if name == "flow_3d_walls":
        p = inputs._base(70, 44, 38, fluid="D3Q19", bc=("periodic", "periodic", "walls"), drho=0.5,
                         g=(0.0, 0.0, -1e-4), sigma=1e-3, nu=(0.1, 0.05))
        phi0, rng = _drops2d((38, 44, 70), 4, 6.0, 10.0, 4.0, 14, wall_axes=(2,))
        mu = rng.normal(0.0, 5e-4, (2, 38, 44, 70))
        return p, phi0, mu[0], mu[1], 40
    if name == "flow_3d_periodic_mean":
        p = inputs._base(36, 33, 35, fluid="D3Q19", drho=0.5, g=(0.0, 0.0, -1e-4), sigma=1e-3,
                         nu=(0.1, 0.05), gravity_mean_subtract=True)
        rng = np.random.default_rng(15)
        phi0 = 0.5 + rng.uniform(-0.05, 0.05, (35, 33, 36))
        z = np.zeros_like(phi0)
        return p, phi0, z, z.copy(), 30
    if name == "flow_3d_allwalls_fp64":
        p = inputs._base(19, 17, 15, fluid="D3Q19", bc=("walls", "walls", "walls"), drho=0.5,
                         g=(1e-4, -2e-4, -1e-4), sigma=1e-3, nu=(0.1, 0.05))
        phi0, rng = _drops2d((15, 17, 19), 1, 5.0, 5.5, 4.0, 16, wall_axes=(0, 1, 2))
        mu = rng.normal(0.0, 1e-3, (2, 15, 17, 19))
        return p, phi0, mu[0], mu[1], 25
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def oracle_case(name):
    p, phi0, muA0, muB0, steps = case(name)
    prm, st = oracle_run(p, phi0, muA0, muB0, steps)
    from oracle import lbm as olbm
    return oracle_moments(prm, st), oracle_populations(prm, st), olbm.diagnostics(st, prm)


def _scale(ora, k):
    if k in ("muA", "muB"):
        return max(np.abs(ora["cA"]).max(), np.abs(ora["cB"]).max())
    if k in ("ux", "uy", "uz"):
        return max(np.abs(ora["ux"]).max(), np.abs(ora["uy"]).max(), np.abs(ora["uz"]).max(), 1e-300)
    if k == "p":
        return max(np.abs(ora["p"]).max(), 1e-300)
    return max(np.abs(ora[k]).max(), 1e-300)


FP64_CASES = ["c1a_couple_fp64", "c1b_couple_paper_fp64", "noflow_2d", "flow_2d_walls", "flow_3d_allwalls_fp64"]
FP32_CASES = ["noflow_2d", "flow_2d_walls", "noflow_3d", "flow_3d_walls", "flow_3d_periodic_mean"]


@pytest.mark.parametrize("name", FP64_CASES)
def test_parity_fp64(name):
    _require_gpu()
    p, phi0, muA0, muB0, steps = case(name)
    print(f"[parity fp64] {name} shape={phi0.shape} steps={steps}", flush=True)
    _, mom, pops, diag = _gpu_run(p, "fp64", phi0, muA0, muB0, steps)
    ora_m, ora_p, ora_d = oracle_case(name)
    err_p = max_abs(pops, ora_p)
    assert err_p <= 1e-12, err_p
    for k in MOMENT_NAMES:
        assert max_abs(mom[k], ora_m[k]) <= 1e-12 * max(1.0, _scale(ora_m, k)), k
    for k in ("sum_cA", "sum_cB", "sum_phi", "interface_measure", "free_energy", "mean_radius"):
        assert abs(diag[k] - ora_d[k]) <= 1e-11 * max(1.0, abs(ora_d[k])), k
    # the flow diagnostics are small numbers: relative bars
    for k in ("kinetic_energy", "max_u"):
        assert abs(diag[k] - ora_d[k]) <= 1e-11 * abs(ora_d[k]) + 1e-30, (k, diag[k], ora_d[k])
    assert diag["nan_count"] == 0
    assert diag["droplets"] == ora_d["droplets"]


@pytest.mark.parametrize("name", FP32_CASES)
def test_parity_fp32(name):
    _require_gpu()
    p, phi0, muA0, muB0, steps = case(name)
    print(f"[parity fp32] {name} shape={phi0.shape} steps={steps}", flush=True)
    _, mom, pops, diag = _gpu_run(p, "fp32", phi0, muA0, muB0, steps)
    ora_m, ora_p, ora_d = oracle_case(name)
    errs = field_errors(mom, ora_m)
    print({k: (f"{a:.2e}", f"{b:.2e}") for k, (a, b) in errs.items()}, flush=True)
    for k in ("phi", "cA", "cB"):
        assert errs[k][0] <= 1e-5, (k, errs[k])
    for k in ("muA", "muB", "p", "ux", "uy", "uz"):
        assert errs[k][1] <= 1e-5 * _scale(ora_m, k) + 1e-12, (k, errs[k])
    assert rel_l2(pops, ora_p) <= 1e-5
    for k in ("sum_cA", "sum_cB"):
        assert abs(diag[k] - ora_d[k]) <= 1e-5 * abs(ora_d[k]), k


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("name", ["noflow_2d", "flow_2d_walls", "flow_3d_walls"])
def test_parity_16bit(name, prec):
    _require_gpu()
    p, phi0, muA0, muB0, steps = case(name)
    print(f"[parity {prec}] {name} shape={phi0.shape} steps={steps}", flush=True)
    _, mom, pops, diag = _gpu_run(p, prec, phi0, muA0, muB0, steps)
    ora_m, _, ora_d = oracle_case(name)
    errs = field_errors(mom, ora_m)
    print({k: (f"{a:.2e}", f"{b:.2e}") for k, (a, b) in errs.items()}, flush=True)
    for k in ("cA", "cB"):
        assert errs[k][0] <= 1e-3, (k, errs[k])
    assert errs["phi"][0] <= 1e-2
    assert diag["nan_count"] == 0


def test_mass_conservation_fp64_long():
    """C1a for its full 2000 steps: per-component mass conserved to 1e-12."""
    _require_gpu()
    w = inputs.diffusion_couple_tie()
    sim = _sim(w.params, "fp64", w.phi0, w.muA0, w.muB0)
    d0 = sim.diagnostics()
    sim.step(w.steps)
    d1 = sim.diagnostics()
    for k in ("sum_cA", "sum_cB"):
        assert abs(d1[k] - d0[k]) <= 1e-12 * abs(d0[k]), k


def test_save_restore_and_determinism():
    _require_gpu()
    p, phi0, muA0, muB0, _ = case("flow_3d_periodic_mean")
    a = _sim(p, "fp32", phi0, muA0, muB0)
    a.step(10)
    ck = a.save()
    a.step(10)
    ref = a.populations().clone()
    b = _sim(p, "fp32", phi0, muA0, muB0)
    b.step(3)
    b.restore(ck)
    b.step(10)
    assert torch.equal(b.populations(), ref)
    c = _sim(p, "fp32", phi0, muA0, muB0)
    c.step(20)
    assert torch.equal(c.populations(), ref)

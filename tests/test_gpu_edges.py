"""Degenerate and ragged shapes on the GPU against the FP64 oracle (FP64 storage,
populations within 1e-12): axes of one node (periodic onto itself), axes of two nodes
between walls, sizes one past the 64 x 4 work-group tile, planar 3D runs, and zero
steps.  Every case has flow, capillary and buoyancy forces, and noise in mu."""

import functools

import numpy as np
import pytest

from helpers import MOMENT_NAMES, gpu_config, max_abs, oracle_moments, oracle_params, oracle_populations
from oracle import lbm as olbm
from paper_2409_03401_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _fields(shape, seed):
    """A smooth phase field with an interface through the box and noise in mu."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = 0.3 * x + 0.5 * y + 0.7 * z
    phi = 0.5 * (1.0 + np.tanh((s - s.mean()) / 2.0 + 0.3 * np.sin(0.9 * x + 0.4 * z)))
    mu = rng.normal(0.0, 1e-3, (2,) + shape)
    return phi, mu[0], mu[1]


FLOW3 = dict(fluid="D3Q19", drho=0.5, g=(1e-4, -2e-4, -1e-4), sigma=1e-3, nu=(0.1, 0.05))
FLOW2 = dict(fluid="D2Q9", drho=0.5, g=(1e-4, -2e-4, 0.0), sigma=1e-3, nu=(0.1, 0.05))

CASES = {
    # name: (grid nx, ny, nz, extra parameters, steps)
    "3d_tile_plus_one": ((65, 5, 3), dict(bc=("periodic", "periodic", "walls"), **FLOW3), 8),
    "3d_column_1x1": ((1, 1, 40), dict(bc=("periodic", "periodic", "walls"), **FLOW3), 10),
    "3d_planar_nz1": ((33, 20, 1), dict(bc=("walls", "periodic", "periodic"), **FLOW3), 10),
    "3d_all_walls_2x2x2": ((2, 2, 2), dict(bc=("walls", "walls", "walls"), **FLOW3), 10),
    "3d_walls_on_one_node_axis": ((17, 1, 9), dict(bc=("periodic", "walls", "walls"), **FLOW3), 8),
    "2d_walls_two_rows": ((70, 2, 1), dict(bc=("periodic", "walls", "periodic"), **FLOW2), 12),
    "2d_one_column": ((1, 50, 1), dict(bc=("periodic", "walls", "periodic"), **FLOW2), 12),
    "2d_segment_plus_one_noflow": ((257, 3, 1), dict(bc=("walls", "periodic", "periodic")), 12),
}


@functools.lru_cache(maxsize=None)
def case(name):
    (nx, ny, nz), extra, steps = CASES[name]
    scalar = "D3Q7" if extra.get("fluid") == "D3Q19" or (nz > 1) else "D2Q5"
    p = inputs._base(nx, ny, nz, W=3.0, **dict(extra, scalar=scalar))
    return (p, *_fields((nz, ny, nx), sum(map(ord, name))), steps)


@functools.lru_cache(maxsize=None)
def oracle_case(name):
    p, phi0, muA0, muB0, steps = case(name)
    prm = oracle_params(p)
    st = olbm.run(olbm.init(phi0, muA0, muB0, prm), prm, steps)
    return oracle_moments(prm, st), oracle_populations(prm, st)


@pytest.mark.parametrize("name", list(CASES))
def test_edge_case_parity_fp64(name):
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation
    p, phi0, muA0, muB0, steps = case(name)
    print(f"[edge] {name} grid=({p['nx']}, {p['ny']}, {p['nz']}) bc={p['bc']} steps={steps}", flush=True)
    sim = Simulation(gpu_config(p, "fp64"), phi0, muA0, muB0)
    sim.step(steps)
    pops = sim.populations().cpu().numpy()
    mom = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    ora_m, ora_p = oracle_case(name)
    assert max_abs(pops, ora_p) <= 1e-12
    for k in MOMENT_NAMES:
        assert max_abs(mom[k], ora_m[k]) <= 1e-12 * max(1.0, np.abs(ora_m[k]).max()), k


def test_zero_steps_is_the_initial_state():
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation
    p, phi0, muA0, muB0, _ = case("3d_tile_plus_one")
    sim = Simulation(gpu_config(p, "fp64"), phi0, muA0, muB0)
    before = sim.populations().clone()
    sim.step(0)
    assert torch.equal(sim.populations(), before) and sim.step_count == 0
    prm = oracle_params(p)
    assert max_abs(before.cpu().numpy(), oracle_populations(prm, olbm.init(phi0, muA0, muB0, prm))) <= 1e-14

"""The NaN count of lbm_diagnostics (nodes whose phi, c^A or c^B is not finite): a state
with non-finite populations planted at three nodes reports exactly those nodes, and
the count survives into the next step's state."""

import math

import numpy as np
import pytest

from helpers import gpu_config
from paper_2409_03401_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_nan_count(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03401_amd.lbm import Simulation
    nx, ny = 70, 40
    p = inputs._base(nx, ny, 1, fluid="D2Q9", bc=("periodic", "walls", "periodic"), drho=0.5,
                     g=(0.0, -1e-4, 0.0), sigma=1e-3, nu=(0.1, 0.05))
    phi0 = inputs.droplet_field((1, ny, nx), [((35.0, 20.0, 0.0), 8.0)], 4.0, wall_axes=(1,))
    z = np.zeros_like(phi0)
    sim = Simulation(gpu_config(p, prec), phi0, z, z)
    assert sim.diagnostics()["nan_count"] == 0
    pops = sim.populations().cpu().numpy()
    qf = 9
    # a NaN in g_0 at node 100 (phi), an inf in hA_0 at node 1234 (c^A), a NaN in hB_0 at node 2000 (c^B)
    pops[qf + 0].reshape(-1)[100] = math.nan
    pops[qf + 5].reshape(-1)[1234] = math.inf
    pops[qf + 10].reshape(-1)[2000] = math.nan
    sim.set_populations(pops)
    assert sim.diagnostics()["nan_count"] == 3
    sim.step(1)
    assert sim.diagnostics()["nan_count"] >= 3

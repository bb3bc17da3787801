"""The windowed oracle of test_gpu_fullsize.py reproduces the full-domain oracle
exactly at the window centre (CPU): the dependence radius argument behind the
full-size sampled parity tests."""

import numpy as np
import pytest

from helpers import MOMENT_NAMES, oracle_params
from oracle import lbm as olbm
from paper_2409_03401_amd import inputs

import test_gpu_fullsize as fs


def _full(w, steps):
    prm = oracle_params(w.params)
    st = olbm.run(olbm.init(w.phi0, w.muA0, w.muB0, prm), prm, steps)
    return {k: np.asarray(v) for k, v in olbm.moments(st, prm).items()}


CASES = {
    "drop_2d_walls": (lambda: inputs.single_drop_2d(n=48, R=9.0, centre=(20.0, 30.0, 0.0)), 2),
    "sediment_3d_walls": (lambda: inputs.sediment_3d(n=32, ndrops=2, rmin=5.0, rmax=7.0), 1),
    "spinodal_mean_subtract": (lambda: inputs.spinodal_3d(n=24), 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_window_matches_full_domain(name):
    build, steps = CASES[name]
    w = build()
    full = _full(w, steps)
    for c in fs.sample_nodes(w, count=6):
        ora, _ = fs.window_oracle(w, c, steps)
        for k in MOMENT_NAMES:
            assert abs(ora[k] - full[k][c]) <= 1e-13 * max(1.0, np.abs(full[k]).max()), (name, c, k)

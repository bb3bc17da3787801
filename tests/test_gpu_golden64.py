"""The 64^3 crop of the sediment workload against stored FP64 oracle values at 1000
and 10000 steps (tests/golden/sediment64_oracle.npz, written by
tests/golden/make_sediment64.py from the oracle alone).

Bars: relative L2 over the 4096 sampled nodes of the conserved fields c^A, c^B:
1e-5 with FP32 storage, 1e-3 with FP16/BF16 storage; per-component mass drift
relative to the oracle's totals below the same bars.  The other fields' errors are
printed (relative L2 and max-abs per field)."""

import os

import numpy as np
import pytest

from helpers import gpu_config
from paper_2409_03401_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sediment64_oracle.npz")
MOMENTS = ("phi", "cA", "cB", "muA", "muB", "p", "ux", "uy", "uz")
DIAG = ("sum_cA", "sum_cB", "sum_phi", "kinetic_energy", "max_u", "interface_measure", "free_energy", "nan_count")


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_sediment64_against_oracle(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_03401_amd.lbm import Simulation
    g = np.load(GOLDEN)
    idx = torch.tensor(g["sample_nodes"], device="cuda")
    w = inputs.sediment_3d(n=64, ndrops=4, rmin=10.0, rmax=14.0)
    sim = Simulation(gpu_config(w.params, prec), w.phi0, w.muA0, w.muB0)
    bar = 1e-5 if prec == "fp32" else 1e-3
    done = 0
    for steps in sorted(int(s) for s in g["steps"]):
        if f"cA_{steps}" not in g:
            continue
        sim.step(steps - done)
        done = steps
        mom = sim.moments()
        d = sim.diagnostics()
        od = dict(zip(DIAG, g[f"diag_{steps}"]))
        errs = {}
        for k in MOMENTS:
            gpu = mom[k].reshape(-1).index_select(0, idx).cpu().numpy()
            ora = g[f"{k}_{steps}"]
            errs[k] = (_rel_l2(gpu, ora), float(np.abs(gpu - ora).max()))
        print(f"[golden64 {prec} step {steps}] " + ", ".join(f"{k} {a:.2e}/{b:.2e}" for k, (a, b) in errs.items()),
              flush=True)
        print(f"  mass drift vs oracle: cA {abs(d['sum_cA'] - od['sum_cA']) / od['sum_cA']:.2e} "
              f"cB {abs(d['sum_cB'] - od['sum_cB']) / od['sum_cB']:.2e}", flush=True)
        assert d["nan_count"] == 0
        for k in ("cA", "cB"):
            assert errs[k][0] <= bar, (k, errs[k])
            assert abs(d[f"sum_{k}"] - od[f"sum_{k}"]) <= bar * abs(od[f"sum_{k}"])

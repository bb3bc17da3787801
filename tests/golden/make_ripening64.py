"""Writes tests/golden/ripening64_oracle.npz: the FP64 oracle on a 64^3 box of the
sedimentation recipe started from the paper's supersaturated initial condition
(Section 4.2.1, Eq. Compos_Init: compositions stepped at phi = 1/2 for the inventory
whose equilibrium phase fraction is 0.25, mu_0 = 0), D3Q19 + 3 x D3Q7, walls in z,
4 droplets R ~ U[10, 14] (a phase fraction of about 0.11, so the matrix is
supersaturated and the droplets grow while they sediment).  Stored at 1000, 4000 and
10000 steps: every moment at 4096 seeded sample nodes and the diagnostics (droplet
count included).  Calls only the oracle and the seeded input generators.

    python tests/golden/make_ripening64.py [--steps 1000 4000 10000]

Single-threaded numpy; about 0.12 s per step on one core.
"""

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbm as olbm  # noqa: E402
from paper_2409_03401_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ripening64_oracle.npz")
MOMENTS = ("phi", "cA", "cB", "muA", "muB", "p", "ux", "uy", "uz")
N_SAMPLES = 4096
PHI_EQ = 0.25


def workload():
    return inputs.sediment_3d(n=64, ndrops=4, rmin=10.0, rmax=14.0, phi_eq=PHI_EQ)


def sample_nodes(nodes):
    return np.sort(inputs.rng_for(51).choice(nodes, N_SAMPLES, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, nargs="+", default=[1000, 4000, 10000])
    args = ap.parse_args()
    w = workload()
    prm = olbm.Params(**w.params)
    st = olbm.init(w.phi0, w.muA0, w.muB0, prm, c0=w.c0)
    idx = sample_nodes(w.nodes)
    out = {"sample_nodes": idx, "steps": np.array(sorted(args.steps))}
    t0 = time.time()
    for target in sorted(args.steps):
        while st.step < target:
            st = olbm.step(st, prm)
            if st.step % 250 == 0:
                print(f"step {st.step} ({time.time() - t0:.0f} s)", flush=True)
        m = olbm.moments(st, prm)
        for k in MOMENTS:
            out[f"{k}_{target}"] = np.asarray(m[k]).reshape(-1)[idx]
        d = olbm.diagnostics(st, prm)
        out[f"diag_{target}"] = np.array([d[k] for k in olbm.DIAG_NAMES])
        np.savez(OUT, **out)
        print(f"wrote {OUT} through step {target}: droplets {d['droplets']}, <R> {d['mean_radius']:.3f}, "
              f"max|u| {d['max_u']:.3e}", flush=True)


if __name__ == "__main__":
    main()

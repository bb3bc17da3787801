"""Writes tests/golden/adjoint_crop4096_oracle.npz: reference derivatives of a loss of
the final phase field over a long run, for the end-to-end adjoint test.

Workload: the 64 x 64 crop of the sedimenting-drop case (inputs.single_drop_2d, its own
parameters: D2Q9 fluid, D2Q5 scalars, walls in y), T = 4096 steps.  Loss
L = sum_x (phi_T(x) - target(x))^2 with target = the oracle's phi_T when every mobility
(M_phi, M_A, M_B) is raised by 10 %.  Stored: the target, the loss, and the oracle's
complex-step derivatives (step 1e-30) through the whole run of L with respect to
  s  a common scale of the five mobilities (theta_j = s m_j, at s = 1),
  W  the interface width,
  v  the direction v in phi_0 (stored), v = N(0, 1) (|d phi_0 / dx| + 0.01), seed 400.
Calls only the oracle and the seeded input generators.

    python tests/golden/make_adjoint_crop4096.py

About 4 minutes on one core (complex FP64 numpy).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbm as olbm  # noqa: E402
from paper_2409_03401_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_crop4096_oracle.npz")
STEPS = 4096
H_CS = 1e-30


def workload():
    w = inputs.single_drop_2d(n=64, R=12.0, centre=(32.0, 40.0, 0.0))
    return w, dict(w.params)


def direction(phi0):
    rng = inputs.rng_for(400)
    return rng.standard_normal(phi0.shape) * (np.abs(np.gradient(phi0, axis=1)) + 0.01)


def final_phi(p, phi0, muA0, muB0):
    prm = olbm.Params(**p)
    st = olbm.run(olbm.init(phi0, muA0, muB0, prm), prm, STEPS)
    return np.asarray(olbm.moments(st, prm)["phi"])


def main():
    w, p = workload()
    muA0, muB0 = w.muA0, w.muB0
    t0 = time.time()
    q = dict(p, M_phi=1.1 * p["M_phi"], M_A=tuple(1.1 * m for m in p["M_A"]),
             M_B=tuple(1.1 * m for m in p["M_B"]))
    target = final_phi(q, w.phi0, muA0, muB0)
    print(f"target ({time.time() - t0:.0f} s)", flush=True)
    loss = float(np.sum((final_phi(p, w.phi0, muA0, muB0) - target) ** 2))
    print(f"loss {loss:.10e} ({time.time() - t0:.0f} s)", flush=True)

    def cs(pp, phi0):
        phi = final_phi(pp, phi0, muA0.astype(complex), muB0.astype(complex))
        return float(np.sum((phi - target) ** 2).imag / H_CS)

    ps = dict(p, M_phi=p["M_phi"] * (1 + 1j * H_CS), M_A=tuple(m * (1 + 1j * H_CS) for m in p["M_A"]),
              M_B=tuple(m * (1 + 1j * H_CS) for m in p["M_B"]))
    dL_ds = cs(ps, w.phi0 + 0j)
    print(f"dL/ds {dL_ds:.10e} ({time.time() - t0:.0f} s)", flush=True)
    dL_dW = cs(dict(p, W=p["W"] + 1j * H_CS), w.phi0 + 0j)
    print(f"dL/dW {dL_dW:.10e} ({time.time() - t0:.0f} s)", flush=True)
    v = direction(w.phi0)
    dL_dv = cs(p, w.phi0 + 1j * H_CS * v)
    print(f"dL/dphi0.v {dL_dv:.10e} ({time.time() - t0:.0f} s)", flush=True)
    np.savez(OUT, steps=np.array(STEPS), target=target, loss=np.array(loss), dL_ds=np.array(dL_ds),
             dL_dW=np.array(dL_dW), v=v, dL_dv=np.array(dL_dv))
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()

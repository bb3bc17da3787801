"""The discrete adjoint of the step on the paper's own lattices (D2Q9 / D3Q19 for g,
h^A, h^B), against complex-step derivatives of the FP64 oracle, with the bars of the
reduced-lattice adjoint tests: every column of J^T lambda (2D) or sampled columns
(3D) within 2e-6 (FP64), <lambda, J v> = <J^T lambda, v> within 1e-5 on a grid
spanning many adjoint work-groups, and the gradient of a phase-field loss through the
differentiable run in M_phi, W and a direction of phi_0."""

import numpy as np
import pytest

from helpers import gpu_config, oracle_params, oracle_populations
from oracle import lbm as olbm
from paper_2409_03401_amd import inputs
from test_gpu_adjoint import (H_CS, THETA_KEYS, _gpu_adjoint_step, _oracle_column, _oracle_step_pops,
                              _oracle_theta_jvp)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = {
    "d2q9_scalars_flow_walls_y": dict(nx=8, ny=6, fluid="D2Q9", scalar="D2Q9", bc=("periodic", "walls", "periodic"),
                                      W=3.0, lam=2.0, M_phi=0.12, M_A=(0.1, 0.07), M_B=(0.05, 0.09), drho=0.5,
                                      g=(2e-4, -1e-3, 0.0), sigma=0.02, nu=(0.1, 0.05)),
    "d3q19_scalars_flow_walls_z": dict(nx=4, ny=4, nz=5, fluid="D3Q19", scalar="D3Q19",
                                       bc=("periodic", "periodic", "walls"), W=2.5, lam=2.0, M_phi=0.1,
                                       M_A=(0.1, 0.07), M_B=(0.05, 0.09), drho=0.5, g=(1e-4, 2e-4, -1e-3),
                                       sigma=0.02, nu=(0.1, 0.05)),
}


def _case(name, seed):
    p = {**inputs._base(CASES[name]["nx"], CASES[name]["ny"], CASES[name].get("nz", 1)), **CASES[name]}
    prm = oracle_params(p)
    shape = prm.shape
    rng = inputs.rng_for(seed)
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    r = np.sqrt((xx - shape[2] / 2) ** 2 + (yy - shape[1] / 2) ** 2 + (zz - shape[0] / 2) ** 2 * (shape[0] > 1))
    phi0 = 0.5 * (1 + np.tanh((0.35 * min(shape[1:]) - r))) + 0.05 * rng.uniform(-1, 1, shape)
    muA0, muB0 = 0.01 * rng.standard_normal(shape), 0.01 * rng.standard_normal(shape)
    pops = oracle_populations(prm, olbm.run(olbm.init(phi0, muA0, muB0, prm), prm, 2))
    lam = rng.standard_normal(pops.shape).astype(np.float32).astype(np.float64)
    return p, pops, phi0, muA0, muB0, lam


@pytest.mark.parametrize("name,seed", [("d2q9_scalars_flow_walls_y", 300), ("d3q19_scalars_flow_walls_z", 301)])
def test_paper_lattice_adjoint_entrywise(name, seed):
    _require_gpu()
    p, pops, phi0, muA0, muB0, lam = _case(name, seed)
    print(f"[adjoint paper lattice] {name} pops {pops.shape}", flush=True)
    got, gth = _gpu_adjoint_step(p, "fp64", pops, phi0, muA0, muB0, lam)
    if pops.shape[1] > 1:
        nodes = pops[0].size
        pick = sorted({0, nodes - 1, nodes // 2} | set(inputs.rng_for(8).integers(0, nodes, 4).tolist()))
        cols = [s * nodes + i for s in range(pops.shape[0]) for i in pick]
    else:
        cols = list(range(pops.size))
    want = np.array([np.dot(lam.ravel(), _oracle_column(pops, p, j).ravel()) for j in cols])
    g = got.ravel()[cols]
    scale = np.max(np.abs(want))
    err = np.max(np.abs(g - want)) / scale
    print(f"  columns {len(want)}: max err / max |want| = {err:.3e}", flush=True)
    assert err < 2e-6
    for j in range(6):
        t = np.dot(lam.ravel(), _oracle_theta_jvp(pops, p, j).ravel())
        print(f"  d/d{THETA_KEYS[j]}: gpu {gth[j]:.10e} oracle {t:.10e}", flush=True)
        assert abs(gth[j] - t) <= 2e-6 * max(abs(t), 1e-3 * scale)


def test_paper_lattice_adjoint_dot_product():
    """A 2D grid spanning several work-groups with a ragged edge."""
    _require_gpu()
    p = {**inputs._base(150, 45, 1), **dict(fluid="D2Q9", scalar="D2Q9", bc=("periodic", "walls", "periodic"),
                                            W=4.0, lam=inputs.LAMBDA_TIE, M_phi=0.1, M_A=(0.1, 0.07),
                                            M_B=(0.05, 0.09), drho=0.5, g=(0.0, -1e-4, 0.0), sigma=0.01,
                                            nu=(0.1, 0.05))}
    prm = oracle_params(p)
    rng = inputs.rng_for(302)
    drops = inputs.place_droplets(prm.shape, 3, 5, 9, p["W"], rng, wall_axes=(1,))
    phi0 = inputs.droplet_field(prm.shape, drops, p["W"], wall_axes=(1,))
    muA0, muB0 = 0.01 * rng.standard_normal(prm.shape), 0.01 * rng.standard_normal(prm.shape)
    pops = oracle_populations(prm, olbm.run(olbm.init(phi0, muA0, muB0, prm), prm, 2))
    lam = rng.standard_normal(pops.shape).astype(np.float32).astype(np.float64)
    got, _ = _gpu_adjoint_step(p, "fp64", pops, phi0, muA0, muB0, lam)
    for trial in range(3):
        v = rng.standard_normal(pops.shape)
        jv = _oracle_step_pops(pops + 1j * H_CS * v, p).imag / H_CS
        lhs, rhs = float(np.dot(lam.ravel(), jv.ravel())), float(np.dot(got.ravel(), v.ravel()))
        print(f"  trial {trial}: {lhs:.12e} {rhs:.12e} rel {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_paper_lattice_phase_field_run_gradient():
    """L = sum (phi_T - phi_0)^2 through the differentiable run (checkpointed adjoint)
    against complex-step derivatives of the oracle run."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import LBMConfig, phase_field_run
    p = inputs._base(30, 24, 1, W=3.0, scalar="D2Q9", fluid="D2Q9", bc=("periodic", "walls", "periodic"),
                     drho=0.5, g=(0.0, -1e-4, 0.0), sigma=1e-3, nu=(0.1, 0.05))
    rng = inputs.rng_for(303)
    drops = inputs.place_droplets((1, 24, 30), 2, 4.0, 6.0, 3.0, rng, wall_axes=(1,))
    phi0 = inputs.droplet_field((1, 24, 30), drops, 3.0, wall_axes=(1,))
    mu = rng.normal(0.0, 1e-3, (2, 1, 24, 30))
    steps = 16
    cfg = LBMConfig(**p, precision="fp64")
    phi_t = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
    theta = torch.tensor([p["M_phi"], *p["M_A"], *p["M_B"], p["W"]], dtype=torch.float64, requires_grad=True)
    target = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    loss = ((phase_field_run(phi_t, theta, cfg, steps, mu[0], mu[1]) - target) ** 2).sum()
    loss.backward()
    v = rng.standard_normal(phi0.shape)

    def oracle_loss(q, dphi):
        qp = olbm.Params(**q)
        st = olbm.run(olbm.init(phi0 + dphi, mu[0].astype(complex), mu[1].astype(complex), qp), qp, steps)
        return np.sum((np.asarray(olbm.moments(st, qp)["phi"]) - phi0) ** 2)

    h = 1e-30
    checks = (("M_phi", float(theta.grad[0]), oracle_loss(dict(p, M_phi=p["M_phi"] + 1j * h), 0j).imag / h),
              ("W", float(theta.grad[5]), oracle_loss(dict(p, W=p["W"] + 1j * h), 0j).imag / h),
              ("phi0.v", float((phi_t.grad.cpu().numpy() * v).sum()), oracle_loss(p, 1j * h * v).imag / h))
    for name, g, want in checks:
        print(f"  {name}: gpu {g:.10e} oracle {want:.10e}", flush=True)
        assert abs(g - want) <= 1e-6 * abs(want) + 1e-12, name

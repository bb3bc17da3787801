"""The hand-written discrete adjoint of the GPU step against the FP64 oracle.

The oracle has no reverse mode of its own.  Its forward step is pinned to the paper
(test_oracle_pins.py) and is analytic in its inputs, so complex-step evaluation
gives exact directional derivatives: J v = Im(step(P + i h v)) / h.  The adjoint
is checked against that in three ways:

  * per step, entry by entry: (J^T lambda)_j = <lambda, J e_j> for every column j
    on tiny grids (every column in 2D, a sample of columns in 3D), plus the six
    parameter partials <lambda, dP'/dtheta_j>;
  * per step, dot products <lambda, J v> = <J^T lambda, v> for random v on grids
    that span several work-group tiles and the walls;
  * end to end through PhaseFieldRun (sqrt(T) checkpointing) on a 64 x 64 crop of
    the sedimenting-drop workload: dL/dM, dL/dW and directional derivatives in phi_0
    against the oracle (complex step through the whole run) and against central
    finite differences of the GPU forward (h = 1e-3).

Adjoint populations are stored in FP32, so agreement is ~1e-7 relative per step in
FP64 storage; the bars below are stated per check.
"""

import functools
import os

import numpy as np
import pytest

from helpers import gpu_config, oracle_params, oracle_populations, rel_l2
from oracle import lbm as olbm
from paper_2409_03401_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H_CS = 1e-30   # complex-step size
THETA_KEYS = ("M_phi", "M_A0", "M_A1", "M_B0", "M_B1", "W")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _theta_params(p, j, dv):
    """Oracle parameter dict with theta_j shifted by dv (may be complex)."""
    q = dict(p)
    if j == 0:
        q["M_phi"] = p["M_phi"] + dv
    elif j in (1, 2):
        m = list(p["M_A"]); m[j - 1] = m[j - 1] + dv; q["M_A"] = tuple(m)
    elif j in (3, 4):
        m = list(p["M_B"]); m[j - 3] = m[j - 3] + dv; q["M_B"] = tuple(m)
    else:
        q["W"] = p["W"] + dv
    return q


def _split(pops, prm):
    """[slot][z][y][x] canonical array -> oracle State (f, g, hA, hB)."""
    qf = prm.flat.Q if prm.fluid else 0
    qs = prm.slat.Q
    f = pops[:qf] if qf else None
    return olbm.State(g=pops[qf:qf + qs], hA=pops[qf + qs:qf + 2 * qs], hB=pops[qf + 2 * qs:], f=f)


def _oracle_step_pops(pops, p):
    prm = oracle_params(p)
    return oracle_populations(prm, olbm.step(_split(pops, prm), prm))


# ----------------------------------------------------------------------------------------
# tiny per-step cases: a drop with noise so that u, F and the source are all non-zero

STEP_CASES = {
    # name: (params, precision, warm-up steps)
    "d2q9_walls_y_fp64": (dict(nx=8, ny=6, fluid="D2Q9", scalar="D2Q5", bc=("periodic", "walls", "periodic"),
                               W=3.0, lam=2.0, M_phi=0.12, M_A=(0.1, 0.07), M_B=(0.05, 0.09),
                               drho=0.5, g=(2e-4, -1e-3, 0.0), sigma=0.02, nu=(0.1, 0.05)), "fp64", 3),
    "d2q9_periodic_fp32": (dict(nx=9, ny=7, fluid="D2Q9", scalar="D2Q5", W=3.0, lam=2.0, M_phi=0.1,
                                M_A=(0.1, 0.07), M_B=(0.05, 0.09), drho=0.4, g=(0.0, -1e-3, 0.0), sigma=0.02,
                                nu=(0.1, 0.05)), "fp32", 3),
    "d2q5_noflow_walls_x_fp64": (dict(nx=10, ny=5, scalar="D2Q5", bc=("walls", "periodic", "periodic"), W=3.0,
                                      lam=2.0, M_phi=0.1, M_A=(0.1, 0.07), M_B=(0.05, 0.09)), "fp64", 3),
    "d3q19_walls_xz_fp64": (dict(nx=4, ny=5, nz=4, fluid="D3Q19", scalar="D3Q7",
                                 bc=("walls", "periodic", "walls"), W=2.5, lam=2.0, M_phi=0.1, M_A=(0.1, 0.07),
                                 M_B=(0.05, 0.09), drho=0.5, g=(1e-4, 2e-4, -1e-3), sigma=0.02,
                                 nu=(0.1, 0.05)), "fp64", 2),
}


@functools.lru_cache(maxsize=None)
def step_case(name):
    """(params, precision, P^n [slot][z][y][x], phi0, muA0, muB0, lambda)."""
    p, prec, warm = STEP_CASES[name]
    p = {**inputs._base(p["nx"], p["ny"], p.get("nz", 1)), **p}
    prm = oracle_params(p)
    shape = prm.shape
    rng = inputs.rng_for(100 + sorted(STEP_CASES).index(name))
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    r = np.sqrt((xx - shape[2] / 2) ** 2 + (yy - shape[1] / 2) ** 2 + (zz - shape[0] / 2) ** 2 * (shape[0] > 1))
    phi0 = 0.5 * (1 + np.tanh((0.35 * min(shape[1:]) - r))) + 0.05 * rng.uniform(-1, 1, shape)
    muA0 = 0.01 * rng.standard_normal(shape)
    muB0 = 0.01 * rng.standard_normal(shape)
    st = olbm.run(olbm.init(phi0, muA0, muB0, prm), prm, warm)
    pops = oracle_populations(prm, st)
    if prec == "fp32":
        pops = pops.astype(np.float32).astype(np.float64)  # the state the GPU holds
    lam = rng.standard_normal(pops.shape).astype(np.float32).astype(np.float64)
    return p, prec, pops, phi0, muA0, muB0, lam


def _gpu_adjoint_step(p, prec, pops, phi0, muA0, muB0, lam):
    from paper_2409_03401_amd.lbm import Simulation
    sim = Simulation(gpu_config(p, prec), phi0, muA0, muB0)
    sim.set_populations(pops)
    ck = sim.save()
    work = sim.adjoint_workspace()
    sim.adjoint_set(work, lam)
    sim.adjoint_step_phi(ck, sim.phase_field(ck), work)
    out = sim.adjoint_get(work).cpu().numpy()
    return out, sim.adjoint_theta(work).cpu().numpy()


def _oracle_column(pops, p, j):
    v = np.zeros(pops.size)
    v[j] = 1.0
    out = _oracle_step_pops(pops + 1j * H_CS * v.reshape(pops.shape), p)
    return out.imag / H_CS


def _oracle_theta_jvp(pops, p, j):
    out = _oracle_step_pops(pops.astype(complex), _theta_params(p, j, 1j * H_CS))
    return out.imag / H_CS


@pytest.mark.parametrize("name", ["d2q9_walls_y_fp64", "d2q9_periodic_fp32", "d2q5_noflow_walls_x_fp64",
                                  "d3q19_walls_xz_fp64"])
def test_adjoint_step_entrywise(name):
    """(J^T lambda)_j for every column (2D) or sampled columns (3D), and the theta partials."""
    _require_gpu()
    p, prec, pops, phi0, muA0, muB0, lam = step_case(name)
    print(f"[adjoint entrywise] {name} pops {pops.shape}", flush=True)
    got, gth = _gpu_adjoint_step(p, prec, pops, phi0, muA0, muB0, lam)
    n = pops.size
    if pops.shape[1] > 1:  # 3D: every slot at corner, edge and face nodes plus random nodes
        nodes = pops[0].size
        nz, ny, nx = pops.shape[1:]
        pick = {0, nodes - 1, (nz - 1) * ny * nx, nx - 1, (ny // 2) * nx + nx // 2}
        pick |= set(inputs.rng_for(7).integers(0, nodes, 6).tolist())
        cols = [s * nodes + i for s in range(pops.shape[0]) for i in sorted(pick)]
    else:
        cols = range(n)
    want = np.array([np.dot(lam.ravel(), _oracle_column(pops, p, j).ravel()) for j in cols])
    g = got.ravel()[list(cols)]
    scale = np.max(np.abs(want))
    err = np.max(np.abs(g - want)) / scale
    print(f"  columns {len(want)}: max err / max |want| = {err:.3e}, rel L2 {rel_l2(g, want):.3e}")
    bar = 2e-6 if prec == "fp64" else 2e-5
    assert err < bar
    for j in range(6):
        t = np.dot(lam.ravel(), _oracle_theta_jvp(pops, p, j).ravel())
        print(f"  d/d{THETA_KEYS[j]}: gpu {gth[j]:.10e} oracle {t:.10e}")
        assert abs(gth[j] - t) <= bar * max(abs(t), 1e-3 * scale)


DOT_CASES = {
    # grids spanning many 256-node work-groups of the adjoint kernels, with a ragged edge
    "d2q9_walls_y_150x77": (dict(nx=150, ny=77, fluid="D2Q9", scalar="D2Q5", bc=("periodic", "walls", "periodic"),
                                 W=4.0, lam=inputs.LAMBDA_TIE, M_phi=0.1, M_A=(0.1, 0.07), M_B=(0.05, 0.09),
                                 drho=0.5, g=(0.0, -1e-4, 0.0), sigma=0.01, nu=(0.1, 0.05)), "fp64"),
    "d3q19_walls_y_70x44x38": (dict(nx=70, ny=44, nz=38, fluid="D3Q19", scalar="D3Q7",
                                    bc=("periodic", "walls", "periodic"), W=4.0, lam=inputs.LAMBDA_TIE,
                                    M_phi=0.1, M_A=(0.1, 0.07), M_B=(0.05, 0.09), drho=0.5, g=(0.0, -1e-4, 0.0),
                                    sigma=0.01, nu=(0.1, 0.05)), "fp64"),
    "d3q19_allwalls_19x17x15_fp32": (dict(nx=19, ny=17, nz=15, fluid="D3Q19", scalar="D3Q7",
                                          bc=("walls", "walls", "walls"), W=3.0, lam=2.0, M_phi=0.1,
                                          M_A=(0.1, 0.07), M_B=(0.05, 0.09), drho=0.5, g=(1e-4, 0.0, -5e-4),
                                          sigma=0.01, nu=(0.1, 0.05)), "fp32"),
}


@pytest.mark.parametrize("name", sorted(DOT_CASES))
def test_adjoint_step_dot_product(name):
    """<lambda, J v> (oracle complex step) = <J^T lambda, v> (GPU) for random v."""
    _require_gpu()
    p, prec = DOT_CASES[name]
    p = {**inputs._base(p["nx"], p["ny"], p.get("nz", 1)), **p}
    prm = oracle_params(p)
    shape = prm.shape
    rng = inputs.rng_for(200 + sorted(DOT_CASES).index(name))
    wall_axes = tuple(a for a in range(3) if p["bc"][a] == "walls" and shape[2 - a] > 1)
    drops = inputs.place_droplets(shape, 3, 5, 9, p["W"], rng, wall_axes=wall_axes)
    phi0 = inputs.droplet_field(shape, drops, p["W"], wall_axes=wall_axes)
    muA0 = 0.01 * rng.standard_normal(shape)
    muB0 = 0.01 * rng.standard_normal(shape)
    st = olbm.run(olbm.init(phi0, muA0, muB0, prm), prm, 2)
    pops = oracle_populations(prm, st)
    if prec == "fp32":
        pops = pops.astype(np.float32).astype(np.float64)
    lam = rng.standard_normal(pops.shape).astype(np.float32).astype(np.float64)
    print(f"[adjoint dot] {name} pops {pops.shape}", flush=True)
    got, _ = _gpu_adjoint_step(p, prec, pops, phi0, muA0, muB0, lam)
    for trial in range(3):
        v = rng.standard_normal(pops.shape)
        jv = _oracle_step_pops(pops + 1j * H_CS * v, p).imag / H_CS
        lhs = float(np.dot(lam.ravel(), jv.ravel()))
        rhs = float(np.dot(got.ravel(), v.ravel()))
        # for random vectors the sum is ~|lambda| |Jv| / sqrt(n); FP32 rounding of the
        # adjoint entries perturbs it by ~1e-7 |lambda| |Jv| / sqrt(n)
        print(f"  trial {trial}: <lam, Jv> = {lhs:.12e}  <J^T lam, v> = {rhs:.12e}  rel {abs(lhs - rhs) / abs(lhs):.2e}")
        assert abs(lhs - rhs) <= (1e-5 if prec == "fp64" else 1e-4) * abs(lhs)


def test_adjoint_init_entrywise():
    """Adjoint of lbm_init (mu_0 fixed): dL/dphi_0 per node and the theta partials."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation
    p, prec, pops, phi0, muA0, muB0, lam = step_case("d2q9_walls_y_fp64")
    prm = oracle_params(p)
    sim = Simulation(gpu_config(p, prec), phi0, muA0, muB0)
    work = sim.adjoint_workspace()
    sim.adjoint_set(work, lam)
    gphi = torch.empty(prm.shape, dtype=torch.float64, device="cuda")
    sim.adjoint_init(work, gphi)
    gphi = gphi.cpu().numpy()
    gth = sim.adjoint_theta(work).cpu().numpy()

    def init_pops(ph, q):
        qp = oracle_params(q)
        return oracle_populations(qp, olbm.init(ph, muA0.astype(complex), muB0.astype(complex), qp))

    want = np.zeros(phi0.size)
    for j in range(phi0.size):
        d = np.zeros(phi0.size)
        d[j] = H_CS
        want[j] = np.dot(lam.ravel(), (init_pops(phi0 + 1j * d.reshape(phi0.shape), p).imag / H_CS).ravel())
    err = np.max(np.abs(gphi.ravel() - want)) / np.max(np.abs(want))
    print(f"[adjoint init] dL/dphi0 max err / max = {err:.3e}")
    assert err < 2e-6
    for j in range(6):
        t = np.dot(lam.ravel(), (init_pops(phi0.astype(complex), _theta_params(p, j, 1j * H_CS)).imag / H_CS).ravel())
        print(f"  d/d{THETA_KEYS[j]}: gpu {gth[j]:.10e} oracle {t:.10e}")
        assert abs(gth[j] - t) <= 2e-6 * max(abs(t), 1e-3 * np.max(np.abs(want)))


# ----------------------------------------------------------------------------------------
# end to end: PhaseFieldRun on a 64 x 64 crop of the sedimenting-drop workload

def _crop_case(kind):
    """(params, phi0, muA0, muB0, steps, target)."""
    w = inputs.single_drop_2d(n=64, R=12.0, centre=(32.0, 40.0, 0.0))
    p = dict(w.params)
    if kind == "crop":          # the workload's own parameters, T = 256
        steps, muA0, muB0 = 256, w.muA0, w.muB0
    else:                       # stronger forcing and unequal mobilities, T = 64
        rng = inputs.rng_for(300)
        p.update(g=(0.0, -5e-4, 0.0), sigma=5e-3, M_A=(0.1, 0.06), M_B=(0.05, 0.09))
        steps = 64
        muA0 = 0.01 * rng.standard_normal(w.phi0.shape)
        muB0 = 0.01 * rng.standard_normal(w.phi0.shape)
    # target: the oracle's phi(T) with every mobility raised by 10 %
    q = dict(p, M_phi=1.1 * p["M_phi"], M_A=tuple(1.1 * m for m in p["M_A"]),
             M_B=tuple(1.1 * m for m in p["M_B"]))
    qp = oracle_params(q)
    target = np.asarray(olbm.moments(olbm.run(olbm.init(w.phi0, muA0, muB0, qp), qp, steps), qp)["phi"])
    return p, w.phi0, muA0, muB0, steps, target


@functools.lru_cache(maxsize=None)
def crop_case(kind):
    return _crop_case(kind)


def _oracle_loss(p, phi0, muA0, muB0, steps, target):
    prm = oracle_params(p)
    st = olbm.run(olbm.init(phi0, muA0.astype(complex), muB0.astype(complex), prm), prm, steps)
    phi = np.asarray(olbm.moments(st, prm)["phi"])
    return np.sum((phi - target) ** 2)


@pytest.mark.parametrize("kind,prec", [("crop", "fp32"), ("crop", "fp64"), ("forced", "fp64"), ("forced", "fp32")])
def test_phase_field_run_gradients(kind, prec):
    _require_gpu()
    from paper_2409_03401_amd.lbm import LBMConfig, phase_field_run, with_theta
    p, phi0, muA0, muB0, steps, target = crop_case(kind)
    print(f"[adjoint e2e] {kind} {prec} T={steps}", flush=True)
    cfg = gpu_config(p, prec)
    dev = "cuda"
    phi0_t = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
    M = torch.tensor(p["M_phi"], dtype=torch.float64, requires_grad=True)
    W = torch.tensor(p["W"], dtype=torch.float64, requires_grad=True)
    # one mobility scale s multiplies all five mobilities; theta_j = s * m_j
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    m0 = torch.tensor([p["M_phi"], *p["M_A"], *p["M_B"]], dtype=torch.float64)
    theta = torch.cat([s * m0, W.reshape(1)])
    tgt = torch.tensor(target, dtype=torch.float64, device=dev)
    phiT = phase_field_run(phi0_t, theta, cfg, steps, muA0, muB0)
    loss = ((phiT - tgt) ** 2).sum()
    loss.backward()
    g_s, g_W = float(s.grad), float(W.grad)
    g_phi = phi0_t.grad.cpu().numpy()

    # oracle: complex step through the whole run
    def cs(q, dphi=None):
        ph = phi0 + (1j * H_CS * dphi if dphi is not None else 0j)
        return _oracle_loss(q, ph, muA0, muB0, steps, target).imag / H_CS

    ps = dict(p, M_phi=p["M_phi"] * (1 + 1j * H_CS), M_A=tuple(m * (1 + 1j * H_CS) for m in p["M_A"]),
              M_B=tuple(m * (1 + 1j * H_CS) for m in p["M_B"]))
    o_s = cs(ps)
    o_W = cs(dict(p, W=p["W"] + 1j * H_CS))
    rng = inputs.rng_for(400)
    v = rng.standard_normal(phi0.shape) * (np.abs(np.gradient(phi0, axis=1)) + 0.01)
    o_v = cs(p, v)
    g_v = float(np.sum(g_phi * v))
    L0 = float(loss.detach())
    print(f"  loss {L0:.6e}")
    print(f"  dL/ds  gpu {g_s:.8e} oracle {o_s:.8e}")
    print(f"  dL/dW  gpu {g_W:.8e} oracle {o_W:.8e}")
    print(f"  dL/dphi0.v gpu {g_v:.8e} oracle {o_v:.8e}")
    bar = 1e-5 if prec == "fp64" else 2e-3
    for g, o in ((g_s, o_s), (g_W, o_W), (g_v, o_v)):
        assert abs(g - o) <= bar * abs(o) + 1e-9 * L0

    # central finite differences of the GPU forward, h = 1e-3
    if prec == "fp64":
        from paper_2409_03401_amd.lbm import Simulation

        def gpu_loss(c, ph):
            sim = Simulation(c, ph, muA0, muB0)
            sim.step(steps)
            return float(((sim.moments(["phi"])["phi"] - tgt) ** 2).sum())

        h = 1e-3
        fd_W = (gpu_loss(with_theta(cfg, [*m0.tolist(), p["W"] + h]), phi0) -
                gpu_loss(with_theta(cfg, [*m0.tolist(), p["W"] - h]), phi0)) / (2 * h)
        fd_s = (gpu_loss(with_theta(cfg, [*(m0 * (1 + h)).tolist(), p["W"]]), phi0) -
                gpu_loss(with_theta(cfg, [*(m0 * (1 - h)).tolist(), p["W"]]), phi0)) / (2 * h)
        fd_v = (gpu_loss(cfg, phi0 + h * v) - gpu_loss(cfg, phi0 - h * v)) / (2 * h)
        print(f"  FD h=1e-3: dL/ds {fd_s:.8e} dL/dW {fd_W:.8e} dL/dphi0.v {fd_v:.8e}")
        for g, fd in ((g_s, fd_s), (g_W, fd_W), (g_v, fd_v)):
            assert abs(g - fd) <= 1e-3 * abs(fd) + 1e-9 * L0


GOLDEN_LONG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_crop4096_oracle.npz")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_phase_field_run_gradients_long(prec):
    """T = 4096 on the 64 x 64 crop: dL/ds, dL/dW and dL/dphi_0 . v through
    PhaseFieldRun against the oracle's complex-step derivatives through the whole run
    (stored by tests/golden/make_adjoint_crop4096.py) and, in FP64, against central
    differences of the GPU forward (h = 1e-3).  The adjoint populations are FP32, so
    the bars are wider than at T = 256: 1e-4 relative in FP64 storage, 1e-2 in FP32
    storage (whose forward trajectory itself departs from the oracle's)."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation, phase_field_run, with_theta
    g = np.load(GOLDEN_LONG)
    steps = int(g["steps"])
    w = inputs.single_drop_2d(n=64, R=12.0, centre=(32.0, 40.0, 0.0))
    p = dict(w.params)
    print(f"[adjoint long] {prec} T={steps}", flush=True)
    cfg = gpu_config(p, prec)
    dev = "cuda"
    phi0_t = torch.tensor(w.phi0, dtype=torch.float64, device=dev, requires_grad=True)
    W = torch.tensor(p["W"], dtype=torch.float64, requires_grad=True)
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    m0 = torch.tensor([p["M_phi"], *p["M_A"], *p["M_B"]], dtype=torch.float64)
    theta = torch.cat([s * m0, W.reshape(1)])
    tgt = torch.tensor(g["target"], dtype=torch.float64, device=dev)
    phiT = phase_field_run(phi0_t, theta, cfg, steps, w.muA0, w.muB0)
    loss = ((phiT - tgt) ** 2).sum()
    loss.backward()
    v = g["v"]
    got = {"s": float(s.grad), "W": float(W.grad), "v": float(np.sum(phi0_t.grad.cpu().numpy() * v))}
    ref = {"s": float(g["dL_ds"]), "W": float(g["dL_dW"]), "v": float(g["dL_dv"])}
    L0 = float(g["loss"])
    print(f"  loss gpu {float(loss.detach()):.8e} oracle {L0:.8e}", flush=True)
    bar = 1e-4 if prec == "fp64" else 1e-2
    for k in ("s", "W", "v"):
        rel = abs(got[k] - ref[k]) / abs(ref[k])
        print(f"  dL/d{k}: gpu {got[k]:.8e} oracle (complex step) {ref[k]:.8e} rel err {rel:.2e}", flush=True)
        assert rel <= bar, (k, rel)
    if prec == "fp64":
        def gpu_loss(c, ph):
            sim = Simulation(c, ph, w.muA0, w.muB0)
            sim.step(steps)
            return float(((sim.moments(["phi"])["phi"] - tgt) ** 2).sum())

        h = 1e-3
        fd = {"W": (gpu_loss(with_theta(cfg, [*m0.tolist(), p["W"] + h]), w.phi0) -
                    gpu_loss(with_theta(cfg, [*m0.tolist(), p["W"] - h]), w.phi0)) / (2 * h),
              "s": (gpu_loss(with_theta(cfg, [*(m0 * (1 + h)).tolist(), p["W"]]), w.phi0) -
                    gpu_loss(with_theta(cfg, [*(m0 * (1 - h)).tolist(), p["W"]]), w.phi0)) / (2 * h),
              "v": (gpu_loss(cfg, w.phi0 + h * v) - gpu_loss(cfg, w.phi0 - h * v)) / (2 * h)}
        for k in ("s", "W", "v"):
            rel = abs(got[k] - fd[k]) / abs(fd[k])
            print(f"  dL/d{k}: central difference of the GPU forward {fd[k]:.8e} rel err {rel:.2e}", flush=True)
            assert rel <= 1e-3, (k, rel)


def test_boundary_calls_gradient():
    """The gradient through the boundary calls alone: lbm_save of every state,
    lbm_set_state, lbm_adjoint_step (phi formed inside, parameter gradient added to a
    device array each step) and lbm_init_adjoint, on the strongly forced 64 x 64 case
    in FP64 storage.  dL/dphi_0 equals the checkpointed PhaseFieldRun bitwise, the six
    parameter partials to 1e-12; dL/dM_phi and dL/dW match complex-step derivatives of
    the oracle within 1e-5."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation, phase_field_run, theta_of
    p, phi0, muA0, muB0, steps, target = crop_case("forced")
    cfg = gpu_config(p, "fp64")
    sim = Simulation(cfg, phi0, muA0, muB0)
    ck = [sim.save()]
    for _ in range(steps):
        sim.step(1)
        ck.append(sim.save())
    # lbm_set_state returns to state 0; stepping again reproduces state T bitwise
    sim.set_state(ck[0])
    sim.step(steps)
    assert torch.equal(sim.save(), ck[steps])
    phiT = sim.moments(["phi"])["phi"]
    tgt = torch.tensor(target, dtype=torch.float64, device="cuda")
    work = sim.adjoint_workspace()
    grad = torch.zeros(6, dtype=torch.float64, device="cuda")
    sim.adjoint_seed(ck[steps], (2.0 * (phiT - tgt)).reshape(-1), work)
    for n in reversed(range(steps)):
        sim.adjoint_step(ck[n], work, grad)
    gphi0 = torch.empty(cfg.nodes, dtype=torch.float64, device="cuda")
    sim.init_adjoint(work, gphi0, grad)
    g = grad.cpu().numpy()

    phi0_t = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
    theta = torch.tensor(theta_of(cfg), dtype=torch.float64, requires_grad=True)
    ((phase_field_run(phi0_t, theta, cfg, steps, muA0, muB0) - tgt) ** 2).sum().backward()
    assert torch.equal(gphi0.reshape(phi0_t.shape), phi0_t.grad)
    want = theta.grad.numpy()
    assert np.all(np.abs(g - want) <= 1e-12 * np.abs(want).max()), (g, want)

    h = 1e-30
    for j, key in ((0, "M_phi"), (5, "W")):
        o = _oracle_loss(dict(p, **{key: p[key] + 1j * h}), phi0, muA0, muB0, steps, target).imag / h
        print(f"[boundary adjoint] dL/d{key}: gpu {g[j]:.10e} oracle {o:.10e}", flush=True)
        assert abs(g[j] - o) <= 1e-5 * abs(o)


def test_checkpoint_segments_agree():
    """The gradient does not depend on the checkpoint spacing (recompute is exact)."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import phase_field_run
    p, phi0, muA0, muB0, steps, target = crop_case("forced")
    cfg = gpu_config(p, "fp32")
    tgt = torch.tensor(target, dtype=torch.float64, device="cuda")
    grads = []
    for seg in (1, 7, 64):
        phi0_t = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
        theta = torch.tensor([p["M_phi"], *p["M_A"], *p["M_B"], p["W"]], dtype=torch.float64, requires_grad=True)
        loss = ((phase_field_run(phi0_t, theta, cfg, steps, muA0, muB0, segment=seg) - tgt) ** 2).sum()
        loss.backward()
        grads.append((phi0_t.grad.cpu().numpy(), theta.grad.numpy()))
    for g in grads[1:]:
        assert np.array_equal(g[0], grads[0][0])
        assert np.array_equal(g[1], grads[0][1])


def test_adjoint_unsupported_precisions():
    _require_gpu()
    from paper_2409_03401_amd.lbm import LBMError, Simulation, LBM_EUNSUPPORTED
    p, prec, pops, phi0, muA0, muB0, lam = step_case("d2q9_walls_y_fp64")
    sim = Simulation(gpu_config(p, "bf16"), phi0, muA0, muB0)
    work = sim.adjoint_workspace()
    with pytest.raises(LBMError) as e:
        ck = sim.save()
        sim.adjoint_step_phi(ck, sim.phase_field(ck), work)
    assert e.value.code == LBM_EUNSUPPORTED


def test_step_external_and_phase_field_match_the_handle():
    """lbm_step_external from a checkpoint equals lbm_step bitwise; its phi output and
    lbm_phase_field equal phi of lbm_moments (in the compute type)."""
    _require_gpu()
    from paper_2409_03401_amd.lbm import Simulation
    p, prec, pops, phi0, muA0, muB0, lam = step_case("d2q9_walls_y_fp64")
    for prec in ("fp32", "fp64"):
        sim = Simulation(gpu_config(p, prec), phi0, muA0, muB0)
        sim.step(3)
        a = sim.save()
        phi_m = sim.moments(["phi"], dtype=torch.float64)["phi"].reshape(-1)
        b = torch.empty_like(a)
        phi_src = torch.empty(sim.cfg.nodes, dtype=sim.phi_dtype, device="cuda")
        sim.step_external(a, b, phi_src)
        phi_pf = sim.phase_field(a)
        sim.step(1)
        pop_step = sim.populations()
        sim.restore(b)  # checkpoints carry unwritten slot padding: compare decoded populations
        assert torch.equal(sim.populations(), pop_step)
        assert torch.equal(phi_src, phi_pf)
        assert torch.equal(phi_pf, phi_m.to(sim.phi_dtype))


def test_adjoint_argument_errors():
    _require_gpu()
    import ctypes
    from paper_2409_03401_amd.lbm import LBM_EINVAL, Simulation, lib
    p, prec, pops, phi0, muA0, muB0, lam = step_case("d2q9_walls_y_fp64")
    sim = Simulation(gpu_config(p, "fp32"), phi0, muA0, muB0)
    work = sim.adjoint_workspace()
    ck = sim.save()
    null = ctypes.c_void_p()
    L = lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.lbm_adjoint_step_phi(sim._h, ctypes.c_void_p(ck.data_ptr()), null, ctypes.c_void_p(work.data_ptr()),
                                  s) == LBM_EINVAL
    assert L.lbm_adjoint_step_phi(sim._h, ctypes.c_void_p(ck.data_ptr()), ctypes.c_void_p(ck.data_ptr()), null,
                                  s) == LBM_EINVAL
    grad = torch.zeros(6, dtype=torch.float64, device="cuda")
    assert L.lbm_adjoint_step(sim._h, ctypes.c_void_p(ck.data_ptr()), ctypes.c_void_p(work.data_ptr()), null,
                              s) == LBM_EINVAL
    assert L.lbm_adjoint_step(sim._h, null, ctypes.c_void_p(work.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                              s) == LBM_EINVAL
    assert L.lbm_init_adjoint(sim._h, ctypes.c_void_p(work.data_ptr()), null, ctypes.c_void_p(grad.data_ptr()),
                              s) == LBM_EINVAL
    assert L.lbm_step_external(sim._h, ctypes.c_void_p(ck.data_ptr()), ctypes.c_void_p(ck.data_ptr()), null,
                               s) == LBM_EINVAL
    assert L.lbm_adjoint_theta(sim._h, ctypes.c_void_p(work.data_ptr()), null, s) == LBM_EINVAL
    with pytest.raises(ValueError):
        sim.adjoint_seed(ck, torch.zeros(3, dtype=torch.float64, device="cuda"), work)


"""Throughput of the fused coupled LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sediment_3d_256]

Prints one JSON line.  A step is one pass of the whole hot path (scalar moments with
the phi predictor, LDS-staged grad/lap phi, capillary + buoyancy force, collision of
f, g, h^A, h^B, streaming with bounce-back walls) over every node of the workload.
`value` is million lattice-node updates per second over the timed steps with all
inputs resident in HBM.  `roofline` prices the fused step kernel against the HBM peak
with its algorithmic bytes (every population read once and written once per update).
`cpu_baseline` is the FP64 numpy oracle timed on a bounded crop of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure

WORKLOADS = {
    # name: (builder kwargs, precision)
    "sediment_3d_256": dict(kind="sediment_3d", n=256, precision="fp32"),
    "sediment_3d_256_bf16": dict(kind="sediment_3d", n=256, precision="bf16"),
    "sediment_3d_256_fp16": dict(kind="sediment_3d", n=256, precision="fp16"),
    "spinodal_3d_512_bf16": dict(kind="spinodal_3d", n=512, precision="bf16"),
    "ostwald_2d_1024": dict(kind="ostwald_2d", n=1024, precision="fp32"),
    "single_drop_2d_512": dict(kind="single_drop_2d", n=512, precision="fp32"),
    # the paper's own discretisation and initial condition (D2Q9 for every equation)
    "ostwald_paper_2d_4096": dict(kind="ostwald_paper_2d", n=4096, precision="fp32"),
    "ostwald_paper_2d_4096_bf16": dict(kind="ostwald_paper_2d", n=4096, precision="bf16"),
    # the two-relaxation-time collision on the sedimentation workload
    "sediment_3d_256_trt": dict(kind="sediment_3d", n=256, precision="fp32", collision="TRT"),
    "sediment_3d_256_mrt": dict(kind="sediment_3d", n=256, precision="fp32", collision="MRT"),
    # the variable-density flow model (density ratio 1.5) on the sedimentation workload
    "sediment_3d_256_vd": dict(kind="sediment_3d", n=256, precision="fp32", variable_density=True),
    # general curvature matrices of the free energies (2 x 2 closure per node)
    "sediment_3d_256_kappa": dict(kind="sediment_3d", n=256, precision="fp32",
                                  kappa=((1.0, 0.1, 0.9), (0.95, -0.05, 1.2))),
    # ripening with sedimentation at 512^3 (the paper's 3D run shape, one GPU's share)
    "ripening_sediment_3d_512_bf16": dict(kind="sediment_3d", n=512, precision="bf16", ndrops=2000,
                                          rmin=6.0, rmax=12.0, phi_eq=0.25),
}


def slot_bytes(precision, k):
    return {"fp64": 8, "fp32": 4}.get(precision, 4 if k == 0 else 2)


def bytes_per_update(cfg):
    """Algorithmic HBM bytes per lattice update: each stored population read and written once."""
    b = 0
    for q in ([cfg.qf] if cfg.qf else []) + [cfg.qs] * 3:
        b += sum(slot_bytes(cfg.precision, k) for k in range(q))
    return 2 * b


def build_workload(name):
    w = _build_workload(name)
    spec = WORKLOADS[name]
    if spec.get("collision"):
        w.params = dict(w.params, collision=spec["collision"], trt_magic=(3.0 / 16.0, 0.25),
                        mrt_rates=((1.2, 1.1, 1.2), (1.1, 1.0, 1.2)))
    if spec.get("variable_density"):
        w.params = dict(w.params, variable_density=True)
    if spec.get("kappa"):
        w.params = dict(w.params, kappa=spec["kappa"])
    return w


def _build_workload(name):
    from paper_2409_03401_amd import inputs
    spec = WORKLOADS[name]
    kind = spec["kind"]
    if kind == "sediment_3d":
        kw = {k: spec[k] for k in ("ndrops", "rmin", "rmax", "phi_eq") if k in spec}
        return inputs.sediment_3d(n=spec["n"], precision=spec["precision"], **kw)
    if kind == "spinodal_3d":
        return inputs.spinodal_3d(n=spec["n"], precision=spec["precision"])
    if kind == "ostwald_2d":
        return inputs.ostwald_2d(n=spec["n"], precision=spec["precision"])
    if kind == "single_drop_2d":
        return inputs.single_drop_2d(n=spec["n"], precision=spec["precision"])
    if kind == "ostwald_paper_2d":
        return inputs.ostwald_paper_2d(n=spec["n"], precision=spec["precision"])
    raise KeyError(name)


def time_gpu(w, steps, warmup):
    import torch
    from paper_2409_03401_amd.lbm import LBMConfig, Simulation

    cfg = LBMConfig(**w.params, precision=w.precision)
    sim = Simulation(cfg, w.phi0, w.muA0, w.muB0, c0=w.c0)
    stream = torch.cuda.current_stream()
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kernel_ms = e0.elapsed_time(e1) / steps
    diag = sim.diagnostics()
    resident = sim.state.numel()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return cfg, wall, kernel_ms, diag, resident


def copy_ceiling(mib=1024, reps=5):
    """Device-to-device copy of `mib` MiB (torch copy kernel): a measured HBM ceiling
    for plain streaming on this GPU, read + write bytes per second."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def profiled_traffic(workload, kernel_sha):
    """HBM bytes per launch of the step kernel from the committed counter summary
    (profiles/k_lbm_<workload>_hbm.md), if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"k_lbm_{workload}_hbm.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2409_03401_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hpp", ".hip")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def cpu_baseline(budget_s=12.0):
    """The oracle as it stands on a 64^3 crop of the sediment workload (same recipe:
    walls in z, D3Q19 + 3 x D3Q7, 4 droplets R ~ U[10, 14]), timed for about budget_s."""
    from oracle import lbm as olbm
    from paper_2409_03401_amd import inputs
    w = inputs.sediment_3d(n=64, ndrops=4, rmin=10.0, rmax=14.0)
    prm = olbm.Params(**w.params)
    st = olbm.init(w.phi0, w.muA0, w.muB0, prm)
    st = olbm.step(st, prm)  # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        st = olbm.step(st, prm)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s and n >= 3:
            break
    nodes = w.nodes
    return {"value": nodes * n / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"64^3 crop of the sediment workload, D3Q19 + 3xD3Q7, FP64 numpy, {n} steps "
                      f"in {el:.1f} s (single thread; host has {os.cpu_count()} logical CPUs)"}


def adjoint_timing(n=512, steps=4096, segment=None, kind="single_drop_2d"):
    """Forward and backward wall time of the differentiable run on the sedimenting
    drop (n x n, D2Q9 + 3 x D2Q5, FP32 storage, T = steps, checkpoints every
    ceil(sqrt(T)) steps).  The backward pass includes the recomputation of every
    segment, the adjoint steps and the adjoint of the initialisation."""
    import torch
    from paper_2409_03401_amd import inputs
    from paper_2409_03401_amd.lbm import LBMConfig, Simulation, phase_field_run, theta_of

    w = inputs.single_drop_2d(n=n) if kind == "single_drop_2d" else inputs.sediment_3d(n=n, ndrops=max(4, n // 4))
    cfg = LBMConfig(**w.params, precision="fp32")
    sim = Simulation(cfg, w.phi0, w.muA0, w.muB0)
    sim.step(16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    sim.close()
    del sim

    target = torch.tensor(w.phi0, dtype=torch.float64, device="cuda")
    # the first pass fills the caching allocator with the checkpoint and segment
    # buffers; the second is timed
    for _ in range(2):
        phi0 = torch.tensor(w.phi0, dtype=torch.float64, device="cuda", requires_grad=True)
        theta = torch.tensor(theta_of(cfg), dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phiT = phase_field_run(phi0, theta, cfg, steps, w.muA0, w.muB0, segment)
        loss = ((phiT - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    finite = bool(torch.isfinite(phi0.grad).all()) and bool(torch.isfinite(theta.grad).all())
    del phi0, theta, target, phiT, loss
    torch.cuda.empty_cache()
    seg = segment or (math.isqrt(steps - 1) + 1)
    return {
        "workload": f"{kind}_{n}_fp32",
        "steps": steps,
        "segment": seg,
        "forward_ms": round(fwd * 1e3, 2),
        "forward_with_checkpoints_ms": round((t1 - t0) * 1e3, 2),
        "backward_ms": round((t2 - t1) * 1e3, 2),
        "ratio": round((t2 - t1) / fwd, 3),
        "gradients_finite": finite,
    }


def series_run(name, steps, every):
    """Droplet count, mean radius and max |u| over a run (diagnostics every `every`
    steps, recorded on the GPU), with a least-squares fit of <R>^3 = a + k t over the
    second half of the records (coarsening law of the ripening workload)."""
    import numpy as np
    import torch
    from paper_2409_03401_amd.lbm import LBMConfig, Simulation
    w = build_workload(name)
    cfg = LBMConfig(**w.params, precision=w.precision)
    sim = Simulation(cfg, w.phi0, w.muA0, w.muB0, c0=w.c0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = sim.run_series(steps, every)
    wall = time.perf_counter() - t0
    t = d["step"].astype(float)
    R3 = d["mean_radius"] ** 3
    h = len(t) // 2
    k, a = np.polyfit(t[h:], R3[h:], 1)
    fit = a + k * t[h:]
    r2 = 1.0 - np.sum((R3[h:] - fit) ** 2) / max(np.sum((R3[h:] - R3[h:].mean()) ** 2), 1e-300)
    return {
        "workload": name, "steps": steps, "every": every,
        "MLUPS_with_diagnostics": round(cfg.nodes * steps / wall / 1e6, 1),
        "placed_droplets": len(w.drops) if w.drops else None,
        "step": d["step"].tolist(), "droplets": d["droplets"].tolist(),
        "mean_radius": [round(v, 4) for v in d["mean_radius"]],
        "max_u": [float(f"{v:.4e}") for v in d["max_u"]],
        "nan_count": int(d["nan_count"].max()),
        "R3_fit_second_half": {"slope_per_step": float(f"{k:.5e}"), "intercept": round(a, 3), "r2": round(r2, 5)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sediment_3d_256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 16-bit storage variants and the adjoint timing")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the differentiable run (forward, backward, ratio)")
    ap.add_argument("--adjoint-n", type=int, nargs="+", default=[512, 2048],
                    help="grid sizes n (n x n) for --adjoint-only")
    ap.add_argument("--adjoint-steps", type=int, default=4096)
    ap.add_argument("--adjoint-kind", default="single_drop_2d", choices=["single_drop_2d", "sediment_3d"])
    ap.add_argument("--series", default=None, choices=sorted(WORKLOADS),
                    help="only record the diagnostics time series of a workload (droplet count, <R>, max |u|)")
    ap.add_argument("--series-steps", type=int, default=20000)
    ap.add_argument("--series-every", type=int, default=500)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to scale HBM counters")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs one simulation domain on one GPU; "
                                   "multi-GPU runs (--gpus > 1) are not supported"}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    if args.series:
        print(f"[bench] diagnostics series of {args.series}: {args.series_steps} steps, every "
              f"{args.series_every}", file=sys.stderr, flush=True)
        print(json.dumps({"series": series_run(args.series, args.series_steps, args.series_every)}), flush=True)
        return

    if args.adjoint_only:
        res = {}
        for n in args.adjoint_n:
            print(f"[bench] adjoint timing at {n}^2", file=sys.stderr, flush=True)
            res[str(n)] = adjoint_timing(n=n, steps=args.adjoint_steps, kind=args.adjoint_kind)
        print(json.dumps({"adjoint": res}), flush=True)
        return

    print(f"[bench] building workload {args.workload}", file=sys.stderr, flush=True)
    w = build_workload(args.workload)
    print(f"[bench] timing {args.steps} steps after {args.warmup} warm-up steps", file=sys.stderr, flush=True)
    cfg, wall, kernel_ms, diag, resident = time_gpu(w, args.steps, args.warmup)
    if diag["nan_count"] != 0:
        print(json.dumps({"error": "non-finite state after the timed steps"}))
        sys.exit(1)
    nodes = cfg.nodes
    mlups = nodes * args.steps / wall / 1e6
    bpu = bytes_per_update(cfg)
    achieved = bpu * nodes / (kernel_ms * 1e-3) / 1e9

    print("[bench] measuring the copy ceiling", file=sys.stderr, flush=True)
    ceiling = copy_ceiling()

    extra = {}
    if not args.no_extra and args.workload == "sediment_3d_256":
        for prec in ("bf16", "fp16"):
            print(f"[bench] timing the {prec} storage variant", file=sys.stderr, flush=True)
            w16 = build_workload(f"sediment_3d_256_{prec}")
            c16, wall16, kms16, d16, _ = time_gpu(w16, args.steps, args.warmup)
            extra[f"{prec}_store"] = {
                "MLUPS": round(c16.nodes * args.steps / wall16 / 1e6, 1),
                "bytes_per_update": bytes_per_update(c16),
                "kernel_ms": round(kms16, 4),
                "GBps": round(bytes_per_update(c16) * c16.nodes / (kms16 * 1e-3) / 1e9, 1),
            }

    if not args.no_extra and args.workload == "sediment_3d_256":
        # model variants (collision operators, variable density, the paper's lattices)
        variants = {}
        for name in ("sediment_3d_256_trt", "sediment_3d_256_mrt", "sediment_3d_256_vd", "sediment_3d_256_kappa",
                     "ostwald_paper_2d_4096", "ostwald_paper_2d_4096_bf16"):
            print(f"[bench] timing the variant {name}", file=sys.stderr, flush=True)
            wv = build_workload(name)
            cv, wallv, kmsv, _, _ = time_gpu(wv, args.steps, args.warmup)
            variants[name] = {
                "MLUPS": round(cv.nodes * args.steps / wallv / 1e6, 1),
                "bytes_per_update": bytes_per_update(cv),
                "kernel_ms": round(kmsv, 4),
                "GBps": round(bytes_per_update(cv) * cv.nodes / (kmsv * 1e-3) / 1e9, 1),
            }
        extra["variants"] = variants

    if not args.no_extra:
        print("[bench] timing the adjoint (forward, recompute + backward)", file=sys.stderr, flush=True)
        extra["adjoint"] = adjoint_timing()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    out = {
        "metric": "MLUPS coupled step",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}.get(cfg.precision, "f32"),
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": [cfg.nx, cfg.ny, cfg.nz],
            "lattices": f"{cfg.fluid or 'none'} + 3x{cfg.scalar}",
            "storage": cfg.precision,
            "boundaries": list(cfg.bc),
            "parallelism": "single GPU",
            "resident_bytes": resident,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic(args.workload, kernel_sources_sha()),
            "kernel": "k_lbm (fused step)",
            "bytes_per_update": bpu,
            "kernel_ms": round(kernel_ms, 4),
            "copy_ceiling_GBps": round(ceiling, 1),
            "frac_of_copy_ceiling": round(achieved / ceiling, 4),
        },
        "cpu_baseline": cpu,
    }
    if extra:
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

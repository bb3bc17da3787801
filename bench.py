"""Throughput of the fused coupled LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload spinodal_3d_512_bf16]

Prints one JSON line.  A step is one pass of the whole hot path (scalar moments with
the phi predictor, LDS-staged grad/lap phi, capillary + buoyancy force, collision of
f, g, h^A, h^B, streaming with periodic or bounce-back boundaries) over every node of
the workload.  The default workload is the largest single-GPU configuration: a 512^3
periodic box, D3Q19 + 3 x D3Q7, BF16 moving populations with FP32 compute, buoyancy
with the mean subtracted.  `value` is million lattice-node updates per second over the
timed steps with all inputs resident in HBM.  `roofline` prices the fused step kernel
against the HBM peak with its algorithmic bytes (every population read once and
written once per update) and against the measured 1:1 read/write stream ceiling of
the library's streaming probe.  `cpu_baseline` is the FP64 numpy oracle on a bounded
crop of the same workload, at one thread and on all host cores (one independent crop
per core), timed before the GPU is touched.
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
    "spinodal_3d_256_bf16": dict(kind="spinodal_3d", n=256, precision="bf16"),
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


def stream_ceiling(mib=2048, reps=5, grids=(1024, 2048, 4096, 8192, 16384, 65536)):
    """Measured HBM ceilings from the library's streaming probe (lbm_probe_stream:
    16-byte non-temporal loads and stores, grid-stride loop), best over a sweep of grid
    sizes: copy (1:1 read/write, the pattern of a step; read + write bytes per second),
    read only and write only, in GB/s, on buffers of `mib` MiB each."""
    import ctypes
    import torch
    from paper_2409_03401_amd import lbm as L
    n = mib * (1 << 20)
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    out = {}
    for mode, name, factor in ((0, "copy", 2), (1, "read", 1), (2, "write", 1)):
        best, best_grid = 0.0, None
        for grid in grids:
            def launch():
                L._check(L.lib().lbm_probe_stream(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                                  ctypes.c_size_t(n), mode, grid, ctypes.c_void_p(stream.cuda_stream)))
            launch()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                launch()
            e1.record(stream)
            torch.cuda.synchronize()
            gbs = factor * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
            if gbs > best:
                best, best_grid = gbs, grid
        out[name] = {"GBps": round(best, 1), "grid": best_grid}
    del a, b
    torch.cuda.empty_cache()
    return out


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
        if name.endswith((".hpp", ".hip")) and name != "probe.hip":
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def _oracle_crop_worker(args):
    """Step the oracle on a 64^3 crop of the workload recipe for about budget_s;
    returns (node updates, seconds).  Runs in its own process for the all-core leg."""
    name, budget_s = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import lbm as olbm
    w = _crop_workload(name)
    prm = olbm.Params(**w.params)
    st = olbm.init(w.phi0, w.muA0, w.muB0, prm, c0=w.c0)
    st = olbm.step(st, prm)  # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        st = olbm.step(st, prm)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s and n >= 3:
            return w.nodes * n, el, n


def _crop_workload(name):
    """The 64^3 crop of a 3D workload's recipe that the oracle is timed on."""
    from paper_2409_03401_amd import inputs
    if WORKLOADS[name]["kind"] == "spinodal_3d":
        return inputs.spinodal_3d(n=64)
    return inputs.sediment_3d(n=64, ndrops=4, rmin=10.0, rmax=14.0)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(name, budget_s=10.0, max_workers=16):
    """The oracle as it stands (FP64 numpy, never tuned for this) on a 64^3 crop of the
    workload's recipe: one process on one thread, then one independent crop per host
    core (up to max_workers processes, the machine's CPU share) stepping at once.  Must run
    before the GPU is touched (the pool forks)."""
    import multiprocessing as mp
    upd, el, n = _oracle_crop_worker((name, budget_s))
    single = upd / el / 1e6
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    workers = max(1, min(cores, max_workers))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_crop_worker, [(name, budget_s)] * workers)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    allcore = total / wall / 1e6
    crop = "spinodal box" if WORKLOADS[name]["kind"] == "spinodal_3d" else "sediment workload"
    return {"value": round(allcore, 3), "unit": "MLUPS", "cores": workers, "kind": "oracle",
            "single_thread": {"value": round(single, 3), "unit": "MLUPS", "cores": 1, "steps": n},
            "sample": f"64^3 crop of the {crop} recipe, D3Q19 + 3xD3Q7, FP64 numpy oracle; "
                      f"1 thread: {n} steps in {el:.1f} s; all cores: {workers} processes, one crop each, "
                      f"{total / 64 ** 3:.0f} crop-steps in {wall:.1f} s; host {_cpu_model()}, "
                      f"{cores} logical CPUs available"}


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


def variant_line(name, steps, warmup):
    """Throughput line of one more workload (same timing as the headline)."""
    print(f"[bench] timing {name}", file=sys.stderr, flush=True)
    w = build_workload(name)
    c, wall, kms, d, _ = time_gpu(w, steps, warmup)
    bpu = bytes_per_update(c)
    return {"MLUPS": round(c.nodes * steps / wall / 1e6, 1), "bytes_per_update": bpu,
            "kernel_ms": round(kms, 4), "GBps": round(bpu * c.nodes / (kms * 1e-3) / 1e9, 1),
            "nan_count": int(d["nan_count"])}


# extra throughput lines of the default run: the sedimentation workload at the three
# storage precisions, the model variants, the paper's own discretisation
EXTRA_LINES = ("sediment_3d_256", "sediment_3d_256_bf16", "sediment_3d_256_fp16", "sediment_3d_256_trt",
               "sediment_3d_256_mrt", "sediment_3d_256_vd", "sediment_3d_256_kappa", "ostwald_paper_2d_4096",
               "ostwald_paper_2d_4096_bf16")

NORTH_STAR_FRAC = 0.70   # the forward-step bandwidth target, as a fraction of the HBM peak


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="spinodal_3d_512_bf16", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workload lines and the adjoint timing")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the differentiable run (forward, backward, ratio)")
    ap.add_argument("--adjoint-n", type=int, nargs="+", default=[512, 2048],
                    help="grid sizes n (n x n) of the adjoint timing")
    ap.add_argument("--adjoint-steps", type=int, default=4096)
    ap.add_argument("--adjoint-kind", default="single_drop_2d", choices=["single_drop_2d", "sediment_3d"])
    ap.add_argument("--series", default=None, choices=sorted(WORKLOADS),
                    help="only record the diagnostics time series of a workload (droplet count, <R>, max |u|)")
    ap.add_argument("--series-steps", type=int, default=20000)
    ap.add_argument("--series-every", type=int, default=500)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to scale HBM counters")
    ap.add_argument("--box", type=int, nargs=3, default=None, metavar=("NX", "NY", "NZ"),
                    help="only time the sedimentation recipe (walls in z) on an NX x NY x NZ box")
    ap.add_argument("--box-precision", default="fp32", choices=["fp64", "fp32", "bf16", "fp16"])
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

    # the oracle's timing forks a process per core: it runs before the GPU is touched
    cpu = None
    if not (args.no_cpu_baseline or args.series or args.adjoint_only or args.box):
        print("[bench] timing the CPU oracle (one thread, then all cores)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload)

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

    if args.box:
        from paper_2409_03401_amd import inputs
        nx, ny, nz = args.box
        print(f"[bench] sedimentation box {nx} x {ny} x {nz}, {args.box_precision}", file=sys.stderr, flush=True)
        # droplet count scaled with the volume (64 in 256^3)
        w = inputs.sediment_3d(n=nx, ny=ny, nz=nz, precision=args.box_precision,
                               ndrops=max(4, nx * ny * nz // 262144))
        cfg, wall, kernel_ms, diag, _ = time_gpu(w, args.steps, args.warmup)
        print(json.dumps({"box": [nx, ny, nz], "precision": args.box_precision,
                          "MLUPS": round(cfg.nodes / (kernel_ms * 1e-3) / 1e6, 1), "kernel_ms": round(kernel_ms, 4),
                          "bytes_per_update": bytes_per_update(cfg), "nan_count": diag["nan_count"]}), flush=True)
        return

    print(f"[bench] building workload {args.workload}", file=sys.stderr, flush=True)
    w = build_workload(args.workload)
    print(f"[bench] timing {args.steps} steps after {args.warmup} warm-up steps", file=sys.stderr, flush=True)
    cfg, wall, kernel_ms, diag, resident = time_gpu(w, args.steps, args.warmup)
    del w
    if diag["nan_count"] != 0:
        print(json.dumps({"error": "non-finite state after the timed steps"}))
        sys.exit(1)
    nodes = cfg.nodes
    mlups = nodes * args.steps / wall / 1e6
    bpu = bytes_per_update(cfg)
    achieved = bpu * nodes / (kernel_ms * 1e-3) / 1e9

    print("[bench] measuring the streaming ceilings", file=sys.stderr, flush=True)
    ceilings = stream_ceiling()
    copy_gbs = ceilings["copy"]["GBps"]

    extra = {}
    if not args.no_extra:
        extra["lines"] = {name: variant_line(name, args.steps, args.warmup)
                          for name in EXTRA_LINES if name != args.workload}
        adj = {}
        for n in args.adjoint_n:
            print(f"[bench] timing the adjoint at {n}^2 (forward, recompute + backward)", file=sys.stderr,
                  flush=True)
            adj[str(n)] = adjoint_timing(n=n, steps=args.adjoint_steps)
        extra["adjoint"] = adj

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
        "dtype": {"fp64": "f64"}.get(cfg.precision, "f32"),
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
            "stream_ceilings_GBps": ceilings,
            "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
            "target_frac": NORTH_STAR_FRAC,
            "gap_to_target_GBps": round(NORTH_STAR_FRAC * HBM_PEAK_GBS - achieved, 1),
            "copy_ceiling_frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
        },
        "cpu_baseline": cpu,
    }
    if extra:
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

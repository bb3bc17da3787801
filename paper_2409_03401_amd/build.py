"""Build liblbm.so (the HIP library behind include/lbm.h) in-tree for gfx950.

    python -m paper_2409_03401_amd.build

compiles every source under csrc/ with hipcc and links them into
paper_2409_03401_amd/liblbm.so.  Cross-compiles without a GPU.
"""

import os
import subprocess
import tempfile
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "liblbm.so")
BUILD_DIR = os.path.join(PKG, "_build")

# the longest compiles first, so that the parallel build ends together
SOURCES = ["lbm_mrt_3d_q19_flow_fp.hip", "lbm_mrt_3d_q19_flow_16.hip", "lbm_mrt_3d_q19.hip", "lbm_gk_3d.hip",
           "lbm_trt_3d.hip", "lbm_mrt_2d.hip", "lbm_paper_3d.hip", "lbm_3d.hip", "lbm_2d.hip", "lbm_trt_2d.hip",
           "lbm_gk_2d.hip", "lbm_vd_3d.hip", "lbm_mrt_3d.hip", "lbm_paper_2d.hip", "lbm_vd_2d.hip", "lbm_api.hip",
           "probe.hip", "lbm_nc3_3d.hip", "lbm_nc3_2d.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, out: str = OUT, extra_flags=()) -> str:
    """Compile and link.  `extra_flags` are appended to every hipcc line (for
    tuning builds, e.g. -DLBM_WAVES_PER_EU=3); `out` is the library path."""
    build_dir = BUILD_DIR if out == OUT else out + ".build"
    os.makedirs(build_dir, exist_ok=True)
    t0 = time.time()
    objs = []
    # at most `jobs` compilers at once (each large translation unit takes a few GB)
    jobs = max(1, min(int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 4), 8))
    pending = list(SOURCES)
    running = []
    failed = []

    # each compiler writes its messages to a file of its own: a pipe read only after the
    # compiler exits would block it once the messages fill the pipe buffer
    def reap(entry):
        src, p, log = entry
        p.wait()
        log.seek(0)
        text = log.read().decode(errors="replace")
        log.close()
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)

    for src in SOURCES:
        objs.append(os.path.join(build_dir, src.replace(".hip", ".o")))
    while pending or running:
        while pending and len(running) < jobs:
            src = pending.pop(0)
            obj = os.path.join(build_dir, src.replace(".hip", ".o"))
            cmd = [HIPCC, *CFLAGS, *extra_flags, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            log = tempfile.TemporaryFile()
            running.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
        done = [e for e in running if e[1].poll() is not None]
        if not done:
            time.sleep(0.2)
            continue
        for e in done:
            running.remove(e)
            reap(e)
    if failed:
        msg = "\n".join(f"--- {s} ---\n{t}" for s, t in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = out + ".tmp"
    link = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} in {time.time() - t0:.1f} s", flush=True)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("-q", action="store_true")
    ap.add_argument("--out", default=OUT)
    ap.add_argument("flags", nargs="*", help="extra hipcc flags, e.g. -DLBM_WAVES_PER_EU=3")
    a = ap.parse_args()
    build(verbose=not a.q, out=os.path.abspath(a.out), extra_flags=a.flags)

"""The benchmark's contract, checked on the CPU: more than one GPU is refused with a
message, the algorithmic bytes per update follow from a count of the stored populations,
and every committed profile summary that carries a kernel-source hash was taken on the
current kernel sources (so the traffic figure the benchmark quotes from it is live)."""

import glob
import json
import os
import re
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 2, r.stderr[-2000:]
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and "--gpus > 1" in msg["error"]


# Stored populations per node: the fluid lattice (qf, 0 without flow) and three scalar
# lattices of qs directions.  FP32 / FP64 store every population at that width; 16-bit
# storage keeps the rest population of each lattice in FP32 and the moving ones in 16 bits.
# Each population is read once and written once per update.
@pytest.mark.parametrize("precision, qf, qs, expect", [
    ("fp32", 19, 7, 2 * 4 * (19 + 3 * 7)),                     # D3Q19 + 3 x D3Q7: 320
    ("fp64", 19, 7, 2 * 8 * (19 + 3 * 7)),                     # 640
    ("bf16", 19, 7, 2 * (4 * 4 + 2 * (18 + 3 * 6))),            # 176
    ("fp16", 19, 7, 2 * (4 * 4 + 2 * (18 + 3 * 6))),            # 176
    ("fp32", 9, 5, 2 * 4 * (9 + 3 * 5)),                       # D2Q9 + 3 x D2Q5: 192
    ("fp32", 0, 9, 2 * 4 * 3 * 9),                             # 3 x D2Q9, no flow: 216
    ("bf16", 0, 9, 2 * 3 * (4 + 2 * 8)),                       # 120
])
def test_bytes_per_update_counts_the_stored_populations(precision, qf, qs, expect):
    assert bench.bytes_per_update(SimpleNamespace(precision=precision, qf=qf, qs=qs)) == expect


def test_profile_summaries_match_the_kernel_sources():
    sha = bench.kernel_sources_sha()
    found = 0
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        m = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", open(path).read())
        if m:
            found += 1
            assert m.group(1) == sha, f"{os.path.basename(path)} was taken on other kernel sources"
    assert found >= 1

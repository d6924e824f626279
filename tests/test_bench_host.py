"""Host-side checks of the benchmark driver and of the committed counter
summaries it reads (no GPU needed)."""
import glob
import json
import os
import subprocess
import sys

from paper_2508_15967_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def _entries(pattern):
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", pattern))):
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        out.append((os.path.basename(path), kv))
    return out


def test_counter_summaries_are_well_formed():
    """Every traffic_/fp64_ file names a benchmark kernel and workload (as its
    file name does), a 16-hex-digit source hash and positive figures; the
    HBM total is the sum of the read and write bytes."""
    names = {W.make(c, 1).name for c in ("1", "2", "3", "4", "5", "cp")}
    names |= {W.coldplasma("O").name, W.coldplasma("X").name}
    kernels = {"rg_rk4_r1", "rg_rk4_r2", "rg_rk4_r4", "rg_rk4_r1o4", "rg_rk4_adjoint", "rg_dopri_persistent"}
    traffic, fp64 = _entries("traffic_*.txt"), _entries("fp64_*.txt")
    assert traffic and fp64
    for fname, kv in traffic + fp64:
        assert kv["kernel"] in kernels and kv["workload"] in names, fname
        assert fname.endswith(f"_{kv['kernel']}_{kv['workload']}.txt"), fname
        assert len(kv["source_hash"]) == 16 and int(kv["source_hash"], 16) >= 0, fname
    for fname, kv in traffic:
        f, w, t = (int(kv[k]) for k in ("fetch_bytes_per_launch", "write_bytes_per_launch", "hbm_bytes_per_launch"))
        assert f > 0 and w > 0 and t == f + w, fname
    for fname, kv in fp64:
        assert float(kv["fp64_flops_per_ray_step"]) > 0 and float(kv["valu_per_wave_step"]) > 0, fname

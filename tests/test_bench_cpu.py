"""The benchmark's host-side pieces, on the CPU: its Table B.1 split agrees
with the oracle's, its per-cell algorithmic bytes and flops are the counts
of the method's cost model worked out by hand for the workloads, more than
one GPU is refused before anything touches a device, and every committed
rocprofv3 summary that records a source hash was taken on the current
kernel sources (otherwise its traffic figure is stale)."""
import glob
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_table_split_matches_the_oracle(orc):
    for k in range(1, 10):
        m, q, r, _ = orc.table_row(k)
        assert (bench.TABLE_Q[k], bench.TABLE_R[k]) == (q, r), k
        assert q * r >= m


@pytest.mark.parametrize("C,N,D,per_cell", [(4096, 1, 1, 56), (1 << 20, 4, 3, 312),
                                            (1 << 20, 16, 3, 1080), (1 << 18, 8, 3, 568)])
def test_algorithmic_bytes(C, N, D, per_cell):
    # read rho_g, N densities, N stopping times, D (N + 1) velocities; write D (N + 1)
    assert bench.algorithmic_bytes(C, N, D) == 8.0 * C * (1 + 2 * N + 2 * D * (N + 1))
    assert bench.algorithmic_bytes(C, N, D) == per_cell * C


def test_algorithmic_flops_of_the_stiff_cell():
    # N = 16 (n = 17), k* = 7 (m = 20, q = 4, r = 5), s = 20, D = 3:
    # (r - 1 + s) 2 n^3 = 24 * 9826 = 235824; (q - 1) 2 n (3 n - 2) = 3 * 1666 = 4998;
    # 2 m n^2 = 11560; 2 D n^2 = 1734; total 254116
    f = bench.algorithmic_flops(np.array([7]), np.array([20]), np.array([20]), 16, 3)
    assert float(f[0]) == 254116.0
    # N = 1 (n = 2), k* = 1 (m = 2, q = 1, r = 2), s = 0, D = 1: 16 + 0 + 16 + 8
    f = bench.algorithmic_flops(np.array([1]), np.array([2]), np.array([0]), 1, 1)
    assert float(f[0]) == 40.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_forward_kernel_names():
    assert bench.forward_kernel(16, "wave", 1 << 20) == "k_forward_wave"
    assert bench.forward_kernel(20, "wave", 1 << 18) == "k_forward_big"
    assert bench.forward_kernel(4, "lane", 1 << 20) == "k_forward_lane"
    assert bench.forward_kernel(6, "lane", 1 << 20) == "k_forward_lane"
    assert bench.forward_kernel(7, "lane", 1 << 20) == "k_forward_lane_stream"
    assert bench.forward_kernel(8, "lane", 1 << 18) == "k_forward_lane_stream"
    assert bench.forward_kernel(8, "lane", 1 << 29) == "k_forward_lane"
    assert bench.forward_kernel(10, "lane", 1 << 18) == "k_forward_pair"


def _profiles_with_hash():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        fields = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and line.split(":")[0] in ("source_sha256", "hbm_bytes_per_launch"):
                    k, v = line.split(":", 1)
                    fields[k] = v.strip()
        if "source_sha256" in fields:
            base = os.path.basename(path)[:-3]
            kernel = max((k for k in bench.KERNEL_SOURCES if base.startswith(k + "_")), key=len)
            out.append((os.path.basename(path), kernel, base[len(kernel) + 1:], fields))
    return out


@pytest.mark.parametrize("name,kernel,workload,fields", _profiles_with_hash(),
                         ids=[p[0] for p in _profiles_with_hash()])
def test_profile_summaries_match_the_sources(name, kernel, workload, fields):
    assert fields["source_sha256"] == bench.source_hash(kernel), name
    assert float(fields["hbm_bytes_per_launch"]) > 0
    assert bench.profiled_traffic(kernel, workload) == float(fields["hbm_bytes_per_launch"])


def test_side_measurements_fail_in_place():
    """A child that cannot measure (here: no GPU) costs only the side keys,
    each an error entry, never the caller's line."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("the failure path needs a process without a GPU")
    res = bench._side_in_child(timeout_s=300)
    assert set(res) == set(bench.SIDE_KEYS)
    for key in bench.SIDE_KEYS:
        assert "error" in res[key], key

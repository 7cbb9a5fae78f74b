"""GPU parity of the one-lane forward's load schedules: the streaming kernel
(N = 7, 8) at sizes past one pass of the resident grid, where every
wavefront walks several cells and loads the next cell's inputs while it
computes the current one, and the one-shot kernel that issues all of a
cell's loads before the exponential (N = 1, 2, 4, 5, 6).  Ragged tails, one to
three velocity components, a padded leading dimension, in place, and bad
cells placed in different passes.  Same bars as the other parity tests
(``tests/bars.py``: 1e-13 against the exact exponential, 1e-13 +
e(oracle, exact) against the oracle per cell; momentum 1e-12).
"""
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W
from bars import check_forward
from test_parity_gpu import run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_25347_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ops(dev):
    from paper_2509_25347_amd import ops as _ops
    return _ops


def _make(N, cells, D):
    return W.make_stiff(N, cells, D=D) if N % 2 == 0 else W.make_jittered(N, cells, D=D)


@pytest.mark.parametrize("N,D,cells", [(5, 3, 300_007), (6, 2, 270_001), (7, 1, 200_003),
                                       (7, 3, 300_007), (8, 2, 150_001), (8, 3, 200_003),
                                       (1, 1, 50_001), (2, 3, 70_001), (4, 2, 100_003),
                                       (4, 3, 65_536)])
def test_multi_pass_parity(ops, dev, orc, N, D, cells):
    d = _make(N, cells, D)
    ref, kms, nrm, st = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"])
    print(f"stream parity N={N} D={D} cells={cells}", flush=True)
    got = run(ops, d, dev)
    check_forward(orc, got, ref, d, f"N={N} D={D}")


@pytest.mark.parametrize("N", [1, 4, 6, 7, 8])
def test_in_place_and_padded_ld_bit_equal(ops, dev, N):
    cells, ld = 150_001, 150_080
    d = _make(N, cells, 3)
    T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("rho_g", "rho_d", "t_stop", "v")}
    print(f"stream in place / padded ld N={N}", flush=True)
    base = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    inplace = T["v"].clone()
    ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], inplace, d["dt"], out=inplace)

    def padded(x):
        p = torch.full(x.shape[:-1] + (ld,), float("nan"), dtype=x.dtype, device=dev)
        p[..., :cells] = x
        return p[..., :cells]

    rd, ts, v = padded(T["rho_d"]), padded(T["t_stop"]), padded(T["v"])
    out = padded(torch.zeros_like(T["v"]))
    ops.expm_apply(T["rho_g"], rd, ts, v, d["dt"], out=out)
    torch.cuda.synchronize()
    assert torch.equal(base, inplace)
    assert torch.equal(base, out)


def test_bad_cells_in_different_passes(ops, dev, orc):
    N, cells = 8, 200_003
    d = _make(N, cells, 3)
    rg, rd, ts, v = (d[k].copy() for k in ("rho_g", "rho_d", "t_stop", "v"))
    bad = {5: "rho_g", 70_000: "t", 140_001: "v", cells - 1: "rho_d"}
    rg[5] = 0.0
    ts[3, 70_000] = np.nan
    v[2, 4, 140_001] = np.inf
    rd[7, cells - 1] = -1.0
    ref, kms, nrm, st = orc.apply_cells(rg, rd, ts, v, d["dt"])
    print("stream bad cells N=8", flush=True)
    ops.clear_status()
    got = run(ops, dict(rho_g=rg, rho_d=rd, t_stop=ts, v=v, dt=d["dt"]), dev)
    status = ops.get_status()
    assert status == st == (orc.BAD_DENSITY | orc.BAD_STOPPING_TIME | orc.BAD_VELOCITY)
    for c in bad:
        assert np.isnan(got[:, :, c]).all(), c
    check_forward(orc, got, ref, dict(rho_g=rg, rho_d=rd, t_stop=ts, v=v, dt=d["dt"]),
                  "stream bad cells")


def test_first_call_under_graph_capture(dev):
    """The streaming launch asks the runtime for its occupancy on first use;
    a process whose very first library call is captured into a HIP graph
    (N = 7, so that path) must replay to the eager result bit for bit."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = f"""
import sys
sys.path.insert(0, {root!r})
import numpy as np, torch
from paper_2509_25347_amd import ops, workloads as W
dev = torch.device("cuda:0")
d = W.make_jittered(7, 70_001)
T = {{k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}}
o = torch.full_like(T["v"], float("nan"))
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g):
    ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], out=o)
for _ in range(3):
    o.fill_(float("nan"))
    g.replay()
    torch.cuda.synchronize()
    ref = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    torch.cuda.synchronize()
    assert torch.equal(o, ref)
print("ok", flush=True)
"""
    print("stream first call under capture (subprocess)", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=150)
    assert r.returncode == 0 and "ok" in r.stdout, (r.returncode, r.stdout[-1000:], r.stderr[-3000:])


@pytest.mark.parametrize("N", [1, 3, 4, 6, 7, 8, 9, 11, 13, 16])
def test_results_do_not_depend_on_the_launch(ops, dev, N):
    """Cells are independent: the first 3001 cells of a 200_003-cell launch
    (several passes of the streaming grid, or a large one-shot grid) carry
    the same bits as a launch of those 3001 cells alone, and a second launch
    repeats the first bit for bit."""
    d = _make(N, 200_003, 3)
    T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("rho_g", "rho_d", "t_stop", "v")}
    print(f"launch independence N={N}", flush=True)
    full = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    again = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    k = 3001
    sub = {n: T[n][..., :k].contiguous() for n in T}
    part = ops.expm_apply(sub["rho_g"], sub["rho_d"], sub["t_stop"], sub["v"], d["dt"])
    torch.cuda.synchronize()
    assert torch.equal(full, again)
    assert torch.equal(full[..., :k], part)


@pytest.mark.parametrize("N", [3, 6, 8, 10, 12])
def test_adjoint_does_not_depend_on_the_launch(ops, dev, N):
    """The fused forward + adjoint of the first 2001 cells of a 100_003-cell
    launch equals that of a launch of those cells alone, bit for bit, and a
    second launch repeats the first."""
    d = _make(N, 100_003, 3)
    w = np.random.default_rng(N).standard_normal(d["v"].shape)
    T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("rho_g", "rho_d", "t_stop", "v")}
    T["w"] = torch.from_numpy(w).to(dev)
    print(f"adjoint launch independence N={N}", flush=True)

    def run_bwd(X):
        return ops.expm_apply_backward(X["rho_g"], X["rho_d"], X["t_stop"], X["v"], X["w"],
                                       d["dt"])

    full, again = run_bwd(T), run_bwd(T)
    k = 2001
    part = run_bwd({n: T[n][..., :k].contiguous() for n in T})
    torch.cuda.synchronize()
    for a, b, p in zip(full, again, part):
        if a is None:
            continue
        assert torch.equal(a, b)
        assert torch.equal(a[..., :k], p)


@pytest.mark.parametrize("N", [7, 8])
@pytest.mark.parametrize("cells", [1, 63, 64, 65, 257, 65_536, 65_537, 131_073])
def test_stream_sizes_at_the_pass_boundaries(ops, dev, orc, N, cells):
    """Sizes around a wavefront, a workgroup and one or two passes of the
    resident grid (65 536 cells at one wavefront per SIMD on 256 CUs)."""
    d = _make(N, cells, 3)
    ref, kms, nrm, st = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"])
    print(f"stream sizes N={N} cells={cells}", flush=True)
    got = run(ops, d, dev)
    check_forward(orc, got, ref, d, f"N={N} cells={cells}")


@pytest.mark.parametrize("N", [4, 8])
def test_arrays_past_32_bit_offsets(ops, dev, N):
    """Arrays whose byte span passes 2^32 (here by a large leading dimension)
    leave the one-lane kernels' 32-bit buffer offsets for the 64-bit
    addressed one-shot kernel: the same cells give the same bits as in a
    compact layout (about 20 GB of device memory, only the first cells of
    each row written)."""
    d = _make(N, 1000, 1)
    C = 1000
    ld = (1 << 32) // (8 * N) + 64  # 8 (N ld + C) > 2^32 for the velocity rows
    print(f"32-bit offsets N={N} ld={ld}", flush=True)
    T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("rho_g", "rho_d", "t_stop", "v")}
    ref = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    big = {}
    for k in ("rho_d", "t_stop", "v"):
        full = torch.empty(tuple(T[k].shape[:-1]) + (ld,), dtype=torch.float64, device=dev)
        full[..., :C] = T[k]
        big[k] = full[..., :C]
    out = ops.expm_apply(T["rho_g"], big["rho_d"], big["t_stop"], big["v"], d["dt"])
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    del big, out
    torch.cuda.empty_cache()

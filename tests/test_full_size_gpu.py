"""The full-size workloads in the launch configuration the benchmark times
(the same ops calls, default mapping and Taylor cap), against the oracle:

* every cell of the N = 1 (4096 cells), N = 4 (2^20) and N = 8 (2^18)
  forwards, to the parity bars of ``tests/bars.py`` (1e-13 against the exact
  exponential on every cell; 1e-13 + e(oracle, exact) against the oracle,
  1e-13 outright on the N = 1 cells; momentum 1e-12);
* the fused forward + adjoint of the N = 8 workload: the oracle's gradients on
  sampled cells (including the first and last), and on every cell the sum
  rule of the velocity gradient (E 1 = 1, so the entries of E^T w sum to
  those of w) and the fused forward equal to the plain one.
"""
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W
from test_adjoint_gpu import check_vs_oracle, group_err
from bars import check_forward

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


def _sample(C, n=1024, seed=0):
    return np.unique(np.concatenate([np.arange(32), np.arange(C - 32, C),
                                     np.random.default_rng(seed).integers(0, C, n)]))


def _sub(d, idx):
    return {k: (d[k][..., idx] if k != "dt" else d[k]) for k in d}


@pytest.mark.parametrize("name", ["n1_closed_form", "n4_3d", "n8_adjoint_3d"])
def test_full_size_forward_every_cell(ops, dev, orc, name):
    d = W.make(name)
    T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("rho_g", "rho_d", "t_stop", "v")}
    print(f"full-size forward {name}", flush=True)
    ops.clear_status()
    out = torch.empty_like(T["v"])
    ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"], out=out)
    torch.cuda.synchronize()
    assert ops.get_status() == 0
    got = out.cpu().numpy()
    ref, kms, nrm, st = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"])
    assert st == 0
    e_go, e_gx, e_ox = check_forward(orc, got, ref, d, name, tight=name == "n1_closed_form")
    print(f"{name}: max e vs oracle {e_go.max():.2e}, vs exact {e_gx.max():.2e}, "
          f"oracle vs exact {e_ox.max():.2e}", flush=True)


def test_full_size_adjoint(ops, dev, orc):
    d = W.make("n8_adjoint_3d", with_weights=True)
    T = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("rho_g", "rho_d", "t_stop", "v", "w")}
    print("full-size adjoint n8_adjoint_3d", flush=True)
    ops.clear_status()
    res = ops.expm_apply_backward(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], T["w"], d["dt"],
                                  want_grad_t=True)
    fwd = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    torch.cuda.synchronize()
    assert ops.get_status() == 0
    got = [None if x is None else x.cpu().numpy() for x in res]
    v_out, g_v = got[0], got[1]
    assert all(np.isfinite(x).all() for x in got if x is not None)
    # the fused forward is the plain forward, every cell
    assert group_err(v_out, fwd.cpu().numpy()).max() <= 1e-13
    # sum rule on every cell: sum_j (E^T w)_j = sum_j w_j per component
    w = d["w"]
    dev_sum = np.abs(g_v.sum(axis=1) - w.sum(axis=1))
    assert (dev_sum <= 1e-12 * np.abs(w).sum(axis=1) + 1e-300).all(), dev_sum.max()
    # the oracle's reverse-mode gradient on a sample
    idx = _sample(len(d["rho_g"]), n=2048, seed=1)
    check_vs_oracle(orc, _sub(d, idx), [None if x is None else x[..., idx] for x in got], 1e-10,
                    "n8_adjoint_3d full size")

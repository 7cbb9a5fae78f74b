"""The Collisions tests B and C (Sect. 3, Table 1) as a drag-only time
integration on the GPU (drag_expm_steps): one gas and two dust fluids
relaxing to the centre-of-mass velocity.

Er_1 (the error measure of the Collisions convergence study, eq. Error1_eq:
the mean over the M steps of sum over fluids of |v~ - v| / v at each step's
time) is computed for every time step of the paper's sweep (Delta t doubling
from 1e-4 for B and 1e-3 for C up to t_final = 0.1 and 2) against the exact
solution from the long-double eigen decomposition (oracle/truth.c).  The
paper reports Er_1 ~ 1e-8, flat in Delta t, for its EXP integrator; here it
is 1e-16 .. 2.5e-15 (printed with pytest -s).  The
trajectory is also checked against the analytic solution printed in Table 1
(five decimals; tests/golden/collisions_table1.txt) and against the oracle
integrated step by step.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_25347_amd import _lib, ops as _ops
    _lib.lib()
    return _ops


def table1():
    cols = {"B": {}, "C": {}}
    for line in open(os.path.join(HERE, "golden", "collisions_table1.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, b, c = line.split()
        cols["B"][k], cols["C"][k] = float(b), float(c)
    return cols


SWEEP = {"B": (1e-4, 0.1), "C": (1e-3, 2.0)}


def case_arrays(t):
    rho_g = np.array([t["rho_g"]])
    rho_d = np.array([[t["rho_d1"]], [t["rho_d2"]]])
    t_stop = np.array([[t["T_s1"]], [t["T_s2"]]])
    v = np.array([[[t["v_g"]], [t["v_d1"]], [t["v_d2"]]]])  # [D=1][N+1=3][C=1]
    return rho_g, rho_d, t_stop, v


@pytest.mark.parametrize("case", ["B", "C"])
def test_collisions_er1_sweep(ops, case):
    import oracle
    t = table1()[case]
    rho_g, rho_d, t_stop, v0 = case_arrays(t)
    dev = torch.device("cuda:0")
    T = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (rho_g, rho_d, t_stop, v0)]
    dt0, t_final = SWEEP[case]
    er1 = {}
    j = 0
    while dt0 * 2 ** j <= t_final * (1 + 1e-12):
        dt = dt0 * 2 ** j
        M = int(np.floor(t_final / dt * (1 + 1e-12)))
        out, hist = ops.expm_steps(*T, dt, M, history=True)
        got = hist.cpu().numpy()[:, 0, :, 0]  # [M][3]
        assert np.array_equal(out.cpu().numpy()[0, :, 0], got[-1])
        err = 0.0
        for i in range(M):
            E = oracle.truth_eigen((i + 1) * dt, rho_g[0], rho_d[:, 0], t_stop[:, 0])
            exact = E @ v0[0, :, 0]
            err += np.sum(np.abs(got[i] - exact) / np.abs(exact))
        er1[dt] = err / M
        j += 1
    assert len(er1) >= 10
    print(f"Er_1 {case}: " + ", ".join(f"dt={k:.4g}: {v:.3g}" for k, v in er1.items()))
    worst = max(er1.values())
    # the paper's EXP: ~1e-8, flat in Delta t.  Measured on MI355X: 1e-16 .. 2.5e-15 for
    # every Delta t of both sweeps (flat as well), so the bar leaves a 40x margin
    assert worst <= 1e-13, er1


@pytest.mark.parametrize("case", ["B", "C"])
def test_collisions_against_table1_and_oracle(ops, case):
    """At t = 40 dt (the paper's fixed-step figure: dt = 0.005 for B, 0.05 for
    C) the GPU integration matches the printed analytic solution to its five
    decimals and the oracle's own 40-step integration to rounding."""
    import oracle
    t = table1()[case]
    rho_g, rho_d, t_stop, v0 = case_arrays(t)
    dt = {"B": 0.005, "C": 0.05}[case]
    dev = torch.device("cuda:0")
    T = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (rho_g, rho_d, t_stop, v0)]
    out, hist = ops.expm_steps(*T, dt, 40, history=True)
    got = hist.cpu().numpy()[:, 0, :, 0]
    lam = np.array([t["lambda_1"], t["lambda_2"]])
    coef = np.array([[t["c_g1"], t["c_g2"]], [t["c_d11"], t["c_d12"]], [t["c_d21"], t["c_d22"]]])
    for i in (0, 9, 39):
        ti = (i + 1) * dt
        analytic = t["V_CM"] + coef @ np.exp(lam * ti)
        np.testing.assert_allclose(got[i], analytic, atol=5e-5)
    v = v0.copy()
    for i in range(40):
        v, _, _, st = oracle.apply_cells(rho_g, rho_d, t_stop, v, dt)
        assert st == 0
        assert np.abs(got[i] - v[0, :, 0]).max() <= 1e-13 * max(1.0, i)


@pytest.mark.parametrize("case", ["B", "C"])
def test_collisions_rk1_first_order(ops, case):
    """The same sweep with the backward Euler step (drag_rk1_apply, stepped in
    place): the trajectory follows the oracle's own RK1 integration to
    rounding, Er_1 halves with Delta t (first order: ratios 1.98, 1.97, 1.94
    for B and 1.98, 1.97, 1.93 for C over the first doublings), and it sits
    ten orders of magnitude above the exponential's at every Delta t."""
    import oracle
    t = table1()[case]
    rho_g, rho_d, t_stop, v0 = case_arrays(t)
    dev = torch.device("cuda:0")
    T = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (rho_g, rho_d, t_stop)]
    dt0, t_final = SWEEP[case]
    er1 = {}
    for j in range(6):
        dt = dt0 * 2 ** j
        M = int(np.floor(t_final / dt * (1 + 1e-12)))
        v = torch.from_numpy(v0.copy()).to(dev)
        states = []
        for i in range(M):
            ops.rk1_apply(*T, v, dt, out=v)
            states.append(v.clone())
        got = torch.stack(states).cpu().numpy()[:, 0, :, 0]
        ref = v0.copy()
        err = 0.0
        for i in range(M):
            ref, st = oracle.rk1_cells(rho_g, rho_d, t_stop, ref, dt)
            assert st == 0
            assert np.abs(got[i] - ref[0, :, 0]).max() <= 32 * 2.0 ** -53 * 2 * (i + 1)
            exact = oracle.truth_eigen((i + 1) * dt, rho_g[0], rho_d[:, 0], t_stop[:, 0]) @ v0[0, :, 0]
            err += np.sum(np.abs(got[i] - exact) / np.abs(exact))
        er1[dt] = err / M
    print(f"RK1 Er_1 {case}: " + ", ".join(f"dt={k:.4g}: {v:.3g}" for k, v in er1.items()))
    e = list(er1.values())
    ratios = [e[i + 1] / e[i] for i in range(3)]
    assert all(1.85 <= r <= 2.05 for r in ratios), ratios
    assert min(e) >= 1e-5


def twenty_species():
    """The 20-species Collisions set-up of Sect. 3.1 (reading: 21 log-spaced
    edges on [1e-3, 10], species i between edges i and i+1 with the geometric
    mean as its stopping time, dust-to-gas ratios from eq. dust_to_gas_ratio
    with total 1; v_g = 1 and the dust velocities spread linearly from 2 to
    0.5, since the paper does not list them)."""
    N = 20
    edges = np.logspace(-3, 1, N + 1)
    ts = np.sqrt(edges[:-1] * edges[1:])
    eps = (np.sqrt(edges[1:]) - np.sqrt(edges[:-1])) / (np.sqrt(edges[-1]) - np.sqrt(edges[0]))
    rho_g = np.array([1.0])
    rho_d = eps[:, None].copy()
    t_stop = ts[:, None].copy()
    v0 = np.concatenate([[1.0], np.linspace(2.0, 0.5, N)])[None, :, None].copy()
    return rho_g, rho_d, t_stop, v0


def test_collisions_twenty_species_er1(ops):
    """N = 20 on the GPU's large-N kernel: Er_1 over a Delta t sweep (1e-3
    doubling to t_final = 1) against the exact solution; the paper reports
    ~1e-7 for this case (with its reference solution), here it stays at
    rounding level."""
    import oracle
    rho_g, rho_d, t_stop, v0 = twenty_species()
    dev = torch.device("cuda:0")
    T = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (rho_g, rho_d, t_stop, v0)]
    er1 = {}
    for jj in range(8):
        dt = 1e-3 * 2 ** jj
        M = int(np.floor(1.0 / dt * (1 + 1e-12)))
        out, hist = ops.expm_steps(*T, dt, M, history=True)
        got = hist.cpu().numpy()[:, 0, :, 0]
        err = 0.0
        for i in range(M):
            E = oracle.truth_eigen((i + 1) * dt, rho_g[0], rho_d[:, 0], t_stop[:, 0])
            exact = E @ v0[0, :, 0]
            err += np.sum(np.abs(got[i] - exact) / np.abs(exact))
        er1[dt] = err / M
    print("Er_1 20 species: " + ", ".join(f"dt={k:.4g}: {v:.3g}" for k, v in er1.items()))
    assert max(er1.values()) <= 1e-13, er1

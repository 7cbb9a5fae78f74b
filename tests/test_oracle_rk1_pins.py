"""Pins of the oracle's implicit RK1 drag step v' = (I - dt K)^{-1} v (the
linear system of the paper's implicit-solver appendix, eq. analytic_1, for
velocities), each against something other than the oracle's own Gaussian
elimination: Cramer's rule for N = 1, exact conservation of total momentum,
the residual of the system, numpy's LU solve on dense matrices built here,
the stiff limit (the barycentric velocity), dt = 0, and the paper's O(N)
closed form (eqs. analytic_3 and analytic_4) written out independently."""
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W


def kmat(dt, rho_g, rho_d, t_stop):
    """dt K in the velocity form, dense, built here from the ODE."""
    N = len(rho_d)
    a = dt / t_stop
    e = rho_d / rho_g
    A = np.zeros((N + 1, N + 1))
    A[0, 1:] = e * a
    A[0, 0] = -np.sum(e * a)
    A[1:, 0] = a
    A[np.arange(1, N + 1), np.arange(1, N + 1)] = -a
    return A


def test_n1_cramer(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        rg, rd, t = rng.uniform(0.5, 2), rng.uniform(0, 5), 10 ** rng.uniform(-4, 2)
        v = rng.standard_normal((1, 2, 1))
        dt = 10 ** rng.uniform(-3, 3)
        out, st = orc.rk1_cells(np.array([rg]), np.array([[rd]]), np.array([[t]]), v, dt)
        assert st == 0
        # Cramer's rule in long double, from the inputs
        L = np.longdouble
        a = L(dt) / L(t)
        p = L(rd) / L(rg) * a
        det = 1 + a + p
        x0 = ((1 + a) * L(v[0, 0, 0]) + p * L(v[0, 1, 0])) / det
        x1 = (a * L(v[0, 0, 0]) + (1 + p) * L(v[0, 1, 0])) / det
        np.testing.assert_allclose(out[0, :, 0], [float(x0), float(x1)], rtol=0,
                                   atol=2e-16 * np.abs(v).max())


@pytest.mark.parametrize("name", ["n4_3d", "n16_stiff_3d", "n8_adjoint_3d"])
def test_momentum_residual_and_lu(orc, name):
    d = W.make(name, 300)
    out, st = orc.rk1_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"])
    assert st == 0
    rho = np.concatenate([d["rho_g"][None], d["rho_d"]])
    for c in range(300):
        A = kmat(d["dt"], d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c])
        M = np.eye(len(A)) - A
        for k in range(d["v"].shape[0]):
            v, x = d["v"][k, :, c], out[k, :, c]
            scale = np.abs(rho[:, c] * v).sum()
            # exact conservation: only the final rounding of x remains
            L = np.longdouble
            dp = (rho[:, c].astype(L) * x.astype(L)).sum() - (rho[:, c].astype(L) * v.astype(L)).sum()
            assert abs(float(dp)) <= 4 * 2.0 ** -53 * rho[:, c].sum() * np.abs(v).max()
            assert scale > 0
            assert np.abs(M @ x - v).max() <= 1e-12 * np.abs(M).max() * np.abs(v).max()
            ref = np.linalg.solve(M, v)
            assert np.abs(x - ref).max() <= 1e-12 * np.abs(v).max()


def test_stiff_limit_dt_zero_and_edges(orc):
    d = W.make("n4_3d", 64)
    rho = np.concatenate([d["rho_g"][None], d["rho_d"]])
    # dt >> t_i: every fluid tends to the barycentric velocity, the gap
    # shrinking like t_max / dt (t_i <= 12 here)
    vcm = (rho[None] * d["v"]).sum(axis=1) / rho.sum(axis=0)[None]
    gaps = []
    for dt in (1e4, 1e6):
        out, st = orc.rk1_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], dt)
        assert st == 0
        gaps.append(np.abs(out - vcm[:, None, :]).max() / np.abs(d["v"]).max())
    assert gaps[1] <= 1e-4 and gaps[1] <= gaps[0] / 50, gaps
    out0, _ = orc.rk1_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], 0.0)
    assert np.array_equal(out0, d["v"])
    # a decoupled species (t = inf) keeps its velocity; rho_d = 0 leaves the gas alone
    rd, ts = d["rho_d"].copy(), d["t_stop"].copy()
    ts[1, 3] = np.inf
    rd[:, 4] = 0.0
    out2, st = orc.rk1_cells(d["rho_g"], rd, ts, d["v"], d["dt"])
    assert st == 0
    assert np.array_equal(out2[:, 2, 3], d["v"][:, 2, 3])
    np.testing.assert_allclose(out2[:, 0, 4], d["v"][:, 0, 4], rtol=0, atol=1e-15)
    # bad cells: NaN outputs and the status bits
    rg = d["rho_g"].copy()
    rg[7] = -1.0
    out3, st = orc.rk1_cells(rg, d["rho_d"], d["t_stop"], d["v"], d["dt"])
    assert st == orc.BAD_DENSITY and np.isnan(out3[..., 7]).all()


def test_paper_closed_form(orc):
    """eqs. analytic_3-4 in the paper's variables (q_0 = v_g, q_i = e_i v_i):
    A = 1 + sum_i (1 - 1/(1 + a_i)) e_i, B = sum_i a_i/(1 + a_i) b_i / dt,
    q_0 = (b_0 + dt B) / A, q_i = (b_i + e_i a_i q_0) / (1 + a_i)."""
    d = W.make("n16_stiff_3d", 100)
    out, _ = orc.rk1_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"])
    for c in range(100):
        a = d["dt"] / d["t_stop"][:, c]
        e = d["rho_d"][:, c] / d["rho_g"][c]
        for k in range(3):
            v = d["v"][k, :, c]
            b0, b = v[0], e * v[1:]
            Acal = 1 + np.sum((1 - 1 / (1 + a)) * e)
            dtB = np.sum(a / (1 + a) * b)
            q0 = (b0 + dtB) / Acal
            q = (b + e * a * q0) / (1 + a)
            x = np.concatenate([[q0], q / np.where(e == 0, 1, e)])
            assert np.abs(x - out[k, :, c]).max() <= 1e-13 * np.abs(v).max()

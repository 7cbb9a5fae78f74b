"""Pins of the oracle's reverse-mode gradient.

L = sum_d w_d . v'_d with v'_d = exp(dt K) v_d.  The oracle differentiates
its own computed approximant with (k*, m*, s*) frozen; these tests compare it
with derivatives it does not compute: scipy's Frechet derivative of the
exponential, the derivative of the closed-form two-fluid solution, central
finite differences of a multiprecision forward, and sum rules that follow
from the structure of K (rows summing to zero, momentum conservation).
"""
import mpmath as mp
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W

U = 2.0 ** -53


def _cell(d, c):
    return d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c], d["v"][:, :, c]


def _grad_one(orc, rg, rd, ts, v, w, dt=1.0):
    """Oracle gradients of one cell (arrays shaped for a 1-cell grid)."""
    out = orc.grad_cells(np.array([rg]), rd[:, None], ts[:, None], v[:, :, None],
                         w[:, :, None], dt)
    v_out, g_v, g_logt, g_rho_d, g_rho_g, st = out
    assert st == 0
    return v_out[:, :, 0], g_v[:, :, 0], g_logt[:, 0], g_rho_d[:, 0], g_rho_g[0]


def test_grad_A_matches_scipy_frechet(orc):
    """dL/dA for L = <G, Y(A)> is the Frechet derivative at A^T in the
    direction G; scipy evaluates it from the Pade approximant."""
    sl = pytest.importorskip("scipy.linalg")
    rng = np.random.default_rng(21)
    for name in ("n4_3d", "n8_adjoint_3d"):
        d = W.make(name, 6)
        for c in range(6):
            rg, rd, ts, v = _cell(d, c)
            A, a, e, nrm, bad = orc.build_matrix(1.0, rg, rd, ts)
            G = rng.standard_normal(A.shape)
            Ab = orc.grad_A(A, nrm, G)
            ref = sl.expm_frechet(A.T, G, compute_expm=False)
            scale = np.abs(ref).max()
            assert np.abs(Ab - ref).max() <= 1e-11 * scale, (name, c)


def test_two_fluid_closed_form_derivatives(orc):
    """N = 1: derivatives of v' = V + (v - V) e^{-(1+e) a} with respect to
    log t, rho_1, rho_g and v, by multiprecision differentiation."""
    d = W.make("n1_closed_form", 64)
    rng = np.random.default_rng(5)
    mp.mp.dps = 30
    for c in range(0, 64, 4):
        rg, rd, ts, v = _cell(d, c)
        w = rng.standard_normal(v.shape)

        def loss(logt, r1, r0, vg, v1):
            a = 1 / mp.exp(logt)
            e = r1 / r0
            V = (vg + e * v1) / (1 + e)
            dec = mp.exp(-(1 + e) * a)
            return w[0, 0] * (V + (vg - V) * dec) + w[0, 1] * (V + (v1 - V) * dec)

        x0 = [mp.log(mp.mpf(ts[0])), mp.mpf(rd[0]), mp.mpf(rg),
              mp.mpf(v[0, 0]), mp.mpf(v[0, 1])]
        ref = []
        for k in range(5):
            order = [0] * 5
            order[k] = 1
            ref.append(float(mp.diff(loss, x0, tuple(order))))
        _, g_v, g_logt, g_rho_d, g_rho_g = _grad_one(orc, rg, rd, ts, v, w)
        nrm = orc.build_matrix(1.0, rg, rd, ts)[3]
        got = [g_logt[0], g_rho_d[0], g_rho_g, g_v[0, 0], g_v[0, 1]]
        scale = max(abs(x) for x in ref)
        tol = (1e-13 + 8 * U * nrm) * scale + 1e-15
        for k in range(5):
            assert abs(got[k] - ref[k]) <= tol, (c, k, got[k], ref[k])


def _mp_loss(rg, rd, ts, v, w, dps=34):
    """L in multiprecision: exp(dt K) from mpmath's own expm."""
    with mp.workdps(dps):
        N = len(rd)
        n = N + 1
        a = [1 / mp.mpf(x) for x in ts]
        e = [mp.mpf(x) / mp.mpf(rg) for x in rd]
        A = mp.zeros(n, n)
        for i in range(N):
            A[0, 0] -= e[i] * a[i]
            A[0, i + 1] = e[i] * a[i]
            A[i + 1, 0] = a[i]
            A[i + 1, i + 1] = -a[i]
        E = mp.expm(A)
        L = mp.mpf(0)
        for dd in range(v.shape[0]):
            for j in range(n):
                L += mp.mpf(w[dd, j]) * mp.fsum(E[j, k] * mp.mpf(v[dd, k]) for k in range(n))
        return L


def test_gradient_vs_multiprecision_finite_differences(orc):
    """Central differences, h = 1e-6 (additive in log t and v, relative in
    rho), of a multiprecision forward: truncation error ~h^2, so the oracle's
    gradient must agree to 1e-8 of the largest entry of each group."""
    d = W.make_jittered(3, 3, D=2, cfg=9)
    rng = np.random.default_rng(8)
    h = 1e-6
    for c in range(3):
        rg, rd, ts, v = _cell(d, c)
        w = rng.standard_normal(v.shape)
        _, g_v, g_logt, g_rho_d, g_rho_g = _grad_one(orc, rg, rd, ts, v, w)
        with mp.workdps(34):
            fd_logt, fd_rho = [], []
            for i in range(len(rd)):
                tp, tm = ts.copy(), ts.copy()
                tp[i] = float(mp.mpf(ts[i]) * mp.exp(h))
                tm[i] = float(mp.mpf(ts[i]) * mp.exp(-h))
                # the perturbed t is rounded to double: use the actual step
                hp = float(mp.log(mp.mpf(tp[i]) / mp.mpf(ts[i])))
                hm = float(mp.log(mp.mpf(tm[i]) / mp.mpf(ts[i])))
                fd_logt.append(float((_mp_loss(rg, rd, tp, v, w) - _mp_loss(rg, rd, tm, v, w)) / (hp - hm)))
                rp, rm = rd.copy(), rd.copy()
                rp[i] = rd[i] * (1 + h)
                rm[i] = rd[i] * (1 - h)
                fd_rho.append(float((_mp_loss(rg, rp, ts, v, w) - _mp_loss(rg, rm, ts, v, w)) / (mp.mpf(rp[i]) - mp.mpf(rm[i]))))
            fd_v = np.zeros_like(v)
            for dd in range(v.shape[0]):
                for j in range(v.shape[1]):
                    vp, vm = v.copy(), v.copy()
                    vp[dd, j] += h
                    vm[dd, j] -= h
                    fd_v[dd, j] = float((_mp_loss(rg, rd, ts, vp, w) - _mp_loss(rg, rd, ts, vm, w)) / (mp.mpf(vp[dd, j]) - mp.mpf(vm[dd, j])))
        for got, ref in ((g_logt, np.array(fd_logt)), (g_rho_d, np.array(fd_rho)), (g_v, fd_v)):
            assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max(), (c, got, ref)


def test_sum_rules(orc):
    """E 1 = 1 for every parameter value, so a uniform velocity has zero
    gradient in log t and rho; rho^T E = rho^T, so the weights w = rho give
    zero gradient in log t."""
    d = W.make("n8_adjoint_3d", 8)
    rng = np.random.default_rng(2)
    for c in range(8):
        rg, rd, ts, v = _cell(d, c)
        A, a, e, nrm, bad = orc.build_matrix(1.0, rg, rd, ts)
        w = rng.standard_normal(v.shape)
        vu = np.ones_like(v) * rng.standard_normal((v.shape[0], 1))
        _, g_v, g_logt, g_rho_d, g_rho_g = _grad_one(orc, rg, rd, ts, vu, w)
        _, _, g_logt_ref, g_rho_ref, _ = _grad_one(orc, rg, rd, ts, v, w)
        # zero up to rounding: 1e-10 of the gradient's size for a generic v
        assert np.abs(g_logt).max() <= 1e-10 * np.abs(g_logt_ref).max()
        assert np.abs(g_rho_d).max() <= 1e-10 * np.abs(g_rho_ref).max()
        rho = np.concatenate([[rg], rd])
        wr = np.repeat(rho[None, :], v.shape[0], axis=0)
        _, g_v2, g_logt2, _, _ = _grad_one(orc, rg, rd, ts, v, wr)
        assert np.abs(g_logt2).max() <= 1e-10 * np.abs(g_logt_ref).max() * rho.max()
        # and then dL/dv = rho (momentum is conserved)
        assert np.abs(g_v2 - wr).max() <= 8 * U * nrm * rho.max()

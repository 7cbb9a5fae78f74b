"""Multiprecision central differences of the drag update (TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle/``).

L = sum_d w_d . v'_d with v'_d = exp(dt K) v_d, K read off the drag ODE of
Sect. 2.2 in velocity form (dv_i/dt = -(v_i - v_g)/t_i,
dv_g/dt = sum_i (rho_i/rho_g)(v_i - v_g)/t_i) and the exponential taken by
mpmath at ``dps`` digits, so the forward's rounding (~10^-dps) divided by the
step stays far below the truncation error h^2 L'''/6 of the central
difference.  Steps: additive in log t_i and in v, relative in rho_i and
rho_g; the perturbed inputs are rounded to double and the quotient uses the
step actually taken.  Used to check the library's hand-written adjoint to
1e-8 of each gradient group without differencing an FP64 forward (whose
rounding noise over h = 1e-6 is itself ~1e-8).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def expm_velocity(dt, rho_g, rho_d, t_stop, dps=30):
    """exp(dt K) as an mpmath matrix."""
    with mp.workdps(dps):
        N = len(rho_d)
        n = N + 1
        A = mp.zeros(n, n)
        for i in range(N):
            a = mp.mpf(dt) / mp.mpf(float(t_stop[i]))
            e = mp.mpf(float(rho_d[i])) / mp.mpf(float(rho_g))
            A[i + 1, i + 1] = -a
            A[i + 1, 0] = a
            A[0, i + 1] = e * a
            A[0, 0] -= e * a
        return mp.expm(A)


def loss(E, v, w, dps=30):
    """sum_d w_d . (E v_d) in multiprecision."""
    with mp.workdps(dps):
        D, n = v.shape
        acc = mp.mpf(0)
        for d in range(D):
            for j in range(n):
                acc += mp.mpf(float(w[d, j])) * mp.fsum(
                    E[j, k] * mp.mpf(float(v[d, k])) for k in range(n))
        return acc


def fd_gradients(rho_g, rho_d, t_stop, v, w, dt=1.0, h=1e-6, dps=30):
    """Central differences of L for one cell.

    rho_d, t_stop [N]; v, w [D][N+1].  Returns dict(g_logt [N], g_rho_d [N],
    g_rho_g scalar, g_v [D][N+1]) as float64."""
    N = len(rho_d)
    rho_d = np.asarray(rho_d, dtype=np.float64)
    t_stop = np.asarray(t_stop, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)

    def L(rg, rd, ts, vv):
        return loss(expm_velocity(dt, rg, rd, ts, dps), vv, w, dps)

    with mp.workdps(dps):
        g_logt = np.zeros(N)
        g_rho = np.zeros(N)
        for i in range(N):
            tp, tm = t_stop.copy(), t_stop.copy()
            tp[i] = float(mp.mpf(t_stop[i]) * mp.exp(h))
            tm[i] = float(mp.mpf(t_stop[i]) * mp.exp(-h))
            step = mp.log(mp.mpf(tp[i]) / mp.mpf(tm[i]))
            g_logt[i] = float((L(rho_g, rho_d, tp, v) - L(rho_g, rho_d, tm, v)) / step)
            rp, rm = rho_d.copy(), rho_d.copy()
            rp[i] = rho_d[i] * (1 + h)
            rm[i] = rho_d[i] * (1 - h)
            g_rho[i] = float((L(rho_g, rp, t_stop, v) - L(rho_g, rm, t_stop, v))
                             / (mp.mpf(rp[i]) - mp.mpf(rm[i])))
        gp, gm = rho_g * (1 + h), rho_g * (1 - h)
        g_rho_g = float((L(gp, rho_d, t_stop, v) - L(gm, rho_d, t_stop, v))
                        / (mp.mpf(gp) - mp.mpf(gm)))
        E = expm_velocity(dt, rho_g, rho_d, t_stop, dps)
        g_v = np.zeros_like(v)
        for d in range(v.shape[0]):
            for j in range(v.shape[1]):
                vp, vm = v.copy(), v.copy()
                vp[d, j] += h
                vm[d, j] -= h
                g_v[d, j] = float((loss(E, vp, w, dps) - loss(E, vm, w, dps))
                                  / (mp.mpf(vp[d, j]) - mp.mpf(vm[d, j])))
    return dict(g_logt=g_logt, g_rho_d=g_rho, g_rho_g=g_rho_g, g_v=g_v)

"""Pins of the oracle's diagonal Pade scaling step (Sect. 2.3, eq. PadeEqu
with p = q = m), each against something other than the oracle's own code:

* theta_m recomputed here in multiprecision from the backward-error series
  of r_m (log(e^-x r_m(x)) summed to its first 60 nonzero terms past 2m);
* the coefficients against mpmath's own Pade solver on the Taylor
  coefficients of e^x (so the closed form of eq. PadeEqu is not retyped);
* the selection at every theta boundary and for scaled norms;
* the Dustybox two-fluid closed form (N = 1) and the exact exponential on the
  workloads, to the bar the Taylor oracle meets.
"""
import mpmath as mp
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W

U = 2.0 ** -53
DEGREES = (3, 5, 7, 9, 13)


def theta_mp(m, extra=60):
    """Largest theta with sum_{k>2m} |c_k| theta^(k-1) <= u, where
    log(e^-x r_m(x)) = sum_k c_k x^k, from truncated power series."""
    mp.mp.dps = 60
    nt = 2 * m + 1 + extra
    c = [mp.factorial(2 * m - j) * mp.factorial(m) /
         (mp.factorial(2 * m) * mp.factorial(j) * mp.factorial(m - j)) for j in range(m + 1)]
    P = [c[j] if j <= m else mp.mpf(0) for j in range(nt)]
    Q = [c[j] * (-1) ** j if j <= m else mp.mpf(0) for j in range(nt)]
    R = [mp.mpf(0)] * nt
    for k in range(nt):
        R[k] = (P[k] - sum(Q[i] * R[k - i] for i in range(1, k + 1))) / Q[0]
    G = [sum((-1) ** i / mp.factorial(i) * R[k - i] for i in range(k + 1)) for k in range(nt)]
    G[0] = mp.mpf(0)
    H = [mp.mpf(0)] * nt
    term = [mp.mpf(1)] + [mp.mpf(0)] * (nt - 1)
    for n in range(1, nt):
        term = [sum(term[i] * G[k - i] for i in range(k + 1)) for k in range(nt)]
        for k in range(nt):
            H[k] += (-1) ** (n + 1) * term[k] / n
    u = mp.mpf(2) ** -53
    f = lambda th: sum(abs(H[k]) * th ** (k - 1) for k in range(2 * m + 1, nt)) - u
    return mp.findroot(f, (mp.mpf("1e-4"), mp.mpf(8)), solver="bisect")


@pytest.mark.parametrize("i", range(5))
def test_theta_recomputed(orc, i):
    m, th, _ = orc.pade_row(i)
    assert m == DEGREES[i]
    ref = theta_mp(m)
    assert abs(th - float(ref)) <= 4e-16 * th, (m, th, ref)


@pytest.mark.parametrize("i", range(5))
def test_coefficients_against_mpmath_pade(orc, i):
    m, _, c = orc.pade_row(i)
    mp.mp.dps = 50
    taylor = [1 / mp.factorial(k) for k in range(2 * m + 1)]
    p, q = mp.pade(taylor, m, m)
    p = [x / q[0] for x in p]
    q = [x / q[0] for x in q]
    for j in range(m + 1):
        assert c[j] == float(p[j]), (m, j)
        assert (-1) ** j * c[j] == float(q[j]), (m, j)


def test_selection_boundaries(orc):
    ths = [orc.pade_row(i)[1] for i in range(5)]
    for i, th in enumerate(ths):
        assert orc.pade_select(th) == (DEGREES[i], 0)
        up = float(np.nextafter(th, np.inf))
        assert orc.pade_select(up) == ((DEGREES[i + 1], 0) if i < 4 else (13, 1))
    assert orc.pade_select(0.0) == (3, 0)
    for x in (6.0, 11.0, 1e3, 3.7e6):
        m, s = orc.pade_select(x)
        assert m == 13 and x <= ths[4] * 2.0 ** s and (s == 0 or x > ths[4] * 2.0 ** (s - 1))


def test_dustybox_closed_form(orc):
    """N = 1: the two velocities relax with rate (1 + e) / t toward the
    barycentre; e^(dt K) in closed form."""
    d = W.make("n1_closed_form", 512)
    out, kms, nrm, st = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"],
                                        option=orc.PADE)
    assert st == 0
    rg, rd, t, v = d["rho_g"], d["rho_d"][0], d["t_stop"][0], d["v"][0]
    e = rd / rg
    vcm = (v[0] + e * v[1]) / (1 + e)
    dec = np.exp(-d["dt"] * (1 + e) / t)
    dv = (v[1] - v[0]) * dec
    vg = vcm - e * dv / (1 + e)
    vd = vcm + dv / (1 + e)
    scale = np.abs(v).max(axis=0)
    assert (np.abs(out[0, 0] - vg) / scale).max() <= 2e-15
    assert (np.abs(out[0, 1] - vd) / scale).max() <= 2e-15
    assert set(np.unique(kms[1])) <= set(DEGREES)


@pytest.mark.parametrize("name", ["n4_3d", "n8_adjoint_3d", "n16_stiff_3d"])
def test_against_the_exact_exponential(orc, name):
    d = W.make(name, 64)
    out, kms, nrm, st = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"],
                                        option=orc.PADE)
    assert st == 0
    for c in range(64):
        m, s = orc.pade_select(nrm[c])
        assert (kms[1][c], kms[2][c]) == (m, s)
        E = orc.truth_eigen(d["dt"], d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c])
        exact = d["v"][:, :, c] @ E.T
        scale = np.abs(d["v"][:, :, c]).max(axis=1)
        e = (np.abs(out[:, :, c] - exact).max(axis=1) / scale).max()
        assert e <= max(1e-13, 4 * U * nrm[c]), (name, c, e)

"""Pins of the oracle's second modification (Appendix B: the negligible-term
test of eqs. Pat_Stk4-Pat_stk7 with the bound b_exp of eq. Pat_Stk6), each
against something other than the oracle's own Horner loop:

* b_exp bounds ||T_m(-B)||_1, with T_m(-B) summed here as a plain power
  series (triangle inequality on the block form), and tracks ||e^-B||;
* what the test drops is negligible: ||F_full - F_bt||_1 stays below
  (products skipped) * u / b_exp, the guarantee the test is built on, plus
  the rounding of the products that follow a drop (4 n u ||F||_1);
* at ||B|| = theta_m (the top of Alg. 1's range) nothing is dropped; far
  below it the top block is; B = 0 drops every product and returns 0;
* the full update with the bound test meets the bar the plain method meets
  against the exact exponential (max(1e-13, 4 u ||dt K||_1)), and the test
  does fire on some of the workloads' cells.
"""
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W

U = 2.0 ** -53


def series(B, m):
    """T_m(B) by summing B^i / i! term by term (no blocks, no Horner)."""
    n = B.shape[0]
    T = np.eye(n)
    P = np.eye(n)
    f = 1.0
    for i in range(1, m + 1):
        P = P @ B
        f *= i
        T = T + P / f
    return T


def random_arrowhead(rng, n, scale):
    """A drag-like matrix (rows summing to zero, nonnegative off-diagonal
    entries in the gas row/column) of 1-norm `scale`."""
    a = 10 ** rng.uniform(-2, 1, n - 1)
    e = 10 ** rng.uniform(-2, 0.5, n - 1)
    A = np.zeros((n, n))
    A[0, 1:] = e * a
    A[0, 0] = -np.sum(e * a)
    A[1:, 0] = a
    A[np.arange(1, n), np.arange(1, n)] = -a
    return A * (scale / np.abs(A).sum(axis=0).max())


def test_bexp_bounds_the_negative_series(orc):
    rng = np.random.default_rng(11)
    for _ in range(60):
        n = int(rng.integers(2, 8))
        k = int(rng.integers(2, 10))
        m, q, r, th = orc.table_row(k)
        B = random_arrowhead(rng, n, th * rng.uniform(0.05, 1.0))
        _, _, bexp = orc.taylor_stage(B, k, True)
        tm = np.abs(series(-B, m)).sum(axis=0).max()
        assert tm <= bexp * (1 + 1e-13), (k, tm, bexp)
        # and it is an estimate of ||e^-B||, not a loose bound (B is small)
        assert bexp <= 2.5 * tm


def test_dropped_part_is_below_the_guarantee(orc):
    hits = 0
    for name in ("n8_adjoint_3d", "n1_closed_form", "n4_3d"):
        d = W.make(name, 300)
        for c in range(300):
            A, a, e, nrm, bad = orc.build_matrix(d["dt"], d["rho_g"][c], d["rho_d"][:, c],
                                                 d["t_stop"][:, c])
            k, m, s = orc.select(nrm, 9, 2)
            B = np.ldexp(A, -s)
            F0, sk0, _ = orc.taylor_stage(B, k, False)
            F1, sk1, bexp = orc.taylor_stage(B, k, True)
            assert sk0 == 0
            diff = np.abs(F0 - F1).sum(axis=0).max()
            if sk1 == 0:
                assert np.array_equal(F0, F1)
            else:
                hits += 1
                n = B.shape[0]
                fn = max(1.0, np.abs(F0).sum(axis=0).max())
                assert diff <= sk1 * U / bexp + 4 * n * U * fn, (name, c, diff, sk1, bexp)
    assert hits >= 10


def test_top_of_range_keeps_everything_far_below_drops(orc):
    rng = np.random.default_rng(12)
    for k in range(3, 10):
        m, q, r, th = orc.table_row(k)
        for _ in range(5):
            n = int(rng.integers(3, 7))
            B = random_arrowhead(rng, n, th)
            _, sk, _ = orc.taylor_stage(B, k, True)
            assert sk == 0, k
            Bs = B / 2 ** 12
            F0, _, _ = orc.taylor_stage(Bs, k, False)
            F1, sk, bexp = orc.taylor_stage(Bs, k, True)
            assert sk >= 1, k
            fn = max(1.0, np.abs(F0).sum(axis=0).max())
            assert np.abs(F0 - F1).sum(axis=0).max() <= sk * U / bexp + 4 * n * U * fn
        F, sk, bexp = orc.taylor_stage(np.zeros((4, 4)), k, True)
        assert sk == r - 1 and not F.any() and bexp == 1.0


def test_full_update_with_bound_test_meets_the_exact_bar(orc):
    fired = 0
    for name, C in (("n8_adjoint_3d", 300), ("n1_closed_form", 300), ("n16_stiff_3d", 48),
                    ("n4_3d", 96)):
        d = W.make(name, C)
        out, kms, nrm, st = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"],
                                            option=2 | orc.BOUND_TEST)
        plain, kms2, _, _ = orc.apply_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["dt"])
        assert st == 0 and np.array_equal(kms, kms2)
        for c in range(C):
            E = orc.truth_eigen(d["dt"], d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c])
            exact = d["v"][:, :, c] @ E.T
            scale = np.abs(d["v"][:, :, c]).max(axis=1)
            e = (np.abs(out[:, :, c] - exact).max(axis=1) / scale).max()
            assert e <= max(1e-13, 4 * U * nrm[c]), (name, c, e)
            fired += not np.array_equal(out[:, :, c], plain[:, :, c])
    assert fired >= 5

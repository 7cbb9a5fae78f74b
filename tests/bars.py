"""Parity bars of the drag update, shared by the GPU tests.

Per-cell velocity error: e = max over components d and rows j of
|v'_got - v'_ref| / max_j |v_in[d, j]|.  The output is a convex combination
of the inputs (exp(dt K) is row-stochastic and non-negative), so the input's
largest magnitude is the natural scale; a relative error per entry is
undefined where v' crosses zero.

Bars, checked on every cell whose inputs are valid:

* against the exact exponential (``oracle.truth_apply``: long double, no
  scaling and squaring): e <= 1e-13.  The approximant's backward error is
  bounded by the unit round-off (App. B, eqs. B1-B8), so the library's
  result must stay at the FP64 floor of the exact solution.
* against the method oracle (the paper's steps in FP64, ``oracle``):
  e <= 1e-13 + e(oracle, exact).  The oracle squares the dense (N+1) x (N+1)
  matrix, whose conserved mode carries a rounding defect of order
  u ||dt K||_1 that doubles with every squaring (up to ~5e-13 on the N = 4
  workload); per cell that excess is the oracle's own distance from the
  exact result, measured here, not a blanket allowance.
* ``tight=True`` (workloads where the oracle itself is at the floor: the
  N = 1 closed-form cells, the stiff N = 16 cells, the uneven-N blocks):
  e(got, oracle) <= 1e-13 outright.
* total momentum of every component: |rho^T (v' - v)| / sum_j rho_j |v_j|
  <= 1e-12.
"""
import numpy as np

TOL = 1e-13
MOMENTUM_TOL = 1e-12


def cell_errors(got, ref, v_in):
    """e per cell for arrays shaped [D][N+1][C]."""
    scale = np.abs(v_in).max(axis=1)  # [D][C]
    scale = np.where((scale == 0) | ~np.isfinite(scale), 1.0, scale)
    return (np.abs(got - ref).max(axis=1) / scale).max(axis=0)


def momentum_errors(out, d):
    rho = np.concatenate([d["rho_g"][None, :], d["rho_d"]])
    p0 = (rho[None] * d["v"]).sum(axis=1)
    p1 = (rho[None] * out).sum(axis=1)
    scale = (rho[None] * np.abs(d["v"])).sum(axis=1)
    scale = np.where(scale == 0, 1.0, scale)
    return (np.abs(p1 - p0) / scale).max(axis=0)


def exact(orc, d, dt=None):
    """v' = exp(dt K) v per cell from the long-double truth; NaN on cells with
    invalid inputs."""
    dt = d["dt"] if dt is None else dt
    return orc.truth_apply(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], dt)


def check_forward(orc, got, ref, d, label, tight=False, truth=None, momentum=True):
    """Assert the bars above on the cells where the oracle's result is finite;
    returns the per-cell errors (got vs oracle, got vs exact, oracle vs
    exact) on those cells."""
    good = np.isfinite(ref).all(axis=(0, 1))
    assert np.isfinite(got[..., good]).all(), label
    tr = exact(orc, d) if truth is None else truth
    assert np.isfinite(tr[..., good]).all(), label
    g, r, t, v = got[..., good], ref[..., good], tr[..., good], d["v"][..., good]
    e_go = cell_errors(g, r, v)
    e_gx = cell_errors(g, t, v)
    e_ox = cell_errors(r, t, v)
    if e_go.size:
        assert e_gx.max() <= TOL, (label, "vs exact", e_gx.max(), int(e_gx.argmax()))
        over = e_go - e_ox
        assert over.max() <= TOL, (label, "vs oracle beyond its own error", e_go.max(),
                                   over.max(), int(over.argmax()))
        if tight:
            assert e_go.max() <= TOL, (label, "vs oracle", e_go.max(), int(e_go.argmax()))
        if momentum:
            sub = {k: (d[k][..., good] if k in ("rho_g", "rho_d", "v") else d[k]) for k in d}
            assert momentum_errors(g, sub).max() <= MOMENTUM_TOL, label
    return e_go, e_gx, e_ox


GRAD_TOL = 1e-10


def sens_scale(d):
    """S per cell: sum over components of ||w_c||_inf ||v_c||_inf, the natural
    size of the sensitivities of L = sum w . v'."""
    return (np.abs(d["w"]).max(axis=1) * np.abs(d["v"]).max(axis=1)).sum(axis=0)


def group_err(got, ref, floor=None):
    """Per cell (last axis): max over the group of |got - ref| /
    max(max |ref|, floor)."""
    got, ref = np.asarray(got), np.asarray(ref)
    C = got.shape[-1]
    g = np.moveaxis(got, -1, 0).reshape(C, -1)
    r = np.moveaxis(ref, -1, 0).reshape(C, -1)
    scale = np.abs(r).max(axis=1)
    if floor is not None:
        scale = np.maximum(scale, floor)
    scale = np.where(scale == 0, 1.0, scale)
    return np.abs(g - r).max(axis=1) / scale


def check_gradients(orc, d, grads, label, tol=GRAD_TOL, oracle_grads=None):
    """Gradients (g_v, g_logt, g_rho_d, g_rho_g) of L = sum w . v' against the
    exact gradient (``oracle.truth_grad``, long double) and the oracle's
    reverse-mode gradient, per cell and group, normalised by
    max(max |g_ref|, S) (S / rho_g for the density groups; where every mode of
    a cell has decayed, dL/dlog t is ~1e-16 and only its absolute error is
    meaningful):
      e(got, exact) <= tol,   e(got, oracle) <= tol + e(oracle, exact).
    The oracle differentiates the dense (N+1) chain, whose conserved mode
    costs it up to ~4e-10 in the density gradients of stiff cells; per cell
    that is its own distance from the exact gradient."""
    g_v, g_logt, g_rho, g_rho_g = grads
    if oracle_grads is None:
        ro = orc.grad_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["w"], d["dt"])
        assert ro[-1] == 0, label
        oracle_grads = ro[1:5]
    ex = orc.truth_grad(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["w"], d["dt"])
    S = sens_scale(d)
    Sr = S / d["rho_g"]
    errs = {}
    for name, got, orv, exv, fl in (("g_v", g_v, oracle_grads[0], ex[0], None),
                                    ("g_logt", g_logt, oracle_grads[1], ex[1], S),
                                    ("g_rho_d", g_rho, oracle_grads[2], ex[2], Sr),
                                    ("g_rho_g", g_rho_g[None], oracle_grads[3][None], ex[3][None],
                                     Sr)):
        assert np.isfinite(exv).all(), (label, name, "no exact gradient")
        e_gx = group_err(got, exv, fl)
        e_go = group_err(got, orv, fl)
        e_ox = group_err(orv, exv, fl)
        assert np.isfinite(e_gx).all() and np.isfinite(e_go).all(), (label, name)
        assert e_gx.max() <= tol, (label, name, "vs exact", e_gx.max(), int(e_gx.argmax()))
        over = e_go - e_ox
        assert over.max() <= tol, (label, name, "vs oracle beyond its own error", e_go.max(),
                                   over.max(), int(over.argmax()))
        errs[name] = (e_go, e_gx, e_ox)
    return errs

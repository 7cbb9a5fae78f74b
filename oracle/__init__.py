"""CPU reference (the oracle) for the per-cell drag update v' = exp(dt K) v.

TEST INFRASTRUCTURE ONLY.  The oracle is the parity checker for the HIP
library: a plain, slow, single-threaded FP64 implementation of the paper's
Taylor scaling-and-squaring method (arXiv:2509.25347, Sect. 2.3 and
Appendix B), written in C (``oracle.c``) with long-double truths that do not
use scaling and squaring (``truth.c``).  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the library under ``paper_2509_25347_amd``.

``build()`` compiles ``liboracle.so`` next to this file with
``gcc -O2 -ffp-contract=off`` (every operation one IEEE double rounding).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "truth.c"),
            os.path.join(_HERE, "rk1.c")]

BAD_DENSITY = 1
BAD_STOPPING_TIME = 2
BAD_VELOCITY = 4
BAD_NORM = 8
NMAX = 33

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` and return its path."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp] + _SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.POINTER
    d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
    vp = ctypes.c_void_p
    lib.orc_table_row.argtypes = [i, P(i), P(i), P(i), P(d)]
    lib.orc_table_row.restype = i
    lib.orc_taylor_coef.argtypes = [i]
    lib.orc_taylor_coef.restype = d
    lib.orc_select.argtypes = [d, i, i, P(i), P(i), P(i)]
    lib.orc_select.restype = None
    lib.orc_build.argtypes = [i, d, d, vp, vp, vp, vp, vp, P(d)]
    lib.orc_build.restype = i
    lib.orc_expm.argtypes = [i, vp, d, i, i, i, vp, vp]
    lib.orc_expm.restype = i
    lib.orc_cell_expm.argtypes = [i, d, d, vp, vp, i, i, i, vp, vp]
    lib.orc_cell_expm.restype = i
    lib.orc_apply_cells.argtypes = [i64, i, i, i64, d, i, i, i, vp, vp, vp, vp,
                                    vp, vp, vp]
    lib.orc_apply_cells.restype = i
    lib.orc_grad_A.argtypes = [i, vp, d, i, i, vp, vp, vp]
    lib.orc_grad_A.restype = i
    lib.orc_grad_cells.argtypes = [i64, i, i, i64, d, i, i, vp, vp, vp, vp, vp,
                                   vp, vp, vp, vp, vp]
    lib.orc_grad_cells.restype = i
    lib.orc_pade_row.argtypes = [i, P(i), P(d), vp]
    lib.orc_pade_row.restype = i
    lib.orc_pade_select.argtypes = [d, P(i), P(i)]
    lib.orc_pade_select.restype = None
    lib.orc_taylor_stage.argtypes = [i, vp, i, i, vp, P(i), P(d)]
    lib.orc_taylor_stage.restype = i
    lib.orc_rk1_cells.argtypes = [i64, i, i, i64, d, vp, vp, vp, vp, vp]
    lib.orc_rk1_cells.restype = i
    lib.truth_expm_eigen.argtypes = [i, d, d, vp, vp, vp]
    lib.truth_expm_eigen.restype = i
    lib.truth_expm_taylor.argtypes = [i, vp, i, vp]
    lib.truth_expm_taylor.restype = i
    lib.truth_expm_general.argtypes = [i, d, d, vp, vp, vp]
    lib.truth_expm_general.restype = i
    lib.truth_apply_cells.argtypes = [i64, i, i, i64, d, vp, vp, vp, vp, vp]
    lib.truth_apply_cells.restype = i
    lib.truth_grad_cells.argtypes = [i64, i, i, i64, d] + [vp] * 9
    lib.truth_grad_cells.restype = i
    _lib = lib
    return lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---- Table B.1 and Alg. 1 ----------------------------------------------------

def table_row(k: int):
    """(m_k, q_k, r_k, theta_{m_k}) of Table B.1, k = 1..9."""
    lib = _load()
    m, q, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    th = ctypes.c_double()
    if lib.orc_table_row(k, ctypes.byref(m), ctypes.byref(q), ctypes.byref(r),
                         ctypes.byref(th)) != 0:
        raise ValueError("k must be in 1..9")
    return m.value, q.value, r.value, th.value


def taylor_coef(i: int) -> float:
    return _load().orc_taylor_coef(i)


def select(nrm: float, K: int = 9, option: int = 2):
    """(k*, m*, s*) of Alg. 1 for a finite norm."""
    lib = _load()
    k, m, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib.orc_select(float(nrm), K, option, ctypes.byref(k), ctypes.byref(m),
                   ctypes.byref(s))
    return k.value, m.value, s.value


# ---- one cell ----------------------------------------------------------------

def build_matrix(dt, rho_g, rho_d, t_stop):
    """A = dt K (velocity form), a, e, ||A||_1 and the bad-input bits."""
    lib = _load()
    rho_d = _f64(rho_d)
    t_stop = _f64(t_stop)
    N = rho_d.size
    A = np.zeros((N + 1, N + 1))
    a = np.zeros(N)
    e = np.zeros(N)
    nrm = ctypes.c_double()
    bad = lib.orc_build(N, float(dt), float(rho_g), _ptr(rho_d), _ptr(t_stop),
                        _ptr(A), _ptr(a), _ptr(e), ctypes.byref(nrm))
    return A, a, e, nrm.value, bad


def expm_minus_identity(A, nrm, K=9, option=2, xform=False):
    """Y = T_m(2^-s A)^(2^s) - I and (k*, m*, s*)."""
    lib = _load()
    A = _f64(A)
    n = A.shape[0]
    Y = np.zeros((n, n))
    kms = np.zeros(3, dtype=np.int32)
    rc = lib.orc_expm(n - 1, _ptr(A), float(nrm), K, option, int(bool(xform)),
                      _ptr(Y), _ptr(kms))
    if rc != 0:
        raise ValueError("orc_expm failed (%d)" % rc)
    return Y, tuple(int(x) for x in kms)


def cell_expm(dt, rho_g, rho_d, t_stop, K=9, option=2, xform=False):
    """E = exp(dt K) of one cell by the oracle, and (k*, m*, s*)."""
    lib = _load()
    rho_d = _f64(rho_d)
    t_stop = _f64(t_stop)
    N = rho_d.size
    E = np.zeros((N + 1, N + 1))
    kms = np.zeros(3, dtype=np.int32)
    bad = lib.orc_cell_expm(N, float(dt), float(rho_g), _ptr(rho_d),
                            _ptr(t_stop), K, option, int(bool(xform)), _ptr(E),
                            _ptr(kms))
    if bad:
        raise ValueError("bad cell (bits %d)" % bad)
    return E, tuple(int(x) for x in kms)


BOUND_TEST = 4  # option bit: Sastre's second modification in the Taylor stage
PADE = 8        # option bit: the diagonal Pade scaling step instead of Taylor


def pade_row(i: int):
    """(m, theta_m, coefficients c_0..c_m of N_mm) of the oracle's Pade row i = 0..4."""
    lib = _load()
    m, th = ctypes.c_int(), ctypes.c_double()
    c = np.zeros(14)
    if lib.orc_pade_row(i, ctypes.byref(m), ctypes.byref(th), _ptr(c)) != 0:
        raise ValueError("row must be in 0..4")
    return m.value, th.value, c[: m.value + 1].copy()


def pade_select(nrm: float):
    """(m, s) of the Pade scaling step for a finite norm."""
    lib = _load()
    m, s = ctypes.c_int(), ctypes.c_int()
    lib.orc_pade_select(float(nrm), ctypes.byref(m), ctypes.byref(s))
    return m.value, s.value


def taylor_stage(B, k, bound_test=False):
    """F = T_m(B) - I for row k of Table B.1 on the given (scaled) matrix B,
    with or without the bound test; returns (F, products skipped, b_exp)."""
    lib = _load()
    B = _f64(B)
    n = B.shape[0]
    F = np.zeros((n, n))
    sk = ctypes.c_int()
    be = ctypes.c_double()
    if lib.orc_taylor_stage(n, _ptr(B), int(k), int(bool(bound_test)), _ptr(F),
                            ctypes.byref(sk), ctypes.byref(be)) != 0:
        raise ValueError("bad Taylor-stage arguments")
    return F, sk.value, be.value


def grad_A(A, nrm, G, K=9, option=2):
    """dL/dA for L = <G, Y(A)>, by reverse mode through the stored chain."""
    lib = _load()
    A = _f64(A)
    G = _f64(G)
    n = A.shape[0]
    Ab = np.zeros((n, n))
    kms = np.zeros(3, dtype=np.int32)
    rc = lib.orc_grad_A(n - 1, _ptr(A), float(nrm), K, option, _ptr(G),
                        _ptr(Ab), _ptr(kms))
    if rc != 0:
        raise ValueError("orc_grad_A failed (%d)" % rc)
    return Ab


def truth_eigen(dt, rho_g, rho_d, t_stop):
    """exp(dt K) from the secular-equation eigen-decomposition (long double)."""
    lib = _load()
    rho_d = _f64(rho_d)
    t_stop = _f64(t_stop)
    N = rho_d.size
    E = np.zeros((N + 1, N + 1))
    rc = lib.truth_expm_eigen(N, float(dt), float(rho_g), _ptr(rho_d),
                              _ptr(t_stop), _ptr(E))
    if rc != 0:
        raise ValueError("truth_expm_eigen needs e_i > 0 and distinct a_i")
    return E


def truth_general(dt, rho_g, rho_d, t_stop):
    """exp(dt K) of any valid cell (long double): the eigen-decomposition
    with decoupled (t = inf), dust-free (rho_d = 0) and equal-a species split
    off in closed form."""
    lib = _load()
    rho_d = _f64(rho_d)
    t_stop = _f64(t_stop)
    N = rho_d.size
    E = np.zeros((N + 1, N + 1))
    rc = lib.truth_expm_general(N, float(dt), float(rho_g), _ptr(rho_d),
                                _ptr(t_stop), _ptr(E))
    if rc != 0:
        raise ValueError("truth_expm_general: invalid cell")
    return E


def truth_apply(rho_g, rho_d, t_stop, v, dt):
    """The exact v' = exp(dt K) v for every cell of an SoA grid (long-double
    truth_general); NaN on cells with invalid inputs."""
    lib = _load()
    rho_g, rho_d, t_stop, v = (_f64(x) for x in (rho_g, rho_d, t_stop, v))
    D, n, C = v.shape
    assert rho_d.shape == (n - 1, C) and t_stop.shape == (n - 1, C) and rho_g.shape == (C,)
    out = np.empty_like(v)
    if C:
        lib.truth_apply_cells(C, n - 1, D, C, float(dt), _ptr(rho_g), _ptr(rho_d),
                              _ptr(t_stop), _ptr(v), _ptr(out))
    return out


def truth_grad(rho_g, rho_d, t_stop, v, w, dt):
    """The exact gradient of L = sum w . exp(dt K) v per cell (long double,
    Daleckii-Krein form in the eigenbasis): (g_v, g_logt, g_rho_d, g_rho_g);
    NaN on cells the eigen-decomposition cannot take (a species with e_i = 0
    or a_i = 0, equal a_i) or with invalid inputs."""
    lib = _load()
    rho_g, rho_d, t_stop, v, w = (_f64(x) for x in (rho_g, rho_d, t_stop, v, w))
    D, n, C = v.shape
    assert w.shape == v.shape and rho_d.shape == (n - 1, C) and t_stop.shape == (n - 1, C)
    g_v = np.empty_like(v)
    g_lt = np.empty((n - 1, C))
    g_rd = np.empty((n - 1, C))
    g_rg = np.empty(C)
    if C:
        lib.truth_grad_cells(C, n - 1, D, C, float(dt), _ptr(rho_g), _ptr(rho_d), _ptr(t_stop),
                             _ptr(v), _ptr(w), _ptr(g_v), _ptr(g_lt), _ptr(g_rd), _ptr(g_rg))
    return g_v, g_lt, g_rd, g_rg


def truth_taylor(A, terms=200):
    """The power series of exp(A) in long double (meaningful for ||A||_1 <= 7)."""
    lib = _load()
    A = _f64(A)
    n = A.shape[0]
    E = np.zeros((n, n))
    if lib.truth_expm_taylor(n, _ptr(A), int(terms), _ptr(E)) != 0:
        raise ValueError("bad size")
    return E


# ---- SoA grids (the library's layout) ---------------------------------------

def apply_cells(rho_g, rho_d, t_stop, v, dt, K=9, option=2, xform=False):
    """Oracle v' for every cell of an SoA grid.

    rho_g [C]; rho_d, t_stop [N][C]; v [D][N+1][C].  Returns
    (v_out, kms [3][C] int32, nrm [C], status bits).
    """
    lib = _load()
    rho_g = _f64(rho_g)
    rho_d = _f64(rho_d)
    t_stop = _f64(t_stop)
    v = _f64(v)
    D, n, C = v.shape
    N = n - 1
    assert rho_d.shape == (N, C) and t_stop.shape == (N, C) and rho_g.shape == (C,)
    out = np.empty_like(v)
    kms = np.zeros((3, C), dtype=np.int32)
    nrm = np.zeros(C)
    st = lib.orc_apply_cells(C, N, D, C, float(dt), K, option, int(bool(xform)),
                             _ptr(rho_g), _ptr(rho_d), _ptr(t_stop), _ptr(v),
                             _ptr(out), _ptr(kms), _ptr(nrm))
    if st < 0:
        raise ValueError("orc_apply_cells rejected its arguments (%d)" % st)
    return out, kms, nrm, st


def grad_cells(rho_g, rho_d, t_stop, v, w, dt, K=9, option=2):
    """Oracle gradients of L = sum w . v' for every cell of an SoA grid.

    Returns (v_out, g_v, g_logt, g_rho_d, g_rho_g, status bits).
    """
    lib = _load()
    rho_g = _f64(rho_g)
    rho_d = _f64(rho_d)
    t_stop = _f64(t_stop)
    v = _f64(v)
    w = _f64(w)
    D, n, C = v.shape
    N = n - 1
    assert w.shape == v.shape
    v_out = np.empty_like(v)
    g_v = np.empty_like(v)
    g_logt = np.empty((N, C))
    g_rho_d = np.empty((N, C))
    g_rho_g = np.empty(C)
    st = lib.orc_grad_cells(C, N, D, C, float(dt), K, option, _ptr(rho_g),
                            _ptr(rho_d), _ptr(t_stop), _ptr(v), _ptr(w),
                            _ptr(v_out), _ptr(g_v), _ptr(g_logt), _ptr(g_rho_d),
                            _ptr(g_rho_g))
    if st < 0:
        raise ValueError("orc_grad_cells rejected its arguments (%d)" % st)
    return v_out, g_v, g_logt, g_rho_d, g_rho_g, st


def rk1_cells(rho_g, rho_d, t_stop, v, dt):
    """The implicit RK1 drag step v' = (I - dt K)^{-1} v for every cell
    (dense Gaussian elimination; rk1.c).  Returns (v_out, status bits)."""
    lib = _load()
    rho_g, rho_d, t_stop, v = (_f64(x) for x in (rho_g, rho_d, t_stop, v))
    D, n, C = v.shape
    out = np.empty_like(v)
    st = lib.orc_rk1_cells(C, n - 1, D, C, float(dt), _ptr(rho_g), _ptr(rho_d), _ptr(t_stop),
                           _ptr(v), _ptr(out))
    if st < 0:
        raise ValueError("orc_rk1_cells: bad arguments")
    return out, st

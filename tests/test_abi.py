"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every symbol include/dragexp.h declares;
invalid arguments must be rejected on the host before anything is enqueued;
the library's copy of Table B.1 and its Alg. 1 selection (the same code the
kernels run, compiled for the host) must agree with the oracle exactly.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2509_25347_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.SO_PATH):
        _lib.build()
    return _lib.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "dragexp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(drag_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11, -20):
        s = _lib.status_string(code)
        assert s and s != "unknown status code", code
    assert _lib.status_string(12345) == "unknown status code"


def _apply(L, desc, ptrs=(1, 2, 3, 4, 5)):
    p = [ctypes.c_void_p(x) if x else None for x in ptrs]
    return L.drag_expm_apply(ctypes.byref(desc) if desc is not None else None, *p, None)


def test_argument_errors_return_before_launch(L):
    good = dict(n_cells=10, n_species=4, n_dim=3, ld=10, dt=1.0, k_max=9, option=2)

    def mk(**kw):
        a = dict(good)
        a.update(kw)
        return _lib.make_desc(**a)

    # use fake but non-overlapping pointers: the checks run before any HIP call
    base = [1 << 20, 2 << 20, 3 << 20, 4 << 20, 8 << 20]
    assert _apply(L, None, base) == _lib.ERR_NULL_DESC
    assert _apply(L, mk(n_cells=-1), base) == _lib.ERR_N_CELLS
    assert _apply(L, mk(n_species=0), base) == _lib.ERR_N_SPECIES
    assert _apply(L, mk(n_species=33), base) == _lib.ERR_N_SPECIES
    assert _apply(L, mk(n_dim=0), base) == _lib.ERR_N_DIM
    assert _apply(L, mk(n_dim=4), base) == _lib.ERR_N_DIM
    assert _apply(L, mk(ld=9), base) == _lib.ERR_LD
    assert _apply(L, mk(dt=-1.0), base) == _lib.ERR_DT
    assert _apply(L, mk(dt=float("nan")), base) == _lib.ERR_DT
    assert _apply(L, mk(dt=float("inf")), base) == _lib.ERR_DT
    assert _apply(L, mk(k_max=-1), base) == _lib.ERR_K_MAX
    assert _apply(L, mk(k_max=10), base) == _lib.ERR_K_MAX
    assert _apply(L, mk(option=3), base) == _lib.ERR_OPTION
    assert _apply(L, mk(option=3 | _lib.OPTION_BOUND_TEST), base) == _lib.ERR_OPTION
    assert _apply(L, mk(option=16), base) == _lib.ERR_OPTION
    assert _apply(L, mk(), [1 << 20, 0, 3 << 20, 4 << 20, 8 << 20]) == _lib.ERR_NULL_POINTER
    # v_out overlapping rho_d (not the allowed in-place v_in)
    assert _apply(L, mk(), [1 << 20, 2 << 20, 3 << 20, 4 << 20, (2 << 20) + 8]) == _lib.ERR_ALIAS
    assert _apply(L, mk(), [1 << 20, 2 << 20, 3 << 20, 4 << 20, (4 << 20) + 8]) == _lib.ERR_ALIAS
    # n_cells = 0 is a no-op, even with NULL pointers
    assert _apply(L, mk(n_cells=0, ld=1), [0, 0, 0, 0, 0]) == _lib.OK


def test_backward_argument_errors(L):
    d = _lib.make_desc(10, 4, 3, 10, 1.0)
    nul = [None] * 12
    assert L.drag_expm_apply_backward(None, *nul) == _lib.ERR_NULL_DESC
    bad = _lib.make_desc(10, 20, 3, 10, 1.0)
    assert L.drag_expm_apply_backward(ctypes.byref(bad), *nul) == _lib.ERR_N_SPECIES
    # the forward goes to 32 species, the adjoint stops at 16
    bad17 = _lib.make_desc(10, 17, 3, 10, 1.0)
    assert L.drag_expm_apply_backward(ctypes.byref(bad17), *nul) == _lib.ERR_N_SPECIES
    assert L.drag_expm_apply_backward(ctypes.byref(d), *nul) == _lib.ERR_NULL_POINTER
    # the adjoint takes no bound test (checked before anything is enqueued)
    bt = _lib.make_desc(10, 4, 3, 10, 1.0, 9, 2 | _lib.OPTION_BOUND_TEST)
    ptrs = [ctypes.c_void_p(x) for x in (1 << 20, 2 << 20, 3 << 20, 4 << 20, 5 << 20)]
    outs = [ctypes.c_void_p(x) for x in (6 << 20, 7 << 20, 8 << 20, 9 << 20, 10 << 20, 11 << 20)]
    assert L.drag_expm_apply_backward(ctypes.byref(bt), *ptrs, *outs, None) == _lib.ERR_OPTION


def test_table_matches_oracle(L, orc):
    for k in range(1, 10):
        assert _lib.table_row(k) == orc.table_row(k)


def test_selection_matches_oracle_exactly(L, orc):
    rng = np.random.default_rng(17)
    norms = list(10.0 ** rng.uniform(-10, 12, 4000)) + [0.0]
    for k in range(1, 10):
        th = orc.table_row(k)[3]
        for f in (1, 2, 4, 8, 1 << 20):
            x = th * f
            norms += [x, float(np.nextafter(x, 0)), float(np.nextafter(x, np.inf))]
    for K in range(1, 10):
        for opt in (0, 1, 2):
            for nrm in norms:
                assert _lib.select(nrm, K, opt) == orc.select(nrm, K, opt), (nrm, K, opt)


def test_batched_plan_argument_errors(L):
    plan = ctypes.c_void_p()
    assert L.drag_plan_batched(None, ctypes.byref(plan)) == _lib.ERR_NULL_DESC
    ns = (ctypes.c_int32 * 3)(1, 5, 16)
    P32 = ctypes.POINTER(ctypes.c_int32)
    def d(**kw):
        a = dict(n_blocks=3, block_cells=8, n_dim=3, k_max=9, option=2, dt=1.0)
        a.update(kw)
        return _lib.DragBatchDesc(a["n_blocks"], a["block_cells"], a["n_dim"], a["k_max"],
                                  a["option"], a["dt"], ctypes.cast(ns, P32))
    assert L.drag_plan_batched(ctypes.byref(d(n_blocks=0)), ctypes.byref(plan)) == _lib.ERR_PLAN
    assert L.drag_plan_batched(ctypes.byref(d(n_dim=4)), ctypes.byref(plan)) == _lib.ERR_N_DIM
    assert L.drag_plan_batched(ctypes.byref(d(dt=-1.0)), ctypes.byref(plan)) == _lib.ERR_DT
    assert L.drag_plan_batched(ctypes.byref(d(k_max=-1)), ctypes.byref(plan)) == _lib.ERR_K_MAX
    assert L.drag_plan_batched(ctypes.byref(d(option=5)), ctypes.byref(plan)) == _lib.ERR_OPTION
    bad = (ctypes.c_int32 * 3)(1, 0, 16)
    dd = d()
    dd.n_species = ctypes.cast(bad, P32)
    assert L.drag_plan_batched(ctypes.byref(dd), ctypes.byref(plan)) == _lib.ERR_N_SPECIES
    assert L.drag_expm_apply_batched(None, None, None, None, None) == _lib.ERR_PLAN
    assert L.drag_plan_offsets(None, None, None, None, None) == _lib.ERR_PLAN
    assert L.drag_plan_config(None, None, None) == _lib.ERR_PLAN
    assert L.drag_plan_set_config(None, 6, 0) == _lib.ERR_PLAN
    assert L.drag_plan_destroy(None) == _lib.OK


def test_mapping_controls(L):
    for N in range(1, 17):
        assert _lib.get_mapping(N) in (_lib.MAP_LANE, _lib.MAP_WAVE)
    _lib.set_mapping(3, _lib.MAP_WAVE)
    assert _lib.get_mapping(3) == _lib.MAP_WAVE
    _lib.set_mapping(3, _lib.MAP_AUTO)
    _lib.set_mapping(12, _lib.MAP_LANE)  # the forward's pair of lanes goes to 12
    assert _lib.get_mapping(12) == _lib.MAP_LANE
    _lib.set_mapping(12, _lib.MAP_AUTO)
    with pytest.raises(_lib.DragError):
        _lib.set_mapping(13, _lib.MAP_LANE)
    with pytest.raises(_lib.DragError):
        _lib.set_mapping(0, _lib.MAP_WAVE)


def test_pade_table_matches_oracle(L, orc):
    """The library's Pade rows (degree, theta, coefficients) equal the
    oracle's bit for bit (each side has its own copy)."""
    for i in range(5):
        m, th, c = _lib.pade_row(i)
        mo, tho, co = orc.pade_row(i)
        assert (m, th) == (mo, tho)
        assert np.array_equal(c, co)
    with pytest.raises(_lib.DragError):
        _lib.pade_row(5)


def test_pade_option_errors(L):
    def mk(opt):
        return _lib.make_desc(10, 4, 3, 10, 1.0, 9, opt)
    base = [1 << 20, 2 << 20, 3 << 20, 4 << 20, 5 << 20]
    both = _lib.OPTION_PADE | _lib.OPTION_BOUND_TEST | 2
    assert _apply(L, mk(both), base) == _lib.ERR_OPTION
    assert _apply(L, mk(_lib.OPTION_PADE | 3), base) == _lib.ERR_OPTION
    # the large-N forward (17..32 species) has the plain Taylor step only
    big = _lib.make_desc(10, 20, 3, 10, 1.0, 9, 2 | _lib.OPTION_PADE)
    assert _apply(L, big, base) == _lib.ERR_OPTION
    big = _lib.make_desc(10, 20, 3, 10, 1.0, 9, 2 | _lib.OPTION_BOUND_TEST)
    assert _apply(L, big, base) == _lib.ERR_OPTION
    ptrs = [ctypes.c_void_p(x) for x in base]
    outs = [ctypes.c_void_p(x) for x in (6 << 20, 7 << 20, 8 << 20, 9 << 20, 10 << 20, 11 << 20)]
    d = mk(_lib.OPTION_PADE)
    assert L.drag_expm_apply_backward(ctypes.byref(d), *ptrs, *outs, None) == _lib.ERR_OPTION


def test_taylor_cap_controls(L):
    """K_AUTO resolves per N to a cap in 3..9; overrides stick until reset;
    out-of-range arguments are rejected without changing anything."""
    ks = [_lib.get_k_max(N) for N in range(1, 17)]
    assert all(3 <= k <= 9 for k in ks)
    _lib.set_k_max(5, 8)
    assert _lib.get_k_max(5) == 8
    _lib.set_k_max(5, _lib.K_AUTO)
    assert _lib.get_k_max(5) == ks[4]
    for bad in ((0, 5), (17, 5), (5, 10), (5, -1)):
        with pytest.raises(_lib.DragError):
            _lib.set_k_max(*bad)
    assert [_lib.get_k_max(N) for N in range(1, 17)] == ks
    k = ctypes.c_int32()
    assert L.drag_get_k_max(5, None) == _lib.ERR_NULL_POINTER
    assert L.drag_get_k_max(0, ctypes.byref(k)) == _lib.ERR_N_SPECIES
    assert L.drag_plan_k_max(None, ctypes.byref(k)) == _lib.ERR_PLAN


def test_expm_steps_argument_errors(L):
    """drag_expm_steps rejects a negative step count before touching the GPU."""
    d = _lib.make_desc(0, 2, 1, 1, 0.1, 9, 2)
    assert L.drag_expm_steps(ctypes.byref(d), None, None, None, None, None, -1, None, None) == _lib.ERR_STEPS
    assert L.drag_expm_steps(ctypes.byref(d), None, None, None, None, None, 5, None, None) == _lib.OK
    assert L.drag_expm_steps(None, None, None, None, None, None, 1, None, None) == _lib.ERR_NULL_DESC

"""ctypes binding of libdragexp.so (the C ABI in include/dragexp.h).

Argument marshalling only: every step of the drag update runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.
There is no CPU fallback: without the built library (or without a GPU) the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libdragexp.so")
SOURCES = [os.path.join(_HERE, "csrc", "dragexp.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # MFMA accumulators in ordinary VGPRs: no AGPR round trips around chains
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# status codes (include/dragexp.h)
OK = 0
ERR_NULL_DESC = -1
ERR_N_CELLS = -2
ERR_N_SPECIES = -3
ERR_N_DIM = -4
ERR_LD = -5
ERR_DT = -6
ERR_K_MAX = -7
ERR_OPTION = -8
ERR_NULL_POINTER = -9
ERR_ALIAS = -10
ERR_PLAN = -11
ERR_STEPS = -12
ERR_SCRATCH = -13
STATIC_SCRATCH_BYTES = 1 << 20
ERR_HIP = -20

CELL_BAD_DENSITY = 1
CELL_BAD_STOPPING_TIME = 2
CELL_BAD_VELOCITY = 4
CELL_BAD_NORM = 8

MAP_AUTO, MAP_LANE, MAP_WAVE = 0, 1, 2
K_AUTO = 0
OPTION_BOUND_TEST = 4  # option bit: the second modification (bound test)
OPTION_PADE = 8        # option bit: the diagonal Pade scaling step

EXPORTS = [
    "drag_desc_init", "drag_build", "drag_expm_apply", "drag_expm_steps", "drag_rk1_apply", "drag_expm_apply_backward",
    "drag_plan_batched", "drag_plan_offsets", "drag_expm_apply_batched",
    "drag_plan_autotune", "drag_plan_config", "drag_plan_set_config", "drag_plan_destroy", "drag_get_status", "drag_clear_status", "drag_status_string",
    "drag_table_row", "drag_select", "drag_set_mapping", "drag_get_mapping",
    "drag_set_k_max", "drag_get_k_max", "drag_plan_k_max", "drag_pade_row",
    "drag_expm_apply_batched_static",
]


class DragDesc(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int64),
        ("n_species", ctypes.c_int32),
        ("n_dim", ctypes.c_int32),
        ("ld", ctypes.c_int64),
        ("dt", ctypes.c_double),
        ("k_max", ctypes.c_int32),
        ("option", ctypes.c_int32),
    ]


class DragBatchDesc(ctypes.Structure):
    _fields_ = [
        ("n_blocks", ctypes.c_int32),
        ("block_cells", ctypes.c_int32),
        ("n_dim", ctypes.c_int32),
        ("k_max", ctypes.c_int32),
        ("option", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("n_species", ctypes.POINTER(ctypes.c_int32)),
    ]


class DragError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = status_string(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def build() -> str:
    """Compile libdragexp.so in-tree with hipcc for gfx950."""
    tmp = SO_PATH + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + SOURCES + ["-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO_PATH)
    return SO_PATH


_lib = None


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise RuntimeError(
            "libdragexp.so is not built (run __graft_entry__.build() or "
            "paper_2509_25347_amd._lib.build()); there is no CPU fallback")
    L = ctypes.CDLL(SO_PATH)
    P = ctypes.POINTER
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    desc_p = P(DragDesc)
    L.drag_desc_init.argtypes = [desc_p, i64, i32, i32, d]
    L.drag_desc_init.restype = None
    L.drag_build.argtypes = [desc_p] + [vp] * 9 + [vp]
    L.drag_build.restype = ctypes.c_int
    L.drag_expm_apply.argtypes = [desc_p] + [vp] * 5 + [vp]
    L.drag_expm_apply.restype = ctypes.c_int
    L.drag_expm_apply_backward.argtypes = [desc_p] + [vp] * 11 + [vp]
    L.drag_expm_apply_backward.restype = ctypes.c_int
    L.drag_plan_batched.argtypes = [P(DragBatchDesc), P(vp)]
    L.drag_plan_batched.restype = ctypes.c_int
    L.drag_plan_offsets.argtypes = [vp, vp, vp, P(i64), P(i64)]
    L.drag_plan_offsets.restype = ctypes.c_int
    L.drag_expm_apply_batched.argtypes = [vp, vp, vp, vp, vp]
    L.drag_expm_apply_batched.restype = ctypes.c_int
    L.drag_expm_apply_batched_static.argtypes = [P(DragBatchDesc), vp, vp, vp, vp]
    L.drag_expm_apply_batched_static.restype = ctypes.c_int
    L.drag_plan_autotune.argtypes = [vp, vp, vp, vp, vp, P(i32)]
    L.drag_plan_autotune.restype = ctypes.c_int
    L.drag_rk1_apply.argtypes = [P(DragDesc), vp, vp, vp, vp, vp, vp]
    L.drag_rk1_apply.restype = ctypes.c_int
    L.drag_expm_steps.argtypes = [P(DragDesc), vp, vp, vp, vp, vp, ctypes.c_int64, vp, vp]
    L.drag_expm_steps.restype = ctypes.c_int
    L.drag_plan_config.argtypes = [vp, P(i32), P(i32)]
    L.drag_plan_config.restype = ctypes.c_int
    L.drag_plan_set_config.argtypes = [vp, i32, i32]
    L.drag_plan_set_config.restype = ctypes.c_int
    L.drag_plan_destroy.argtypes = [vp]
    L.drag_plan_destroy.restype = ctypes.c_int
    L.drag_get_status.argtypes = [vp, P(i32)]
    L.drag_get_status.restype = ctypes.c_int
    L.drag_clear_status.argtypes = [vp]
    L.drag_clear_status.restype = ctypes.c_int
    L.drag_status_string.argtypes = [ctypes.c_int]
    L.drag_status_string.restype = ctypes.c_char_p
    L.drag_table_row.argtypes = [ctypes.c_int, P(i32), P(i32), P(i32), P(d)]
    L.drag_table_row.restype = ctypes.c_int
    L.drag_select.argtypes = [d, i32, i32, P(i32), P(i32), P(i32)]
    L.drag_select.restype = ctypes.c_int
    L.drag_set_mapping.argtypes = [i32, i32]
    L.drag_set_mapping.restype = ctypes.c_int
    L.drag_get_mapping.argtypes = [i32, P(i32)]
    L.drag_get_mapping.restype = ctypes.c_int
    L.drag_set_k_max.argtypes = [i32, i32]
    L.drag_set_k_max.restype = ctypes.c_int
    L.drag_get_k_max.argtypes = [i32, P(i32)]
    L.drag_get_k_max.restype = ctypes.c_int
    L.drag_pade_row.argtypes = [i32, P(i32), P(ctypes.c_double), vp]
    L.drag_pade_row.restype = ctypes.c_int
    L.drag_plan_k_max.argtypes = [vp, P(i32)]
    L.drag_plan_k_max.restype = ctypes.c_int
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().drag_status_string(int(code)).decode()


def check(code: int, what: str = "") -> None:
    if code != OK:
        raise DragError(code, what)


def make_desc(n_cells, n_species, n_dim, ld, dt, k_max=9, option=2) -> DragDesc:
    return DragDesc(int(n_cells), int(n_species), int(n_dim), int(ld), float(dt),
                    int(k_max), int(option))


# ---- host-side helpers (no GPU needed) ----------------------------------------

def table_row(k: int):
    m, q, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    th = ctypes.c_double()
    check(lib().drag_table_row(k, ctypes.byref(m), ctypes.byref(q), ctypes.byref(r),
                               ctypes.byref(th)), "drag_table_row")
    return m.value, q.value, r.value, th.value


def select(norm: float, k_max: int = 9, option: int = 2):
    k, m, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().drag_select(float(norm), k_max, option, ctypes.byref(k), ctypes.byref(m),
                            ctypes.byref(s)), "drag_select")
    return k.value, m.value, s.value


def set_mapping(n_species: int, mapping: int) -> None:
    check(lib().drag_set_mapping(n_species, mapping), "drag_set_mapping")


def get_mapping(n_species: int) -> int:
    m = ctypes.c_int32()
    check(lib().drag_get_mapping(n_species, ctypes.byref(m)), "drag_get_mapping")
    return m.value


def pade_row(row: int):
    """(m, theta_m, numerator coefficients) of the library's Pade row 0..4."""
    import numpy as np
    m, th = ctypes.c_int32(), ctypes.c_double()
    c = np.zeros(14)
    check(lib().drag_pade_row(row, ctypes.byref(m), ctypes.byref(th),
                              c.ctypes.data_as(ctypes.c_void_p)), "drag_pade_row")
    return m.value, th.value, c[: m.value + 1].copy()


def set_k_max(n_species: int, k_max: int) -> None:
    """Override the Taylor cap K that K_AUTO means for this N (0 restores)."""
    check(lib().drag_set_k_max(n_species, k_max), "drag_set_k_max")


def get_k_max(n_species: int) -> int:
    """The Taylor cap K that K_AUTO means for this N."""
    k = ctypes.c_int32()
    check(lib().drag_get_k_max(n_species, ctypes.byref(k)), "drag_get_k_max")
    return k.value

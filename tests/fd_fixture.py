"""Reader of tests/golden/fd_gradients.json (multiprecision central
differences of L = sum w . v', written by tests/golden/make_fd_gradients.py
from oracle/mpfd.py)."""
import json
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_gradients.json")


def _arr(x, shape=None):
    a = np.array([float.fromhex(y) for y in x])
    return a if shape is None else a.reshape(shape)


def load(N):
    """SoA inputs (rho_g [C], rho_d, t_stop [N][C], v, w [D][N+1][C], dt) and
    the differences (g_logt, g_rho_d [N][C], g_rho_g [C], g_v [D][N+1][C])."""
    with open(PATH) as f:
        data = json.load(f)
    D = data["D"]
    cells = data["cases"][str(N)]
    col = lambda key, shape: np.stack([_arr(c[key], shape) for c in cells], axis=-1)  # noqa: E731
    d = dict(rho_g=np.array([float.fromhex(c["rho_g"]) for c in cells]),
             rho_d=col("rho_d", (N,)), t_stop=col("t_stop", (N,)),
             v=col("v", (D, N + 1)), w=col("w", (D, N + 1)), dt=data["dt"])
    g = dict(g_logt=col("g_logt", (N,)), g_rho_d=col("g_rho_d", (N,)),
             g_rho_g=np.array([float.fromhex(c["g_rho_g"]) for c in cells]),
             g_v=col("g_v", (D, N + 1)))
    return d, g


def group_rel_err(got, ref):
    """Per cell: max |got - ref| / max |ref| over the group (cell axis last)."""
    g = np.moveaxis(np.asarray(got), -1, 0).reshape(np.shape(got)[-1], -1)
    r = np.moveaxis(np.asarray(ref), -1, 0).reshape(np.shape(ref)[-1], -1)
    return np.abs(g - r).max(axis=1) / np.abs(r).max(axis=1)

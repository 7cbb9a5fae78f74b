"""Seeded synthetic inputs for the drag update (shared by tests and bench).

This module draws inputs only; it holds none of the method's arithmetic.
The paper measures on the Dustywave and Collisions setups (Sect. 3.1, 3.4),
whose Dustywave stopping times come from an external table that is not
reproduced here; these seeded draws stand in for them with the same shapes:
per-cell gas density, N dust densities and N stopping times, and D = 1..3
velocity components of the gas and every dust species.

Layout (structure of arrays, cell index fastest):
    rho_g [C], rho_d [N][C], t_stop [N][C], v [D][N+1][C]
with row 0 of v the gas and rows 1..N the dust species.

Cells are drawn in chunks of ``CHUNK`` with a generator seeded by
(25347 + config id, chunk index), so the first k cells of a workload are the
same whatever its total size: small test cases are prefixes of the full ones.
"""
from __future__ import annotations

import numpy as np

CHUNK = 4096
SEED_BASE = 25347
DT = 1.0

#: name -> (config id, cells, species N, components D)
WORKLOADS = {
    "n1_closed_form": (1, 4096, 1, 1),
    "n4_3d": (2, 1 << 20, 4, 3),
    "n16_stiff_3d": (3, 1 << 20, 16, 3),
    "n8_adjoint_3d": (5, 1 << 18, 8, 3),
}


def _rng(cfg: int, chunk: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE + cfg, chunk])


def _loguniform(rng, lo_exp, hi_exp, size):
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size)


def _chunk_n1(rng, c):
    rho_g = rng.uniform(0.5, 2.0, c)
    eps = _loguniform(rng, -3.0, 1.0, c)
    t = _loguniform(rng, -4.0, 2.0, c) * DT
    v = rng.standard_normal((1, 2, c))
    return rho_g, (eps * rho_g)[None, :], t[None, :], v


def _chunk_jittered(rng, c, N, D, t_lo, t_hi):
    """rho_g ~ U[0.5,2]; eps_i ~ logU[1e-3,1] i.i.d.; t_i log-spaced over
    [t_lo, t_hi] dt with +-20 % uniform jitter; v ~ N(0,1)."""
    rho_g = rng.uniform(0.5, 2.0, c)
    eps = _loguniform(rng, -3.0, 0.0, (N, c))
    if N == 1:
        base = np.array([np.sqrt(t_lo * t_hi)])
    else:
        base = np.logspace(np.log10(t_lo), np.log10(t_hi), N)
    t = base[:, None] * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, (N, c))) * DT
    v = rng.standard_normal((D, N + 1, c))
    return rho_g, eps * rho_g[None, :], t, v


def _chunk_stiff(rng, c, N, D):
    """MRN-like size bins: t_i log-spaced over [1e-6, 1e2] dt (no jitter),
    total dust-to-gas ratio ~ logU[1e-2, 1] split as eps_i ~ sqrt(t_i)
    (grain size a_i ~ t_i in the Epstein regime, eq. 1); N = 1 uses the log
    midpoint t_1 = 1e-2 dt."""
    rho_g = rng.uniform(0.5, 2.0, c)
    if N == 1:
        base = np.array([1e-2])
    else:
        base = np.logspace(-6.0, 2.0, N)
    t = np.repeat(base[:, None], c, axis=1) * DT
    eps_tot = _loguniform(rng, -2.0, 0.0, c)
    wgt = np.sqrt(base) / np.sqrt(base).sum()
    eps = wgt[:, None] * eps_tot[None, :]
    v = rng.standard_normal((D, N + 1, c))
    return rho_g, eps * rho_g[None, :], t, v


def _draw(cfg, n_cells, fn):
    parts = []
    for k in range(0, (n_cells + CHUNK - 1) // CHUNK):
        c = min(CHUNK, n_cells - k * CHUNK)
        parts.append(fn(_rng(cfg, k), c))
    cat = lambda i, ax: np.ascontiguousarray(np.concatenate([p[i] for p in parts], axis=ax))
    return dict(rho_g=cat(0, 0), rho_d=cat(1, 1), t_stop=cat(2, 1), v=cat(3, 2), dt=DT)


def make(name: str, n_cells: int | None = None, with_weights: bool = False) -> dict:
    """Inputs of a named workload (first ``n_cells`` cells if given).

    Returns dict(rho_g, rho_d, t_stop, v, dt[, w]) as float64 numpy arrays.
    """
    cfg, full, N, D = WORKLOADS[name]
    C = full if n_cells is None else int(n_cells)
    if cfg == 1:
        out = _draw(cfg, C, lambda r, c: _chunk_n1(r, c))
    elif cfg == 2:
        out = _draw(cfg, C, lambda r, c: _chunk_jittered(r, c, N, D, 1e-3, 10.0))
    elif cfg == 3:
        out = _draw(cfg, C, lambda r, c: _chunk_stiff(r, c, N, D))
    elif cfg == 5:
        out = _draw(cfg, C, lambda r, c: _chunk_jittered(r, c, N, D, 1e-3, 10.0))
    else:
        raise KeyError(name)
    if with_weights:
        wr = np.random.default_rng([SEED_BASE + cfg, 1 << 30])
        out["w"] = wr.standard_normal(out["v"].shape)
    return out


def make_stiff(N: int, n_cells: int, D: int = 3, cfg: int = 3) -> dict:
    """MRN-like stiff cells (the N = 16 recipe) for any species count N."""
    return _draw(100 + cfg * 32 + N, n_cells, lambda r, c: _chunk_stiff(r, c, N, D))


def make_jittered(N: int, n_cells: int, D: int = 3, cfg: int = 2) -> dict:
    """Jittered log-spaced cells (the N = 4 recipe) for any species count N."""
    return _draw(200 + cfg * 32 + N, n_cells,
                 lambda r, c: _chunk_jittered(r, c, N, D, 1e-3, 10.0))


# ---- AMR-style batches with uneven species counts ----------------------------

def make_batched(n_blocks: int = 4096, block_cells: int = 512, D: int = 3,
                 n_max: int = 16, seed_cfg: int = 4) -> dict:
    """Blocks of ``block_cells`` cells, each with its own N_b ~ U{1..n_max},
    drawn with the stiff recipe for its N_b.

    Returns dict(n_species [B] int32, blocks: list of per-block dicts with
    rho_g [b], rho_d [N_b][b], t_stop [N_b][b], v [D][N_b+1][b], dt).
    """
    rng = np.random.default_rng([SEED_BASE + seed_cfg, 0])
    ns = rng.integers(1, n_max + 1, n_blocks).astype(np.int32)
    blocks = []
    for b in range(n_blocks):
        r = np.random.default_rng([SEED_BASE + seed_cfg, 1 + b])
        rg, rd, t, v = _chunk_stiff(r, block_cells, int(ns[b]), D)
        blocks.append(dict(rho_g=rg, rho_d=rd, t_stop=t, v=v))
    return dict(n_species=ns, blocks=blocks, dt=DT, block_cells=block_cells, D=D)

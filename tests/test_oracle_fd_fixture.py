"""The stored multiprecision finite differences (tests/golden/fd_gradients.json)
against the oracle's reverse-mode gradient, which derives the same numbers
another way (the paper's dense FP64 steps run backwards, Sect. 2.3 and
App. B): 1e-8 of each group's largest entry per cell, on every stored cell;
and one stored cell recomputed from oracle/mpfd.py to the digit."""
import numpy as np
import pytest

from fd_fixture import group_rel_err, load

pytest.importorskip("mpmath")


@pytest.mark.parametrize("N", [5, 8, 10, 12])
def test_fd_fixture_matches_oracle_gradient(orc, N):
    d, g = load(N)
    rv, rgv, rlt, rrho, rrg, st = orc.grad_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"],
                                                 d["w"], d["dt"])
    assert st == 0
    for name, got in (("g_logt", rlt), ("g_rho_d", rrho), ("g_v", rgv)):
        e = group_rel_err(got, g[name])
        assert e.max() <= 1e-8, (N, name, e)
    e = np.abs(rrg - g["g_rho_g"]) / np.abs(g["g_rho_g"])
    assert e.max() <= 1e-8, (N, "g_rho_g", e)


def test_fd_fixture_recomputes():
    from oracle import mpfd
    d, g = load(5)
    c = 3
    r = mpfd.fd_gradients(d["rho_g"][c], d["rho_d"][:, c], d["t_stop"][:, c], d["v"][:, :, c],
                          d["w"][:, :, c], dt=d["dt"])
    assert np.array_equal(r["g_logt"], g["g_logt"][:, c])
    assert np.array_equal(r["g_rho_d"], g["g_rho_d"][:, c])
    assert r["g_rho_g"] == g["g_rho_g"][c]
    assert np.array_equal(r["g_v"], g["g_v"][:, :, c])

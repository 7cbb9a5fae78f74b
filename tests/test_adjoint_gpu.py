"""GPU parity of the fused forward + adjoint (drag_expm_apply_backward).

Gradients of L = sum w . v' with respect to v, log t_i, rho_i and rho_g.
References: the oracle's reverse-mode gradient (a different derivation: it
stores the chain and runs it backwards through the paper's dense steps),
central differences of a multiprecision forward (tests/golden/
fd_gradients.json), central differences of the GPU forward, and sum rules.
Per cell and per group (v, log t, rho_d, rho_g) the error is
    e = max |g - g_ref| / max(max |g_ref|, S),
with S = sum_c ||w_c||_inf ||v_c||_inf the natural size of L's sensitivities
(divided by rho_g for the density gradients): where every mode of a cell has
decayed, dL/dlog t is ~1e-16 and only its absolute error is meaningful.
e <= 1e-10 against the exact gradient (long double, oracle/truth.c), and
e <= 1e-10 + e(oracle, exact) against the oracle's (tests/bars.py).
Against the multiprecision differences: max |g - g_fd| / max |g_fd| <= 1e-8
per cell and group, for every adjoint kernel.  The fused forward v' meets the
forward's parity bars (tests/bars.py).
"""
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W
from bars import GRAD_TOL, check_forward, check_gradients, group_err, sens_scale
from fd_fixture import group_rel_err
from fd_fixture import load as load_fd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_25347_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ops(dev):
    from paper_2509_25347_amd import ops as _ops
    return _ops


def _to(d, dev, keys=("rho_g", "rho_d", "t_stop", "v", "w")):
    return {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in keys}


def _weights(d, seed=0):
    d = dict(d)
    d["w"] = np.random.default_rng(seed).standard_normal(d["v"].shape)
    return d


def gpu_backward(ops, d, dev, **kw):
    T = _to(d, dev)
    res = ops.expm_apply_backward(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], T["w"], d["dt"],
                                  want_grad_t=True, **kw)
    torch.cuda.synchronize()
    return [None if x is None else x.cpu().numpy() for x in res]


def check_vs_oracle(orc, d, got, tol, label):
    """The fused forward against the forward's bars, the gradients against
    the exact gradient and the oracle's (tests/bars.py), and dL/dt against
    dL/dlog t / t."""
    v_out, g_v, g_logt, g_rho, g_rho_g, g_t = got
    ro = orc.grad_cells(d["rho_g"], d["rho_d"], d["t_stop"], d["v"], d["w"], d["dt"])
    assert ro[-1] == 0
    check_forward(orc, v_out, ro[0], d, (label, "fused forward"))
    errs = check_gradients(orc, d, (g_v, g_logt, g_rho, g_rho_g), label, tol,
                           oracle_grads=ro[1:5])
    np.testing.assert_allclose(g_t, g_logt / d["t_stop"], rtol=1e-15, atol=0)
    return errs


@pytest.mark.parametrize("name,cells", [("n8_adjoint_3d", 3000 + 5), ("n4_3d", 2000 + 9),
                                        ("n16_stiff_3d", 600 + 1), ("n1_closed_form", 4096 + 3)])
def test_backward_vs_oracle(ops, dev, orc, name, cells):
    d = _weights(W.make(name, cells))
    got = gpu_backward(ops, d, dev)
    check_vs_oracle(orc, d, got, GRAD_TOL, name)


@pytest.mark.parametrize("N", list(range(1, 17)))
def test_backward_every_n_both_mappings(ops, dev, orc, N):
    from paper_2509_25347_amd import _lib
    d = _weights(W.make_stiff(N, 301) if N % 2 == 0 else W.make_jittered(N, 301), seed=N)
    maps = [_lib.MAP_WAVE] + ([_lib.MAP_LANE] if N <= 10 else [])
    try:
        for mp in maps:
            _lib.set_mapping(N, mp)
            got = gpu_backward(ops, d, dev)
            check_vs_oracle(orc, d, got, GRAD_TOL, f"N={N} map={mp}")
    finally:
        _lib.set_mapping(N, _lib.MAP_AUTO)


@pytest.mark.parametrize("N", [7, 8, 9, 10])
@pytest.mark.parametrize("D", [1, 2])
def test_backward_fewer_components(ops, dev, orc, N, D):
    """D = 1, 2 through the vector-ALU adjoints (the two-lane kernel at N = 8
    carries one direction vector per component): against the oracle."""
    d = _weights(W.make_stiff(N, 257, D=D), seed=10 * N + D)
    got = gpu_backward(ops, d, dev)
    check_vs_oracle(orc, d, got, GRAD_TOL, f"N={N} D={D}")


@pytest.mark.parametrize("N,mapping", [(3, None), (8, None), (10, None), (12, None), (8, 2)])
def test_backward_dt_zero(ops, dev, N, mapping):
    """dt = 0: exp(0) = I, so v' = v, dL/dv = w and every parameter gradient
    vanishes (A = dt K: each derivative carries a factor dt), on every
    adjoint kernel (one lane, two lanes with and without the direction
    recurrence, MFMA, MFMA block form)."""
    from paper_2509_25347_amd import _lib
    d = _weights(W.make_jittered(N, 130), seed=N)
    d["dt"] = 0.0
    try:
        if mapping is not None:
            _lib.set_mapping(N, mapping)
        v_out, g_v, g_logt, g_rho, g_rho_g, g_t = gpu_backward(ops, d, dev)
    finally:
        _lib.set_mapping(N, _lib.MAP_AUTO)
    assert np.array_equal(v_out, d["v"]), (N, mapping)
    np.testing.assert_allclose(g_v, d["w"], rtol=1e-15, atol=1e-15 * np.abs(d["w"]).max())
    for g in (g_logt, g_rho, g_rho_g, g_t):
        assert np.abs(g).max() == 0.0, (N, mapping)


def test_fused_forward_matches_forward(ops, dev):
    for name in ("n8_adjoint_3d", "n16_stiff_3d", "n4_3d"):
        d = _weights(W.make(name, 1000))
        T = _to(d, dev)
        fwd = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"]).cpu().numpy()
        got = gpu_backward(ops, d, dev)
        e = group_err(got[0], fwd)
        assert e.max() <= 1e-13, (name, e.max())


FD_CASES = {
    # name: (cells, N for the mapping override or None, mapping)
    "n8_adjoint_default": (lambda: W.make("n8_adjoint_3d", 6), None, None),
    "n3_lane": (lambda: W.make_jittered(3, 5), 3, 1),
    "n8_mfma_block": (lambda: W.make("n8_adjoint_3d", 6), 8, 2),
    "n12_mfma": (lambda: W.make_stiff(12, 5), 12, 2),
    "n10_pair": (lambda: W.make_jittered(10, 5), 10, 1),
}


MPFD_CASES = {
    # name: (species N of the stored cells, mapping override or None, kernel expected)
    "one_lane_n5": (5, None, "lane"),
    "pair_n8": (8, None, "pair"),
    "mfma_block_n8": (8, 2, "mfma block form"),
    "pair_n10": (10, None, "pair"),
    "mfma_n12": (12, None, "mfma"),
}


@pytest.mark.parametrize("case", sorted(MPFD_CASES))
def test_backward_vs_multiprecision_fd(ops, dev, orc, case):
    """The adjoint against central differences (h = 1e-6) of a multiprecision
    forward (mpmath expm at 30 digits; the stored 8 cells per N of the
    N = 8 adjoint workload's recipe): 1e-8 of each group's largest entry,
    per cell, for every adjoint kernel (one lane per cell, two lanes per cell
    at N = 8 and 10, the MFMA block form, the MFMA kernel above 10); and
    the oracle's gradient on the same cells to 1e-10."""
    from paper_2509_25347_amd import _lib
    N, mapping, _ = MPFD_CASES[case]
    d, fd = load_fd(N)
    if mapping is not None:
        _lib.set_mapping(N, mapping)
    try:
        print(f"adjoint vs multiprecision differences: {case} ({MPFD_CASES[case][2]})", flush=True)
        got = gpu_backward(ops, d, dev)
    finally:
        if mapping is not None:
            _lib.set_mapping(N, _lib.MAP_AUTO)
    v_out, g_v, g_logt, g_rho, g_rho_g, g_t = got
    errs = {"g_logt": group_rel_err(g_logt, fd["g_logt"]),
            "g_rho_d": group_rel_err(g_rho, fd["g_rho_d"]),
            "g_v": group_rel_err(g_v, fd["g_v"]),
            "g_rho_g": np.abs(g_rho_g - fd["g_rho_g"]) / np.abs(fd["g_rho_g"])}
    for k, e in errs.items():
        assert np.isfinite(e).all() and e.max() <= 1e-8, (case, k, e)
    print(case, {k: float(e.max()) for k, e in errs.items()})
    check_vs_oracle(orc, d, got, GRAD_TOL, case)


@pytest.mark.parametrize("case", sorted(FD_CASES))
def test_backward_vs_finite_differences(ops, dev, case):
    """Central differences of the GPU's own FP64 forward with h = 1e-6 in
    each parameter's natural scale: additive in log t_i and v, steps of
    h rho_g in rho_i (the scale of e_i = rho_i / rho_g; a step relative to a
    small rho_i would divide the forward's rounding noise by a tiny number)
    and relative in rho_g.  The forward's rounding noise (~1e-15) over the
    step makes these differences themselves uncertain to a few 1e-8, so the
    bar is 1e-7 of the group scale; the 1e-8 check is the multiprecision one
    above.  One case per adjoint kernel."""
    from paper_2509_25347_amd import _lib
    make, n_map, mapping = FD_CASES[case]
    if n_map is not None:
        _lib.set_mapping(n_map, mapping)
    try:
        _fd_check(ops, dev, _weights(make(), seed=3))
    finally:
        if n_map is not None:
            _lib.set_mapping(n_map, _lib.MAP_AUTO)


def _fd_check(ops, dev, d):
    T = _to(d, dev)
    _, g_v, g_logt, g_rho, g_rho_g = ops.expm_apply_backward(
        T["rho_g"], T["rho_d"], T["t_stop"], T["v"], T["w"], d["dt"])
    w = T["w"]
    h = 1e-6

    def L(rg, rd, ts, v):
        o = ops.expm_apply(rg, rd, ts, v, d["dt"])
        return (o * w).sum(dim=(0, 1))  # per cell

    N = d["rho_d"].shape[0]
    fd_lt = torch.zeros_like(g_logt)
    fd_rho = torch.zeros_like(g_rho)
    for i in range(N):
        tp, tm = T["t_stop"].clone(), T["t_stop"].clone()
        tp[i] *= np.exp(h)
        tm[i] *= np.exp(-h)
        step = torch.log(tp[i] / tm[i])
        fd_lt[i] = (L(T["rho_g"], T["rho_d"], tp, T["v"]) - L(T["rho_g"], T["rho_d"], tm, T["v"])) / step
        rp, rm = T["rho_d"].clone(), T["rho_d"].clone()
        rp[i] += h * T["rho_g"]
        rm[i] -= h * T["rho_g"]
        fd_rho[i] = (L(T["rho_g"], rp, T["t_stop"], T["v"]) - L(T["rho_g"], rm, T["t_stop"], T["v"])) / (rp[i] - rm[i])
    gp, gm = T["rho_g"] * (1 + h), T["rho_g"] * (1 - h)
    fd_rg = (L(gp, T["rho_d"], T["t_stop"], T["v"]) - L(gm, T["rho_d"], T["t_stop"], T["v"])) / (gp - gm)
    fd_v = torch.zeros_like(g_v)
    for dd in range(3):
        for j in range(N + 1):
            vp, vm = T["v"].clone(), T["v"].clone()
            vp[dd, j] += h
            vm[dd, j] -= h
            fd_v[dd, j] = (L(T["rho_g"], T["rho_d"], T["t_stop"], vp) - L(T["rho_g"], T["rho_d"], T["t_stop"], vm)) / (vp[dd, j] - vm[dd, j])
    S = sens_scale(d)
    Sr = S / d["rho_g"]
    for got, ref, fl in ((g_logt, fd_lt, S), (g_rho, fd_rho, Sr), (g_v, fd_v, None)):
        e = group_err(got.cpu().numpy(), ref.cpu().numpy(), fl)
        assert e.max() <= 1e-7, e
    e = (g_rho_g - fd_rg).abs().cpu().numpy() / np.maximum(np.abs(fd_rg.cpu().numpy()), Sr)
    assert e.max() <= 1e-7, e


def test_autograd_function(ops, dev):
    d = _weights(W.make("n4_3d", 64), seed=5)
    T = _to(d, dev)
    leaves = {k: T[k].clone().requires_grad_(True) for k in ("rho_g", "rho_d", "t_stop", "v")}
    out = ops.drag_expm(leaves["rho_g"], leaves["rho_d"], leaves["t_stop"], leaves["v"], d["dt"])
    (out * T["w"]).sum().backward()
    _, g_v, g_logt, g_rho, g_rho_g, g_t = ops.expm_apply_backward(
        T["rho_g"], T["rho_d"], T["t_stop"], T["v"], T["w"], d["dt"], want_grad_t=True)
    assert torch.equal(leaves["v"].grad, g_v)
    assert torch.equal(leaves["rho_d"].grad, g_rho)
    assert torch.equal(leaves["rho_g"].grad, g_rho_g)
    assert torch.equal(leaves["t_stop"].grad, g_t)
    # torch's own finite-difference check on a few cells
    small = {k: v[..., :3].contiguous().detach().requires_grad_(True) for k, v in leaves.items()}
    assert torch.autograd.gradcheck(
        lambda rg, rd, ts, v: ops.drag_expm(rg, rd, ts, v, d["dt"]),
        (small["rho_g"], small["rho_d"], small["t_stop"], small["v"]), eps=1e-6, atol=1e-6,
        rtol=1e-5)


def test_backward_sum_rules(ops, dev):
    """A uniform velocity has zero gradient in log t and rho (rows of exp(dt K)
    sum to one for every parameter value)."""
    d = _weights(W.make("n8_adjoint_3d", 500), seed=7)
    d["v"] = np.repeat(np.random.default_rng(1).standard_normal((3, 1, 500)), 9, axis=1)
    got = gpu_backward(ops, d, dev)
    ref = gpu_backward(ops, _weights(W.make("n8_adjoint_3d", 500), seed=7), dev)
    for k in (2, 3):
        scale = np.abs(ref[k]).max(axis=0)
        assert (np.abs(got[k]).max(axis=0) <= 1e-12 * scale).all()


@pytest.mark.parametrize("mapping", [1, 2])
def test_backward_bad_cells(ops, dev, orc, mapping):
    from paper_2509_25347_amd import _lib
    d = _weights(W.make("n4_3d", 256))
    d["rho_g"] = d["rho_g"].copy()
    d["t_stop"] = d["t_stop"].copy()
    d["w"][0, 1, 5] = np.nan
    d["rho_g"][3] = -1.0
    d["t_stop"][2, 9] = 0.0
    try:
        _lib.set_mapping(4, mapping)
        ops.clear_status()
        got = gpu_backward(ops, d, dev)
        st = ops.get_status()
    finally:
        _lib.set_mapping(4, _lib.MAP_AUTO)
    assert st == (orc.BAD_DENSITY | orc.BAD_STOPPING_TIME | orc.BAD_VELOCITY)
    for c in (3, 5, 9):
        for x in got:
            assert np.isnan(x[..., c]).all(), c
    good = [c for c in range(256) if c not in (3, 5, 9)]
    for x in got:
        assert np.isfinite(x[..., good]).all()


@pytest.mark.parametrize("N", [2, 8, 12])
def test_backward_short_quads(ops, dev, orc, N):
    """MFMA adjoints (block form for N <= 8) on 1..7 cells: quads cut short."""
    from paper_2509_25347_amd import _lib
    try:
        _lib.set_mapping(N, _lib.MAP_WAVE)
        for C in (1, 3, 5, 7):
            d = _weights(W.make_stiff(N, C), seed=C)
            got = gpu_backward(ops, d, dev)
            check_vs_oracle(orc, d, got, GRAD_TOL, f"N={N} C={C}")
    finally:
        _lib.set_mapping(N, _lib.MAP_AUTO)


def test_autograd_with_padded_inputs(ops, dev):
    """DragExpm's forward takes views with a padded leading dimension; its
    backward hands the fused adjoint contiguous copies: the gradients equal
    those of contiguous inputs bit for bit."""
    d = _weights(W.make("n4_3d", 300), seed=11)
    C, ld = 300, 320
    T = _to(d, dev)

    def padded(x):
        p = torch.full(x.shape[:-1] + (ld,), float("nan"), dtype=x.dtype, device=dev)
        p[..., :C] = x
        return p[..., :C]

    grads = []
    for make in (lambda x: x.clone(), padded):
        leaves = {k: make(T[k]).requires_grad_(True) for k in ("rho_d", "t_stop", "v")}
        rg = T["rho_g"].clone().requires_grad_(True)
        out = ops.drag_expm(rg, leaves["rho_d"], leaves["t_stop"], leaves["v"], d["dt"])
        (out * T["w"]).sum().backward()
        grads.append([rg.grad] + [leaves[k].grad for k in ("rho_d", "t_stop", "v")])
    for a, b in zip(*grads):
        assert torch.equal(a, b)

"""Seeded random cases of the forward, the backward Euler step and the
variants on the GPU against the oracle (tests marked gpu): random species
count, cell count (ragged against every launch granularity), leading
dimension, component count, time step over twelve decades, Alg. 1 cap and
option, mapping, and inputs with decoupled species (t = inf), dust-free
species (rho_d = 0) and a few bad cells mixed in.  The bars are those of the
dedicated parity tests: for the exponential, per cell 1e-13 against the exact
exponential and 1e-13 + e(oracle, exact) against the oracle
(``tests/bars.py``; the exact result of cells with decoupled or dust-free
species comes from the general long-double truth); (4N + 16) u for RK1;
gradients 1e-10 of the group's scale against the oracle's; status bits and
NaN cells exactly."""
import numpy as np
import pytest

from bars import check_forward, check_gradients

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_25347_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def random_case(rng):
    N = int(rng.integers(1, 17))
    C = int(rng.choice([1, 2, 3, 5, 15, 17, 63, 65, 255, 257, 511, 700, 1333]))
    D = int(rng.integers(1, 4))
    ld = C + int(rng.choice([0, 0, 1, 7, 64]))
    dt = float(10.0 ** rng.uniform(-6, 6))
    rho_g = rng.uniform(0.1, 10.0, C)
    eps = 10.0 ** rng.uniform(-4, 1, (N, C))
    rho_d = eps * rho_g[None]
    t_stop = 10.0 ** rng.uniform(-4, 3, (N, C))
    v = rng.standard_normal((D, N + 1, C)) * 10.0 ** rng.uniform(-2, 2)
    # structure: decoupled and dust-free species, a few bad cells
    m = rng.random((N, C))
    t_stop[m < 0.05] = np.inf
    rho_d[(m > 0.05) & (m < 0.1)] = 0.0
    if C >= 5 and rng.random() < 0.5:
        cells = rng.choice(C, size=min(3, C), replace=False)
        kinds = rng.integers(0, 4, len(cells))
        for c, k in zip(cells, kinds):
            if k == 0:
                rho_g[c] = -1.0
            elif k == 1:
                t_stop[rng.integers(N), c] = 0.0
            elif k == 2:
                v[rng.integers(D), rng.integers(N + 1), c] = np.nan
            else:
                rho_d[rng.integers(N), c] = np.inf
    return dict(N=N, C=C, D=D, ld=ld, dt=dt, rho_g=rho_g, rho_d=rho_d, t_stop=t_stop, v=v)


def to_dev(case, dev):
    C, ld = case["C"], case["ld"]

    def pad(x):
        y = np.full(x.shape[:-1] + (ld,), np.nan)
        y[..., :C] = x
        return torch.from_numpy(y).to(dev)[..., :C]

    return (torch.from_numpy(case["rho_g"]).to(dev), pad(case["rho_d"]), pad(case["t_stop"]),
            pad(case["v"]))


def cell_errors(got, ref, v_in):
    scale = np.abs(v_in).max(axis=1)
    scale = np.where((scale == 0) | ~np.isfinite(scale), 1.0, scale)
    return (np.abs(got - ref).max(axis=1) / scale).max(axis=0)


@pytest.mark.parametrize("seed", range(100))
def test_random_forward(dev, orc, seed):
    from paper_2509_25347_amd import _lib, ops
    rng = np.random.default_rng(1000 + seed)
    case = random_case(rng)
    N = case["N"]
    K = int(rng.integers(1, 10))
    opt = int(rng.integers(0, 3))
    mapping = int(rng.choice([_lib.MAP_AUTO, _lib.MAP_WAVE] + ([_lib.MAP_LANE] if N <= 12 else [])))
    rg, rd, ts, v = to_dev(case, dev)
    try:
        _lib.set_mapping(N, mapping)
        ops.clear_status()
        out = ops.expm_apply(rg, rd, ts, v, case["dt"], k_max=K, option=opt)
        status = ops.get_status()
    finally:
        _lib.set_mapping(N, _lib.MAP_AUTO)
    got = out.cpu().numpy()
    ref, kms, nrm, st = orc.apply_cells(case["rho_g"], case["rho_d"], case["t_stop"], case["v"],
                                        case["dt"], K=K, option=opt)
    label = (seed, N, case["C"], case["D"], case["dt"], K, opt, mapping)
    assert status == st, label
    assert np.array_equal(np.isnan(got), np.isnan(ref)), label
    check_forward(orc, got, ref, case, label)


@pytest.mark.parametrize("seed", range(40))
def test_random_rk1_and_variants(dev, orc, seed):
    from paper_2509_25347_amd import _lib, ops
    rng = np.random.default_rng(2000 + seed)
    case = random_case(rng)
    N = case["N"]
    rg, rd, ts, v = to_dev(case, dev)
    label = (seed, N, case["C"], case["D"], case["dt"])
    # backward Euler
    ops.clear_status()
    out = ops.rk1_apply(rg, rd, ts, v, case["dt"])
    status = ops.get_status()
    ref, st = orc.rk1_cells(case["rho_g"], case["rho_d"], case["t_stop"], case["v"], case["dt"])
    got = out.cpu().numpy()
    assert status == st, label
    assert np.array_equal(np.isnan(got), np.isnan(ref)), label
    good = ~np.isnan(ref).any(axis=(0, 1))
    if good.any():
        e = cell_errors(got[..., good], ref[..., good], case["v"][..., good])
        assert e.max() <= (4 * N + 16) * U, (label, e.max() / U)
    # the bound test and the Pade step against the oracle's own versions
    for gpu_opt, orc_opt in ((2 | _lib.OPTION_BOUND_TEST, 2 | orc.BOUND_TEST),
                             (_lib.OPTION_PADE, orc.PADE)):
        ops.clear_status()
        out = ops.expm_apply(rg, rd, ts, v, case["dt"], option=gpu_opt)
        status = ops.get_status()
        ref, kms, nrm, st = orc.apply_cells(case["rho_g"], case["rho_d"], case["t_stop"],
                                            case["v"], case["dt"], option=orc_opt)
        got = out.cpu().numpy()
        assert status == st, (label, gpu_opt)
        assert np.array_equal(np.isnan(got), np.isnan(ref)), (label, gpu_opt)
        check_forward(orc, got, ref, case, (label, gpu_opt))


@pytest.mark.parametrize("seed", range(12))
def test_random_batched_plan(dev, orc, seed):
    """Random block tables (block sizes ragged against the 64-cell lane items,
    8-cell MFMA items and 16-cell workgroups; every N; D = 1..3), K_AUTO or a
    fixed cap, a pinned or tuned configuration: every block equals the plain
    launch with the plan's cap and mapping bit for bit, and every block meets
    the parity bars against the oracle and the exact exponential."""
    from paper_2509_25347_amd import _lib, ops
    from paper_2509_25347_amd import workloads as W
    rng = np.random.default_rng(3000 + seed)
    bc = int(rng.choice([1, 3, 17, 64, 65, 200]))
    nb = int(rng.choice([1, 7, 33]))
    D = int(rng.integers(1, 4))
    k_req = int(rng.choice([_lib.K_AUTO, 9, 5]))
    batch = W.make_batched(n_blocks=nb, block_cells=bc, D=D, seed_cfg=50 + seed)
    plan = ops.BatchPlan(batch["n_species"], bc, D, batch["dt"], k_max=k_req)
    fields, v = plan.pack(batch["blocks"], dev)
    out = torch.empty_like(v)
    if rng.random() < 0.5:
        plan.autotune(fields, v, out)
    else:
        plan.set_config(int(rng.integers(4, 13)),
                        str(rng.choice(["persistent", "grid", "per_n", "per_n_pade"])))
    lmax, mode = plan.config()
    ks = plan.k_max()
    got = plan.apply(fields, v)
    torch.cuda.synchronize()
    label = (seed, bc, nb, D, k_req, plan.config())
    try:
        for N in range(1, 17):
            _lib.set_mapping(N, _lib.MAP_LANE if N <= lmax else _lib.MAP_WAVE)
        for b, blk in enumerate(batch["blocks"]):
            N = blk["rho_d"].shape[0]
            T = {k: torch.from_numpy(np.ascontiguousarray(blk[k])).to(dev)
                 for k in ("rho_g", "rho_d", "t_stop", "v")}
            pade = mode == "per_n_pade" and N > lmax
            ref = ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], batch["dt"],
                                 k_max=ks[N - 1], option=_lib.OPTION_PADE if pade else 2)
            g = plan.block_view(got, b)
            assert torch.equal(g, ref), (label, b, N)
            o, kms, nrm, st = orc.apply_cells(blk["rho_g"], blk["rho_d"], blk["t_stop"],
                                              blk["v"], batch["dt"], K=ks[N - 1],
                                              option=orc.PADE if pade else 2)
            check_forward(orc, g.cpu().numpy(), o, dict(blk, dt=batch["dt"]), (label, b))
    finally:
        for N in range(1, 17):
            _lib.set_mapping(N, _lib.MAP_AUTO)
        plan.close()


@pytest.mark.parametrize("seed", range(50))
def test_random_adjoint(dev, orc, seed):
    """Random fused forward + adjoint cases (N, C, D, dt over six decades,
    K, option, mapping) against the exact gradient and the oracle's
    reverse-mode gradient with the bars of the dedicated adjoint tests
    (tests/bars.py: 1e-10 of the group's scale or of S = sum_c ||w_c|| ||v_c||);
    the fused forward's v' meets the forward's parity bars."""
    from paper_2509_25347_amd import _lib, ops
    rng = np.random.default_rng(4000 + seed)
    N = int(rng.integers(1, 17))
    C = int(rng.choice([1, 3, 17, 63, 65, 129, 300]))
    D = int(rng.integers(1, 4))
    dt = float(10.0 ** rng.uniform(-3, 3))
    rho_g = rng.uniform(0.2, 5.0, C)
    rho_d = 10.0 ** rng.uniform(-3, 0.5, (N, C)) * rho_g[None]
    t_stop = 10.0 ** rng.uniform(-3, 2, (N, C))
    v = rng.standard_normal((D, N + 1, C))
    w = rng.standard_normal((D, N + 1, C))
    K = int(rng.integers(5, 10))
    opt = int(rng.integers(0, 3))
    mapping = int(rng.choice([_lib.MAP_AUTO, _lib.MAP_WAVE] + ([_lib.MAP_LANE] if N <= 12 else [])))
    T = {k: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
         for k, x in (("rho_g", rho_g), ("rho_d", rho_d), ("t_stop", t_stop), ("v", v), ("w", w))}
    try:
        _lib.set_mapping(N, mapping)
        res = ops.expm_apply_backward(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], T["w"], dt,
                                      k_max=K, option=opt)
        torch.cuda.synchronize()
    finally:
        _lib.set_mapping(N, _lib.MAP_AUTO)
    v_out, g_v, g_logt, g_rho, g_rho_g = (x.cpu().numpy() for x in res)
    rv, rgv, rlt, rrho, rrg, st = orc.grad_cells(rho_g, rho_d, t_stop, v, w, dt, K=K, option=opt)
    assert st == 0
    label = (seed, N, C, D, dt, K, opt, mapping)
    d = dict(rho_g=rho_g, rho_d=rho_d, t_stop=t_stop, v=v, w=w, dt=dt)
    check_forward(orc, v_out, rv, d, label)
    check_gradients(orc, d, (g_v, g_logt, g_rho, g_rho_g), label,
                    oracle_grads=(rgv, rlt, rrho, rrg))

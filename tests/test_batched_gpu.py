"""GPU tests of the batched uneven-N launch (one hipGraph over AMR blocks).

Each block's result must be bit-identical to the plain per-N launch on that
block with the same mapping (the batched items run the same per-cell code),
and within the parity bars of ``tests/bars.py`` (the uneven-N blocks follow
the stiff recipe, where the oracle sits at the FP64 floor: 1e-13 against it
outright, and 1e-13 against the exact exponential).  Graph replays are
checked against the eager result with other GPU work between replays.
"""
import numpy as np
import pytest

from paper_2509_25347_amd import workloads as W
from bars import check_forward

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


def plain_per_block(ops, batch, dev, lane_max, k_max=None, pade=False):
    """drag_expm_apply on every block with the batched plan's mapping (and
    Taylor cap k_max[N - 1] when given, else K = 9; with ``pade`` the blocks
    above lane_max take the Pade option, as the plan's per_n_pade form)."""
    from paper_2509_25347_amd import _lib
    outs = []
    try:
        for N in range(1, 17):
            _lib.set_mapping(N, _lib.MAP_LANE if N <= lane_max else _lib.MAP_WAVE)
        for blk in batch["blocks"]:
            T = {k: torch.from_numpy(np.ascontiguousarray(blk[k])).to(dev)
                 for k in ("rho_g", "rho_d", "t_stop", "v")}
            N = blk["rho_d"].shape[0]
            K = 9 if k_max is None else k_max[N - 1]
            opt = _lib.OPTION_PADE if pade and N > lane_max else 2
            outs.append(ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"],
                                       batch["dt"], k_max=K, option=opt).cpu().numpy())
    finally:
        for N in range(1, 17):
            _lib.set_mapping(N, _lib.MAP_AUTO)
    return outs


def test_batched_matches_plain_and_oracle(ops, dev, orc):
    batch = W.make_batched(n_blocks=48, block_cells=100, seed_cfg=41)
    plan = ops.BatchPlan(batch["n_species"], 100, 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    out = plan.apply(fields, v)
    torch.cuda.synchronize()
    ref = plain_per_block(ops, batch, dev, lane_max=6)
    for b, blk in enumerate(batch["blocks"]):
        got = plan.block_view(out, b).cpu().numpy()
        assert np.array_equal(got, ref[b]), b
        o, kms, nrm, st = orc.apply_cells(blk["rho_g"], blk["rho_d"], blk["t_stop"], blk["v"],
                                          batch["dt"])
        check_forward(orc, got, o, dict(blk, dt=batch["dt"]), ("block", b), tight=True)
    plan.close()


def test_autotune_and_every_variant_result(ops, dev):
    """The tuned configuration and every pinned one (lane bound 4..12 x the
    four MFMA forms) give the plain per-block result bit for bit: the Taylor
    forms drag_expm_apply's default, the Pade per-N grids its Pade option."""
    batch = W.make_batched(n_blocks=64, block_cells=70, seed_cfg=43)
    plan = ops.BatchPlan(batch["n_species"], 70, 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    out = torch.empty_like(v)
    lm = plan.autotune(fields, v, out)
    assert 4 <= lm <= 12
    mode_t = plan.config()[1]
    assert mode_t in ("persistent", "grid", "per_n", "per_n_pade")
    out2 = plan.apply(fields, v)
    torch.cuda.synchronize()
    tuned_ref = plain_per_block(ops, batch, dev, lane_max=lm, pade=mode_t == "per_n_pade")
    for b in range(len(batch["blocks"])):
        assert np.array_equal(plan.block_view(out2, b).cpu().numpy(), tuned_ref[b]), b
    for lmax in range(4, 13):
        ref_t = plain_per_block(ops, batch, dev, lane_max=lmax)
        ref_p = plain_per_block(ops, batch, dev, lane_max=lmax, pade=True)
        for mode in ("persistent", "grid", "per_n", "per_n_pade"):
            plan.set_config(lmax, mode)
            assert plan.config() == (lmax, mode)
            o = plan.apply(fields, v)
            torch.cuda.synchronize()
            ref = ref_p if mode == "per_n_pade" else ref_t
            for b in range(len(batch["blocks"])):
                assert np.array_equal(plan.block_view(o, b).cpu().numpy(), ref[b]), (lmax, mode, b)
    plan.close()


def test_dt_zero_returns_the_input(ops, dev):
    """dt = 0 through every form of the batched update (each lane bound's grids
    and the four MFMA forms, and the entry point without allocation): exp(0) = I,
    so every block comes back with its input values."""
    batch = W.make_batched(n_blocks=48, block_cells=64, seed_cfg=47)
    plan = ops.BatchPlan(batch["n_species"], 64, 3, 0.0)
    fields, v = plan.pack(batch["blocks"], dev)
    for lmax in (4, 8, 12):
        for mode in ("persistent", "grid", "per_n", "per_n_pade"):
            plan.set_config(lmax, mode)
            out = plan.apply(fields, v)
            torch.cuda.synchronize()
            assert torch.equal(out, v), (lmax, mode)
    plan.close()
    out = ops.expm_apply_batched_static(batch["n_species"], 64, 3, 0.0, fields, v)
    torch.cuda.synchronize()
    assert torch.equal(out, v)


def test_pade_per_n_form_against_the_oracle(ops, dev, orc):
    """The per_n_pade form: blocks above the lane bound against the oracle's
    Pade step (its dense (N+1) form) and the exact exponential, to the
    parity bars; blocks at or below it are the lane kernels' Taylor result."""
    batch = W.make_batched(n_blocks=40, block_cells=96, seed_cfg=48)
    plan = ops.BatchPlan(batch["n_species"], 96, 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    plan.set_config(8, "per_n_pade")
    out = plan.apply(fields, v)
    torch.cuda.synchronize()
    for b, blk in enumerate(batch["blocks"]):
        got = plan.block_view(out, b).cpu().numpy()
        pade = blk["rho_d"].shape[0] > 8
        o, kms, nrm, st = orc.apply_cells(blk["rho_g"], blk["rho_d"], blk["t_stop"], blk["v"],
                                          batch["dt"], option=orc.PADE if pade else 2)
        check_forward(orc, got, o, dict(blk, dt=batch["dt"]), ("block", b, "pade", pade))
    plan.close()


def test_auto_taylor_cap_plan(ops, dev, orc):
    """A K_AUTO plan starts from the library's per-N caps, the autotuner picks
    a cap per N in 3..9, and every block is then bit-identical to the plain
    launch with that cap (and within the oracle's bar for it); v_out of the
    autotune call already holds that result."""
    from paper_2509_25347_amd import _lib
    batch = W.make_batched(n_blocks=64, block_cells=96, seed_cfg=47)
    plan = ops.BatchPlan(batch["n_species"], 96, 3, batch["dt"], k_max=_lib.K_AUTO)
    assert plan.k_max() == [_lib.get_k_max(N) for N in range(1, 17)]
    fields, v = plan.pack(batch["blocks"], dev)
    out = torch.empty_like(v)
    lm = plan.autotune(fields, v, out)
    torch.cuda.synchronize()
    ks = plan.k_max()
    assert all(3 <= k <= 9 for k in ks)
    out2 = plan.apply(fields, v)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    ref = plain_per_block(ops, batch, dev, lane_max=lm, k_max=ks)
    for b, blk in enumerate(batch["blocks"]):
        got = plan.block_view(out2, b).cpu().numpy()
        assert np.array_equal(got, ref[b]), b
        K = ks[blk["rho_d"].shape[0] - 1]
        o, kms, nrm, st = orc.apply_cells(blk["rho_g"], blk["rho_d"], blk["t_stop"], blk["v"],
                                          batch["dt"], K=K)
        check_forward(orc, got, o, dict(blk, dt=batch["dt"]), ("block", b, "K", K))
    plan.close()


def test_graph_replays_and_recapture(ops, dev):
    batch = W.make_batched(n_blocks=40, block_cells=128, seed_cfg=45)
    plan = ops.BatchPlan(batch["n_species"], 128, 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    out = torch.empty_like(v)
    first = plan.apply(fields, v, out).clone()
    # other work on the same GPU between replays, then replay and compare
    junk = torch.randn(1 << 20, dtype=torch.float64, device=dev)
    d = W.make("n16_stiff_3d", 512)
    T = {k: torch.from_numpy(d[k]).to(dev) for k in ("rho_g", "rho_d", "t_stop", "v")}
    for rep in range(4):
        junk = junk * 1.0001 + 1.0
        ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], 1.0)
        out.fill_(np.nan)
        plan.apply(fields, v, out)
        torch.cuda.synchronize()
        assert torch.equal(out, first), rep
    # new pointers: the plan re-captures
    v2 = v.clone()
    out2 = plan.apply(fields, v2)
    assert torch.equal(out2, first)
    # in place
    plan.apply(fields, v2, v2)
    assert torch.equal(v2, first)
    plan.close()


def test_batched_bad_cells_and_errors(ops, dev, orc):
    from paper_2509_25347_amd import _lib
    batch = W.make_batched(n_blocks=8, block_cells=64, seed_cfg=47)
    batch["blocks"][2]["rho_g"] = batch["blocks"][2]["rho_g"].copy()
    batch["blocks"][2]["rho_g"][5] = -1.0
    plan = ops.BatchPlan(batch["n_species"], 64, 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    ops.clear_status()
    out = plan.apply(fields, v)
    assert ops.get_status() == orc.BAD_DENSITY
    assert torch.isnan(plan.block_view(out, 2)[..., 5]).all()
    assert torch.isfinite(plan.block_view(out, 2)[..., :5]).all()
    # an output that overlaps the fields buffer is rejected by the library
    big = torch.empty(plan.fields_total + plan.v_total, dtype=torch.float64, device=dev)
    big[: plan.fields_total] = fields
    f2 = big[: plan.fields_total]
    with pytest.raises(_lib.DragError):
        plan.apply(f2, v, big[plan.fields_total - 8: plan.fields_total - 8 + plan.v_total])
    with pytest.raises(_lib.DragError):
        ops.BatchPlan([3, 17], 64, 3, 1.0)
    plan.close()


def test_full_size_batched_sampled(ops, dev, orc):
    """4096 blocks of 8^3 cells, N_b ~ U{1..16}: 24 sampled blocks against the
    oracle and the exact exponential on every cell, every sampled block's
    momentum conserved, and every output finite and within the inputs'
    range (a convex combination)."""
    batch = W.make_batched()
    plan = ops.BatchPlan(batch["n_species"], batch["block_cells"], 3, batch["dt"])
    fields, v = plan.pack(batch["blocks"], dev)
    out = plan.apply(fields, v)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    rng = np.random.default_rng(0)
    for b in rng.choice(len(batch["blocks"]), 24, replace=False):
        blk = batch["blocks"][b]
        got = plan.block_view(out, b).cpu().numpy()
        o, kms, nrm, st = orc.apply_cells(blk["rho_g"], blk["rho_d"], blk["t_stop"], blk["v"],
                                          batch["dt"])
        assert st == 0
        check_forward(orc, got, o, dict(blk, dt=batch["dt"]), ("block", int(b)), tight=True)
        vmax = np.abs(blk["v"]).max(axis=1)
        assert (np.abs(got).max(axis=1) <= vmax * (1 + 1e-12)).all(), b
    plan.close()

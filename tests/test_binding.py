"""Host-side checks of the Python binding: outputs it allocates share the
caller's leading dimension, since the library addresses every [.][ld] array
with the one ld of the descriptor; and (on a GPU) tensors off the current
device are refused."""
import pytest

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("C,pad", [(63, 0), (63, 1), (1000, 24), (5, 64)])
def test_out_like_keeps_the_leading_dimension(C, pad):
    from paper_2509_25347_amd import ops
    ld = C + pad
    full = torch.zeros((3, 5, ld), dtype=torch.float64)
    v = full[..., :C]
    out = ops._out_like(v, C, ld)
    assert out.shape == v.shape and out.stride() == v.stride()
    # the last element the library writes, (rows - 1) * ld + C - 1, lies in the storage
    rows = 3 * 5
    assert out.untyped_storage().nbytes() >= 8 * ((rows - 1) * ld + C)
    assert ops._ld_of(out, 2, "out") == ld


def test_layout_helpers_reject_uneven_rows():
    from paper_2509_25347_amd import ops
    x = torch.zeros((3, 5, 40), dtype=torch.float64)[:, :, ::2]
    with pytest.raises(ValueError):
        ops._ld_of(x, 2, "x")
    y = torch.zeros((3, 6, 40), dtype=torch.float64)[:, :5, :]  # rows spaced 40, blocks 240
    with pytest.raises(ValueError):
        ops._ld_of(y, 2, "y")


def test_a_single_row_imposes_no_leading_dimension():
    """rho_d and t_stop at N = 1 are one row: a view of a wider array (row
    stride != C) must not clash with v's leading dimension."""
    from paper_2509_25347_amd import ops
    wide = torch.zeros((1, 1000), dtype=torch.float64)[:, :300]
    assert wide.stride(0) == 1000
    assert ops._ld_of(wide, 1, "rho_d") is None
    v = torch.zeros((3, 2, 300), dtype=torch.float64)
    assert ops._ld_of(v, 2, "v") == 300


def test_shapes_share_one_leading_dimension(monkeypatch):
    """_shapes on host tensors (the device check switched off): a padded v
    sets ld even at N = 1, D = 1; mismatched row strides are refused."""
    from paper_2509_25347_amd import ops
    monkeypatch.setattr(ops, "_require", lambda t, name, dev=None: None)
    monkeypatch.setattr(ops, "_current_device", lambda: 0)
    C, ld = 100, 128
    rho_g = torch.zeros(C, dtype=torch.float64)
    rho_d = torch.zeros((1, 1000), dtype=torch.float64)[:, :C]  # one row: no constraint
    t_stop = torch.zeros((1, C), dtype=torch.float64)
    v = torch.zeros((1, 2, ld), dtype=torch.float64)[..., :C]
    assert ops._shapes(rho_g, rho_d, t_stop, v) == (C, 1, 1, ld)
    rho_d4 = torch.zeros((4, ld), dtype=torch.float64)[:, :C]
    t4 = torch.zeros((4, C), dtype=torch.float64)  # ld C against ld 128
    v4 = torch.zeros((3, 5, ld), dtype=torch.float64)[..., :C]
    with pytest.raises(ValueError):
        ops._shapes(rho_g, rho_d4, t4, v4)
    t4p = torch.zeros((4, ld), dtype=torch.float64)[:, :C]
    assert ops._shapes(rho_g, rho_d4, t4p, v4) == (C, 4, 3, ld)


def test_overlapping_rows_are_refused(monkeypatch):
    """An expand()ed view (row stride 0) or rows closer than the cell count
    share storage; the library would read D (N+1) ld doubles from it."""
    from paper_2509_25347_amd import ops
    monkeypatch.setattr(ops, "_require", lambda t, name, dev=None: None)
    monkeypatch.setattr(ops, "_current_device", lambda: 0)
    v = torch.zeros(100, dtype=torch.float64).view(1, 1, 100).expand(3, 2, 100)
    with pytest.raises(ValueError):
        ops._ld_of(v, 2, "v")
    base = torch.zeros(1000, dtype=torch.float64)
    close = base.as_strided((3, 2, 100), (100, 50, 1))  # rows 50 apart, 100 cells each
    with pytest.raises(ValueError):
        ops._ld_of(close, 2, "v")
    rho_d = base.as_strided((4, 100), (60, 1))
    with pytest.raises(ValueError):
        ops._ld_of(rho_d, 1, "rho_d")
    rho_g = torch.zeros(100, dtype=torch.float64)
    t = torch.zeros((1, 100), dtype=torch.float64)
    rd = torch.zeros((1, 100), dtype=torch.float64)
    with pytest.raises(ValueError):
        ops._shapes(rho_g, rd, t, v)


def test_autograd_backward_hands_contiguous_inputs(monkeypatch):
    """The forward accepts padded views; the fused adjoint takes contiguous
    arrays, so DragExpm.backward passes contiguous copies."""
    from paper_2509_25347_amd import ops
    C, ld, N, D = 50, 64, 3, 2
    saved = (torch.zeros(C, dtype=torch.float64),
             torch.zeros((N, ld), dtype=torch.float64)[:, :C],
             torch.ones((N, ld), dtype=torch.float64)[:, :C],
             torch.zeros((D, N + 1, ld), dtype=torch.float64)[..., :C])
    seen = {}

    def fake_backward(rho_g, rho_d, t_stop, v, grad_out, dt, k_max, option, **kw):
        seen["contiguous"] = all(x.is_contiguous() for x in (rho_g, rho_d, t_stop, v, grad_out))
        z = torch.zeros_like
        return None, z(v), z(rho_d), z(rho_d), z(rho_g), z(t_stop)

    monkeypatch.setattr(ops, "expm_apply_backward", fake_backward)

    class Ctx:
        saved_tensors = saved
        dt, k_max, option = 1.0, 9, 2
        needs_input_grad = (True, True, True, True, False, False, False)

    grads = ops.DragExpm.backward(Ctx(), torch.zeros((D, N + 1, ld), dtype=torch.float64)[..., :C])
    assert seen["contiguous"]
    assert grads[3].shape == (D, N + 1, C)


@pytest.mark.gpu
def test_tensors_off_the_current_device_are_refused(monkeypatch):
    """The library launches on the current device with raw pointers: a tensor
    of another device is refused before anything is enqueued (simulated on
    one GPU by moving the current device)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_25347_amd import ops, workloads
    d = workloads.make("n4_3d", 64)
    T = {k: torch.from_numpy(d[k]).cuda() for k in ("rho_g", "rho_d", "t_stop", "v")}
    ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    monkeypatch.setattr(ops, "_current_device", lambda: T["v"].get_device() + 1)
    with pytest.raises(ValueError, match="current device"):
        ops.expm_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])
    with pytest.raises(ValueError, match="current device"):
        ops.rk1_apply(T["rho_g"], T["rho_d"], T["t_stop"], T["v"], d["dt"])

"""PyTorch-facing entry points of the drag update (argument marshalling only).

Tensors must be float64 CUDA (HIP) tensors on one device; every array is
passed as a raw device pointer with its leading dimension, and the work is
enqueued on the current stream.  Layouts (cell index fastest):
    rho_g [C], rho_d [N][C], t_stop [N][C], v [D][N+1][C]
Views whose last stride is 1 and whose row stride is a common ``ld >= C``
are accepted as they are.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib


# torch's raw accessor of the current stream: torch.cuda.current_stream()
# builds a Python stream object per call (about 3 us, as long as a small
# launch), the accessor returns the handle itself.
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_ptr(stream=None):
    """`stream`, else torch's current stream on the current device."""
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    if _raw_stream is not None:
        return ctypes.c_void_p(_raw_stream(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


_current_device = getattr(torch._C, "_cuda_getDevice", None) or torch.cuda.current_device


def _require(t, name, dev=None):
    """A float64 tensor on the current GPU (the library launches on the
    current device and takes raw pointers: memory of another device would be
    read across the fabric, or fault)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype is not torch.float64:
        raise TypeError(f"{name} must be float64 (got {t.dtype}); there is no implicit cast")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    cur = _current_device() if dev is None else dev
    if t.get_device() != cur:
        raise ValueError(f"{name} is on cuda:{t.get_device()} but the current device is "
                         f"cuda:{cur} (use torch.cuda.device(...))")


def _ld_of(t, rows_dims, name):
    """Leading dimension of an SoA array whose last axis is the cell axis:
    the common spacing of its rows, which must be at least the row length
    (expand()ed or overlapping views, whose rows share storage, are refused:
    the library would read past their storage)."""
    st, sh = t.stride(), t.shape
    if st[-1] != 1:
        raise ValueError(f"{name}: the cell axis must be contiguous")
    ld, exp = None, 1
    for ax in range(len(sh) - 2, -1, -1):
        if sh[ax] > 1:
            if ld is None:
                if st[ax] % exp:
                    raise ValueError(f"{name}: rows must be equally spaced (stride ld)")
                ld = st[ax] // exp
            elif st[ax] != ld * exp:
                raise ValueError(f"{name}: rows must be equally spaced (stride ld)")
        exp *= sh[ax]
    if ld is None:
        return None  # one row (rho_g; rho_d at N = 1): its row stride is never used
    if ld < sh[-1]:
        raise ValueError(f"{name}: rows overlap (row stride {ld} below the {sh[-1]} cells)")
    return ld


def _shapes(rho_g, rho_d, t_stop, v):
    dev = _current_device()
    for x, n in ((rho_g, "rho_g"), (rho_d, "rho_d"), (t_stop, "t_stop"), (v, "v")):
        _require(x, n, dev)
    sg, sd, st, sv = rho_g.shape, rho_d.shape, t_stop.shape, v.shape
    if len(sg) != 1 or len(sd) != 2 or len(st) != 2 or len(sv) != 3:
        raise ValueError("expected rho_g [C], rho_d [N][C], t_stop [N][C], v [D][N+1][C]")
    C, N, D = sg[0], sd[0], sv[0]
    if sd != (N, C) or st != (N, C) or sv != (D, N + 1, C):
        raise ValueError("inconsistent shapes")
    if rho_g.stride(0) != 1:
        raise ValueError("rho_g must be contiguous")
    lds = {x for x in (_ld_of(rho_d, 1, "rho_d"), _ld_of(t_stop, 1, "t_stop"),
                       _ld_of(v, 2, "v")) if x is not None}
    if len(lds) > 1:
        raise ValueError("rho_d, t_stop and v must share one leading dimension")
    ld = lds.pop() if lds else C
    return C, N, D, max(ld, C) if C else max(ld, 1)


def _out_like(v, C, ld):
    """An output with v's shape and the shared leading dimension ld (the
    library addresses every [.][ld] array with the one ld of the descriptor)."""
    if ld == C:
        return torch.empty(tuple(v.shape), dtype=v.dtype, device=v.device)
    full = torch.empty(tuple(v.shape[:-1]) + (ld,), dtype=v.dtype, device=v.device)
    return full[..., :C]


def expm_apply(rho_g, rho_d, t_stop, v, dt, k_max=9, option=2, out=None, stream=None):
    """v' = exp(dt K) v for every cell (drag_expm_apply).  ``out`` may be
    ``v`` itself (in place)."""
    C, N, D, ld = _shapes(rho_g, rho_d, t_stop, v)
    if out is None:
        out = _out_like(v, C, ld)
    else:
        _require(out, "out")
        if out.shape != v.shape or _ld_of(out, 2, "out") not in (None, ld) and C:
            raise ValueError("out must have the shape and layout of v")
    desc = _lib.make_desc(C, N, D, ld, dt, k_max, option)
    _lib.check(_lib.lib().drag_expm_apply(ctypes.byref(desc), _ptr(rho_g), _ptr(rho_d),
                                          _ptr(t_stop), _ptr(v), _ptr(out),
                                          _stream_ptr(stream)), "drag_expm_apply")
    return out


def rk1_apply(rho_g, rho_d, t_stop, v, dt, out=None, stream=None):
    """v' = (I - dt K)^-1 v for every cell, the first-order implicit drag step
    by its O(N) closed form (drag_rk1_apply).  ``out`` may be ``v`` itself."""
    C, N, D, ld = _shapes(rho_g, rho_d, t_stop, v)
    if out is None:
        out = _out_like(v, C, ld)
    else:
        _require(out, "out")
        if out.shape != v.shape or _ld_of(out, 2, "out") not in (None, ld) and C:
            raise ValueError("out must have the shape and layout of v")
    desc = _lib.make_desc(C, N, D, ld, dt)
    _lib.check(_lib.lib().drag_rk1_apply(ctypes.byref(desc), _ptr(rho_g), _ptr(rho_d),
                                         _ptr(t_stop), _ptr(v), _ptr(out),
                                         _stream_ptr(stream)), "drag_rk1_apply")
    return out


def expm_steps(rho_g, rho_d, t_stop, v, dt, n_steps, history=False, k_max=9, option=2,
               stream=None):
    """n_steps drag steps of size dt (drag_expm_steps).  Returns v after the
    last step, and with ``history`` also the [n_steps, D, N+1, C] states
    after every step."""
    C, N, D, ld = _shapes(rho_g, rho_d, t_stop, v)
    if ld != C or not v.is_contiguous():
        raise ValueError("expm_steps takes a contiguous v")
    out = torch.empty_like(v)
    hist = (torch.empty((int(n_steps),) + tuple(v.shape), dtype=torch.float64, device=v.device)
            if history else None)
    desc = _lib.make_desc(C, N, D, ld, dt, k_max, option)
    _lib.check(_lib.lib().drag_expm_steps(ctypes.byref(desc), _ptr(rho_g), _ptr(rho_d),
                                          _ptr(t_stop), _ptr(v), _ptr(out), int(n_steps),
                                          _ptr(hist) if hist is not None and n_steps else None,
                                          _stream_ptr(stream)), "drag_expm_steps")
    return (out, hist) if history else out


def build(rho_g, rho_d, t_stop, dt, k_max=9, option=2, stream=None):
    """Per-cell a = dt/t, e = rho_i/rho_g, ||dt K||_1 and (k*, m*, s*)."""
    for x, n in ((rho_g, "rho_g"), (rho_d, "rho_d"), (t_stop, "t_stop")):
        _require(x, n)
    C = rho_g.size(0)
    N = rho_d.size(0)
    ld = _ld_of(rho_d, 1, "rho_d") or C
    dev = rho_g.device
    a = torch.empty((N, C), dtype=torch.float64, device=dev)
    e = torch.empty((N, C), dtype=torch.float64, device=dev)
    nrm = torch.empty(C, dtype=torch.float64, device=dev)
    k = torch.empty(C, dtype=torch.int32, device=dev)
    m = torch.empty(C, dtype=torch.int32, device=dev)
    s = torch.empty(C, dtype=torch.int32, device=dev)
    if ld != C:
        raise ValueError("build() takes contiguous [N][C] inputs")
    desc = _lib.make_desc(C, N, 1, C, dt, k_max, option)
    _lib.check(_lib.lib().drag_build(ctypes.byref(desc), _ptr(rho_g), _ptr(rho_d),
                                     _ptr(t_stop), _ptr(a), _ptr(e), _ptr(nrm), _ptr(k),
                                     _ptr(m), _ptr(s), _stream_ptr(stream)), "drag_build")
    return a, e, nrm, k, m, s


def expm_apply_backward(rho_g, rho_d, t_stop, v, grad_out, dt, k_max=9, option=2,
                        want_v_out=True, want_grad_rho_g=True, want_grad_t=False,
                        stream=None):
    """Fused forward + adjoint (drag_expm_apply_backward).

    Returns (v_out or None, grad_v, grad_log_t, grad_rho_d, grad_rho_g or None),
    plus grad_t_stop as a sixth item when ``want_grad_t``.
    """
    C, N, D, ld = _shapes(rho_g, rho_d, t_stop, v)
    _require(grad_out, "grad_out")
    if grad_out.shape != v.shape:
        raise ValueError("grad_out must have the shape of v")
    if ld != C or not (v.is_contiguous() and grad_out.is_contiguous()):
        raise ValueError("expm_apply_backward takes contiguous inputs")
    dev = v.device
    v_out = torch.empty_like(v) if want_v_out else None
    g_v = torch.empty_like(v)
    g_logt = torch.empty((N, C), dtype=torch.float64, device=dev)
    g_rho = torch.empty((N, C), dtype=torch.float64, device=dev)
    g_rho_g = torch.empty(C, dtype=torch.float64, device=dev) if want_grad_rho_g else None
    g_t = torch.empty((N, C), dtype=torch.float64, device=dev) if want_grad_t else None
    desc = _lib.make_desc(C, N, D, C, dt, k_max, option)
    _lib.check(_lib.lib().drag_expm_apply_backward(
        ctypes.byref(desc), _ptr(rho_g), _ptr(rho_d), _ptr(t_stop), _ptr(v), _ptr(grad_out),
        _ptr(v_out), _ptr(g_v), _ptr(g_logt), _ptr(g_t), _ptr(g_rho), _ptr(g_rho_g),
        _stream_ptr(stream)), "drag_expm_apply_backward")
    if want_grad_t:
        return v_out, g_v, g_logt, g_rho, g_rho_g, g_t
    return v_out, g_v, g_logt, g_rho, g_rho_g


def get_status(stream=None) -> int:
    st = ctypes.c_int32()
    _lib.check(_lib.lib().drag_get_status(_stream_ptr(stream), ctypes.byref(st)),
               "drag_get_status")
    return st.value


def clear_status(stream=None) -> None:
    _lib.check(_lib.lib().drag_clear_status(_stream_ptr(stream)), "drag_clear_status")


class DragExpm(torch.autograd.Function):
    """v' = exp(dt K(t_stop, rho_d, rho_g)) v with the hand-written adjoint.

    Only the inputs are saved; the backward recomputes the Taylor stage and
    the squarings (drag_expm_apply_backward).  Gradients flow to t_stop
    (through log t), rho_d, rho_g and v; dt, k_max and option get None.
    """

    @staticmethod
    def forward(ctx, rho_g, rho_d, t_stop, v, dt, k_max, option):
        ctx.save_for_backward(rho_g, rho_d, t_stop, v)
        ctx.dt, ctx.k_max, ctx.option = dt, k_max, option
        return expm_apply(rho_g, rho_d, t_stop, v, dt, k_max, option)

    @staticmethod
    def backward(ctx, grad_out):
        # the fused adjoint takes contiguous arrays; the forward also accepts
        # views with a padded leading dimension
        rho_g, rho_d, t_stop, v = (x.contiguous() for x in ctx.saved_tensors)
        _, g_v, g_logt, g_rho, g_rho_g, g_t = expm_apply_backward(
            rho_g, rho_d, t_stop, v, grad_out.contiguous(), ctx.dt, ctx.k_max, ctx.option,
            want_v_out=False, want_grad_t=True)
        return (g_rho_g if ctx.needs_input_grad[0] else None,
                g_rho if ctx.needs_input_grad[1] else None,
                g_t if ctx.needs_input_grad[2] else None,
                g_v if ctx.needs_input_grad[3] else None,
                None, None, None)


def drag_expm(rho_g, rho_d, t_stop, v, dt, k_max=9, option=2):
    """Differentiable v' = exp(dt K) v (see DragExpm)."""
    return DragExpm.apply(rho_g, rho_d, t_stop, v, dt, k_max, option)


def expm_apply_batched_static(n_species, block_cells, n_dim, dt, fields, v_in, v_out=None,
                              k_max=9, option=2, stream=None):
    """The batched update without a plan and without allocation in the
    library (drag_expm_apply_batched_static): the block tables go to a static
    device buffer of the library.  Buffers laid out as BatchPlan's for the
    same blocks; ``v_out`` may be ``v_in``.  (Allocating ``v_out`` here when
    it is None is the binding's convenience, not the library's.)"""
    for x, nm in ((fields, "fields"), (v_in, "v_in")):
        _require(x, nm)
    if v_out is None:
        v_out = torch.empty_like(v_in)
    _require(v_out, "v_out")
    ns = [int(x) for x in n_species]
    arr = (ctypes.c_int32 * len(ns))(*ns)
    desc = _lib.DragBatchDesc(len(ns), int(block_cells), int(n_dim), int(k_max), int(option),
                              float(dt), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)))
    bc, D = int(block_cells), int(n_dim)
    f_need = sum(bc * (1 + 2 * n) for n in ns)
    v_need = sum(bc * D * (n + 1) for n in ns)
    if fields.numel() < f_need or v_in.numel() < v_need or v_out.numel() < v_need:
        raise ValueError("buffers smaller than the batch's layout")
    _lib.check(_lib.lib().drag_expm_apply_batched_static(ctypes.byref(desc), _ptr(fields),
                                                         _ptr(v_in), _ptr(v_out),
                                                         _stream_ptr(stream)),
               "drag_expm_apply_batched_static")
    return v_out


class BatchPlan:
    """AMR-style blocks with uneven species counts in one graph launch
    (drag_plan_batched / drag_expm_apply_batched).

    Block b's fields live in one flat float64 buffer at ``field_offset[b]``:
    rho_g [bc] | rho_d [N_b][bc] | t_stop [N_b][bc]; its velocities in a
    second buffer at ``v_offset[b]``: v [D][N_b+1][bc].  ``pack`` lays out
    host arrays that way (input preparation, outside the hot path).
    """

    def __init__(self, n_species, block_cells, n_dim, dt, k_max=9, option=2):
        import numpy as np
        L = _lib.lib()
        self.n_species = [int(x) for x in n_species]
        self.block_cells = int(block_cells)
        self.n_dim = int(n_dim)
        self.dt = float(dt)
        nb = len(self.n_species)
        self._arr = (ctypes.c_int32 * nb)(*self.n_species)
        desc = _lib.DragBatchDesc(nb, self.block_cells, self.n_dim, int(k_max), int(option),
                                  self.dt, ctypes.cast(self._arr, ctypes.POINTER(ctypes.c_int32)))
        plan = ctypes.c_void_p()
        _lib.check(L.drag_plan_batched(ctypes.byref(desc), ctypes.byref(plan)),
                   "drag_plan_batched")
        self._plan = plan
        self.field_offset = np.zeros(nb, dtype=np.int64)
        self.v_offset = np.zeros(nb, dtype=np.int64)
        ft, vt = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(L.drag_plan_offsets(plan, self.field_offset.ctypes.data_as(ctypes.c_void_p),
                                       self.v_offset.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(ft), ctypes.byref(vt)), "drag_plan_offsets")
        self.fields_total, self.v_total = ft.value, vt.value

    def pack(self, blocks, device):
        """Flat (fields, v) GPU buffers from per-block dicts of numpy arrays."""
        import numpy as np
        bc = self.block_cells
        f = np.empty(self.fields_total)
        v = np.empty(self.v_total)
        for b, blk in enumerate(blocks):
            n = self.n_species[b]
            o = self.field_offset[b]
            f[o:o + bc] = blk["rho_g"]
            f[o + bc:o + bc + n * bc] = blk["rho_d"].ravel()
            f[o + bc + n * bc:o + bc + 2 * n * bc] = blk["t_stop"].ravel()
            ov = self.v_offset[b]
            v[ov:ov + self.n_dim * (n + 1) * bc] = blk["v"].ravel()
        return (torch.from_numpy(f).to(device), torch.from_numpy(v).to(device))

    def block_view(self, v, b):
        """The [D][N_b+1][bc] view of block b inside a flat velocity buffer."""
        n = self.n_species[b]
        o = int(self.v_offset[b])
        return v[o:o + self.n_dim * (n + 1) * self.block_cells].view(
            self.n_dim, n + 1, self.block_cells)

    def apply(self, fields, v_in, v_out=None, stream=None):
        for x, nm in ((fields, "fields"), (v_in, "v_in")):
            _require(x, nm)
        if v_out is None:
            v_out = torch.empty_like(v_in)
        _require(v_out, "v_out")
        if fields.numel() < self.fields_total or v_in.numel() < self.v_total or \
                v_out.numel() < self.v_total:
            raise ValueError("buffers smaller than the plan's layout")
        _lib.check(_lib.lib().drag_expm_apply_batched(self._plan, _ptr(fields), _ptr(v_in),
                                                      _ptr(v_out), _stream_ptr(stream)),
                   "drag_expm_apply_batched")
        return v_out

    def autotune(self, fields, v_in, v_out, stream=None) -> int:
        lm = ctypes.c_int32()
        _lib.check(_lib.lib().drag_plan_autotune(self._plan, _ptr(fields), _ptr(v_in),
                                                 _ptr(v_out), _stream_ptr(stream),
                                                 ctypes.byref(lm)), "drag_plan_autotune")
        return lm.value

    MFMA_MODES = {0: "persistent", 1: "grid", 2: "per_n", 3: "per_n_pade"}

    def config(self):
        """(lane_max, mfma_mode) of the current launch configuration; the mode
        is "persistent", "grid" or "per_n" (drag_plan_config)."""
        lm, mm = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.lib().drag_plan_config(self._plan, ctypes.byref(lm), ctypes.byref(mm)),
                   "drag_plan_config")
        return lm.value, self.MFMA_MODES[mm.value]

    def set_config(self, lane_max, mfma_mode):
        """Pin (lane_max, mfma_mode) instead of the tuned configuration
        (drag_plan_set_config); mfma_mode is a key or value of MFMA_MODES."""
        if isinstance(mfma_mode, str):
            mfma_mode = {v: k for k, v in self.MFMA_MODES.items()}[mfma_mode]
        _lib.check(_lib.lib().drag_plan_set_config(self._plan, int(lane_max), int(mfma_mode)),
                   "drag_plan_set_config")

    def k_max(self):
        """The Taylor cap K per species count, index N - 1 (drag_plan_k_max)."""
        ks = (ctypes.c_int32 * 16)()
        _lib.check(_lib.lib().drag_plan_k_max(self._plan, ks), "drag_plan_k_max")
        return list(ks)

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            _lib.lib().drag_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""MI355X (gfx950) brute-force incoherent dedispersion.

A thin Python binding over the C ABI declared in ``include/dd.h``: every
step of the computation runs in the HIP library ``libdd_mi355x.so`` built
in this directory; this module only marshals arguments.  PyTorch supplies
device memory (tensors) and streams.  There is no CPU fallback: if the
library is missing, importing the compute entry points raises.

Usage::

    plan = Plan(freqs_mhz, tsamp_s, nsamp, [(lo, hi, step, ds), ...], "u8")
    out = dedisperse(x_u8_cuda, plan)          # int32 [out_elems]
    per_range = plan.split(out)                # list of [ndms_r, nout_r] views
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from ._lib import DDError, check, lib, library_path  # noqa: F401

DD_U8, DD_F32 = 0, 1
_DTYPES = {"u8": DD_U8, "f32": DD_F32}


class _Range(ctypes.Structure):
    _fields_ = [("dm_lo", ctypes.c_double), ("dm_hi", ctypes.c_double),
                ("dm_step", ctypes.c_double), ("downsample", ctypes.c_int32)]


@dataclass(frozen=True)
class RangeInfo:
    ndms: int
    nout: int
    out_offset: int
    max_shift: int
    downsample: int


class _Options(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("stage_chans", ctypes.c_int32),
                ("dm_tile", ctypes.c_int32), ("time_tile", ctypes.c_int32)]


class Plan:
    """Immutable dedispersion plan (wraps dd_plan_create_ex / dd_plan_destroy).
    `variant`, `stage_chans`, `dm_tile` and `time_tile` fix the strategy
    (0 = library default)."""

    def __init__(self, freqs_mhz, tsamp_s: float, nsamp: int, ranges, dtype: str = "u8",
                 variant: int = 0, stage_chans: int = 0, dm_tile: int = 0, time_tile: int = 0):
        L = lib()
        f = np.ascontiguousarray(freqs_mhz, dtype=np.float64)
        rg = (_Range * len(ranges))(*[_Range(float(a), float(b), float(c), int(d))
                                      for (a, b, c, d) in ranges])
        self._h = ctypes.c_void_p()
        self.dtype = dtype
        self.nchans = int(f.size)
        self.nsamp = int(nsamp)
        self.tsamp = float(tsamp_s)
        opts = _Options(int(variant), int(stage_chans), int(dm_tile), int(time_tile))
        check(L.dd_plan_create_ex(f.ctypes.data_as(ctypes.c_void_p), f.size, float(tsamp_s),
                                  int(nsamp), rg, len(ranges), _DTYPES[dtype], ctypes.byref(opts),
                                  ctypes.byref(self._h)), "dd_plan_create_ex")
        self.args = (f.copy(), float(tsamp_s), int(nsamp), [tuple(r) for r in ranges], dtype)
        nd, oe, ov = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        check(L.dd_plan_info(self._h, ctypes.byref(nd), ctypes.byref(oe), ctypes.byref(ov)),
              "dd_plan_info")
        self.ndms_total, self.out_elems, self.overlap = nd.value, oe.value, ov.value
        nr = ctypes.c_int32()
        check(L.dd_plan_nranges(self._h, ctypes.byref(nr)), "dd_plan_nranges")
        self.ranges = []
        for r in range(nr.value):
            a, b, c, d, e = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(),
                             ctypes.c_int32(), ctypes.c_int32())
            check(L.dd_plan_range(self._h, r, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                  ctypes.byref(d), ctypes.byref(e)), "dd_plan_range")
            self.ranges.append(RangeInfo(a.value, b.value, c.value, d.value, e.value))
        ws = ctypes.c_size_t()
        check(L.dd_workspace_bytes(self._h, ctypes.byref(ws)), "dd_workspace_bytes")
        self.workspace_bytes = ws.value
        tt, dt, cs, wg, va = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                              ctypes.c_int64(), ctypes.c_int32())
        check(L.dd_plan_strategy(self._h, ctypes.byref(tt), ctypes.byref(dt), ctypes.byref(cs),
                                 ctypes.byref(wg), ctypes.byref(va)), "dd_plan_strategy")
        self.strategy = {"time_tile": tt.value, "dm_tile": dt.value,
                         "chans_stage": cs.value, "workgroups": wg.value, "variant": va.value}

    @property
    def handle(self):
        if not self._h:
            raise DDError(-1, "plan has been closed")
        return self._h

    def dms(self) -> np.ndarray:
        out = np.zeros(self.ndms_total, dtype=np.float64)
        check(lib().dd_plan_dms(self.handle, out.ctypes.data_as(ctypes.c_void_p)), "dd_plan_dms")
        return out

    def shifts(self) -> np.ndarray:
        out = np.zeros((self.ndms_total, self.nchans), dtype=np.int32)
        check(lib().dd_plan_shifts(self.handle, out.ctypes.data_as(ctypes.c_void_p)),
              "dd_plan_shifts")
        return out

    def prepare(self) -> None:
        """Upload the device tables to the current device now."""
        check(lib().dd_plan_prepare(self.handle), "dd_plan_prepare")

    def split(self, out):
        """Per-range [ndms_r, nout_r] views of a flat output."""
        return [out[r.out_offset: r.out_offset + r.ndms * r.nout].view(r.ndms, r.nout)
                if hasattr(out, "view") and not isinstance(out, np.ndarray)
                else out[r.out_offset: r.out_offset + r.ndms * r.nout].reshape(r.ndms, r.nout)
                for r in self.ranges]

    def close(self) -> None:
        if self._h:
            lib().dd_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many plans of one dtype dedispersed together (dd_batch_*): u8 plans
    by persistent launches, one per kernel the plans use; f32 plans by one
    shift-and-sum launch over all beams.  The plans must stay alive as long
    as the batch."""

    def __init__(self, plans):
        L = lib()
        self.plans = list(plans)
        dts = {p.dtype for p in self.plans}
        self.dtype = self.plans[0].dtype if len(dts) == 1 else None
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        self._h = ctypes.c_void_p()
        check(L.dd_batch_create(arr, len(self.plans), ctypes.byref(self._h)), "dd_batch_create")
        ib, oe, wb, wi = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_int64()
        check(L.dd_batch_info(self._h, ctypes.byref(ib), ctypes.byref(oe), ctypes.byref(wb),
                              ctypes.byref(wi)), "dd_batch_info")
        self.in_bytes, self.out_elems = ib.value, oe.value
        self.workspace_bytes, self.work_items = wb.value, wi.value
        self.in_offsets, self.out_offsets = [], []
        for b in range(len(self.plans)):
            io, oo = ctypes.c_int64(), ctypes.c_int64()
            check(L.dd_batch_beam(self._h, b, ctypes.byref(io), ctypes.byref(oo)), "dd_batch_beam")
            self.in_offsets.append(io.value)
            self.out_offsets.append(oo.value)
        ng = ctypes.c_int32()
        check(L.dd_batch_groups(self._h, ctypes.byref(ng)), "dd_batch_groups")
        self.groups = []
        for g in range(ng.value):
            va, dt, wi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
            qb = (ctypes.c_int64 * 9)()
            check(L.dd_batch_group(self._h, g, ctypes.byref(va), ctypes.byref(dt),
                                   ctypes.byref(wi), qb), "dd_batch_group")
            self.groups.append({"variant": va.value, "dm_tile": dt.value,
                                "work_items": wi.value, "queue_bounds": list(qb)})

    @property
    def handle(self):
        if not self._h:
            raise DDError(-1, "batch has been closed")
        return self._h

    def prepare(self) -> None:
        check(lib().dd_batch_prepare(self.handle), "dd_batch_prepare")

    def pack(self, inputs, device=None):
        """One batch input buffer (bytes) holding every beam's [nchans, nsamp]
        block (uint8 or float32, the plans' dtype) at its byte offset
        (inputs: numpy arrays or tensors)."""
        import torch
        buf = torch.zeros(max(1, self.in_bytes), dtype=torch.uint8, device=device or "cuda")
        want = torch.uint8 if self.dtype == "u8" else torch.float32
        for p, off, x in zip(self.plans, self.in_offsets, inputs):
            t = torch.as_tensor(x).reshape(-1)
            if t.numel() != p.nchans * p.nsamp or t.dtype != want:
                raise ValueError("beam input has the wrong shape or dtype")
            nb = t.numel() * t.element_size()
            buf[off: off + nb].copy_(t.to(buf.device).view(torch.uint8))
        return buf

    def pack_weights(self, weights, device=None):
        """The batch weight buffer of an f32 batch: each beam's [nchans]
        weights in beam order, concatenated."""
        import torch
        parts = []
        for p, w in zip(self.plans, weights):
            t = torch.as_tensor(w, dtype=torch.float32).reshape(-1)
            if t.numel() != p.nchans:
                raise ValueError("beam weights have the wrong length")
            parts.append(t.to(device or "cuda"))
        return torch.cat(parts).contiguous()

    def split(self, out):
        """Per-beam flat outputs (views)."""
        return [out[o: o + p.out_elems] for p, o in zip(self.plans, self.out_offsets)]

    def split_input(self, buf):
        """Per-beam [nchans, nsamp] views of a float32 buffer in the batch
        input's layout (an f32 batch's dL/dx)."""
        return [buf[o // 4: o // 4 + p.nchans * p.nsamp].view(p.nchans, p.nsamp)
                for p, o in zip(self.plans, self.in_offsets)]

    def split_weights(self, buf):
        """Per-beam views of a buffer of every beam's channels concatenated."""
        out, at = [], 0
        for p in self.plans:
            out.append(buf[at: at + p.nchans])
            at += p.nchans
        return out

    def close(self) -> None:
        if self._h:
            lib().dd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dedisperse_batch(x, batch: Batch, out=None, ws=None, stream=None, weights=None):
    """Batched forward of every beam (dd_batch_forward, or
    dd_batch_forward_weighted with `weights`, the packed f32 weight buffer);
    x is the packed batch input (bytes).  Returns the flat batch output
    (int32 for u8 plans, float32 for f32 plans)."""
    import torch
    if x.dtype != torch.uint8 or not x.is_cuda or not x.is_contiguous() or \
            x.numel() < batch.in_bytes:
        raise ValueError("x must be the packed batch input (bytes) on the device")
    odt = torch.int32 if batch.dtype == "u8" else torch.float32
    if out is None:
        out = torch.empty(batch.out_elems, dtype=odt, device=x.device)
    if out.dtype != odt:
        raise ValueError(f"out must be a {odt} tensor")
    _on(out, x.device, "out")
    if ws is None:
        ws = torch.empty(batch.workspace_bytes, dtype=torch.uint8, device=x.device)
    wsb = _ws_bytes(ws, x.device)
    if weights is not None:
        if (weights.dtype != torch.float32
                or weights.numel() != sum(p.nchans for p in batch.plans)):
            raise ValueError("weights must be the packed float32 weights of every beam")
        _on(weights, x.device, "weights")
        check(lib().dd_batch_forward_weighted(batch.handle, _ptr(x), _ptr(weights), _ptr(out),
                                              out.numel(), _ptr(ws), wsb,
                                              _stream_ptr(stream)), "dd_batch_forward_weighted")
        return out
    check(lib().dd_batch_forward(batch.handle, _ptr(x), _ptr(out), out.numel(), _ptr(ws),
                                 wsb, _stream_ptr(stream)), "dd_batch_forward")
    return out


class Stream:
    """Chunked processing of a long series with the plan's largest delay as
    overlap (dd_stream_*).  push() returns the chunk's flat output; the first
    `step // ds_r` samples of each DM row of range r are its share of the
    one-shot output (emitted() slices them)."""

    def __init__(self, plan: Plan, time_major: bool = False):
        import torch
        self.plan = plan
        self.time_major = bool(time_major)
        self._h = ctypes.c_void_p()
        check(lib().dd_stream_create(plan.handle, int(self.time_major), ctypes.byref(self._h)),
              "dd_stream_create")
        first, step = ctypes.c_int64(), ctypes.c_int64()
        check(lib().dd_stream_info(self._h, ctypes.byref(first), ctypes.byref(step)),
              "dd_stream_info")
        self.first, self.step = first.value, step.value
        dt = torch.uint8 if plan.dtype == "u8" else torch.float32
        self.chunk = torch.empty((plan.nchans, plan.nsamp), dtype=dt, device="cuda")
        self.ws = workspace(plan)
        self.out = _out_tensor(plan, None, "cuda")

    def push(self, block, weights=None, stream=None):
        """Feed the next block ([nchans, n] channel-major or [n, nchans]
        time-major device tensor, n = first for the first push, then step).
        Returns (chunk index, flat output of the chunk)."""
        if block.dim() != 2 or block.dtype != self.chunk.dtype or \
                block.shape[1 if self.time_major else 0] != self.plan.nchans:
            raise ValueError(f"block must be a {self.chunk.dtype} "
                             + ("[n, nchans]" if self.time_major else "[nchans, n]") + " tensor")
        samples = block.shape[0] if self.time_major else block.shape[1]
        block = _on(block.contiguous(), self.chunk.device, "block")
        _check_weights(weights, self.plan, self.chunk.device)
        idx = ctypes.c_int64()
        check(lib().dd_stream_push(self._h, _ptr(block), int(samples), _ptr(self.chunk),
                                   _ptr(weights), _ptr(self.out), self.out.numel(), _ptr(self.ws),
                                   self.ws.numel(), ctypes.byref(idx), _stream_ptr(stream)),
              "dd_stream_push")
        return idx.value, self.out

    def emitted(self, out):
        """Per-range [ndms_r, step // ds_r] slices a chunk contributes."""
        return [o[:, : self.step // r.downsample] for o, r in zip(self.plan.split(out),
                                                                  self.plan.ranges)]

    def reset(self):
        check(lib().dd_stream_reset(self._h), "dd_stream_reset")

    def close(self):
        if self._h:
            lib().dd_stream_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def corner_turn(x, stream=None):
    """[nsamp, nchans] time-major device tensor -> [nchans, nsamp] (dd_corner_turn)."""
    import torch
    if x.dim() != 2 or x.dtype not in (torch.uint8, torch.float32) or not x.is_cuda:
        raise ValueError("x must be a 2-D uint8 or float32 device tensor")
    x = x.contiguous()
    n, c = x.shape
    out = torch.empty((c, n), dtype=x.dtype, device=x.device)
    check(lib().dd_corner_turn(DD_U8 if x.dtype == torch.uint8 else DD_F32, _ptr(x), n, c,
                               _ptr(out), n, _stream_ptr(stream)), "dd_corner_turn")
    return out


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace(plan: Plan, device=None):
    """Allocate the workspace a plan asks for (dd_workspace_bytes)."""
    import torch
    return torch.empty(max(1, plan.workspace_bytes), dtype=torch.uint8,
                       device=device or "cuda")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _on(t, dev, what):
    """t (when given) must be a contiguous tensor on the device `dev`: the
    library hands its address to kernels, which would fault on host memory."""
    if t is not None and (not t.is_cuda or t.device != dev or not t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous tensor on {dev}")
    return t


def _ws_bytes(ws, dev):
    """Bytes of a caller's workspace tensor on `dev` (any dtype)."""
    _on(ws, dev, "ws")
    return ws.numel() * ws.element_size() if ws is not None else 0


def _check_input(x, plan):
    import torch
    want = torch.uint8 if plan.dtype == "u8" else torch.float32
    if x.dtype != want or x.dim() != 2 or tuple(x.shape) != (plan.nchans, plan.nsamp):
        raise ValueError(f"input must be {want} [{plan.nchans}, {plan.nsamp}], got "
                         f"{x.dtype} {tuple(x.shape)}")
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("input must be a contiguous device tensor")


def _check_weights(weights, plan, dev=None):
    import torch
    if weights is None:
        return
    if (weights.dtype != torch.float32 or not weights.is_cuda or not weights.is_contiguous()
            or weights.numel() != plan.nchans):
        raise ValueError(f"weights must be a contiguous device float32 tensor of {plan.nchans}")
    if dev is not None:
        _on(weights, dev, "weights")


def _out_tensor(plan, out, device):
    import torch
    odt = torch.int32 if plan.dtype == "u8" else torch.float32
    if out is None:
        return torch.empty(plan.out_elems, dtype=odt, device=device)
    if out.dtype != odt or not out.is_cuda or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous device {odt} tensor")
    if not isinstance(device, str):
        _on(out, device, "out")
    return out


def dedisperse(x, plan: Plan, out=None, weights=None, ws=None, stream=None, step="all"):
    """Forward dedispersion of a channel-major [nchans, nsamp] device tensor
    (dd_forward).  Returns the flat output: int32 for u8 plans, float32 for
    f32 plans (per-channel float32 `weights` allowed there).

    step="sum" runs only the shift-and-sum (dd_forward_sum); the workspace
    must then hold what bin_input() wrote for the same input."""
    if step not in ("all", "sum"):
        raise ValueError("step must be 'all' or 'sum'")
    if step == "all":
        _check_input(x, plan)
        _check_weights(weights, plan, x.device)
    out = _out_tensor(plan, out, x.device if x is not None else "cuda")
    if ws is None:
        if step == "sum":
            raise ValueError("step='sum' needs the workspace bin_input() filled")
        ws = workspace(plan, out.device)
    wsb = _ws_bytes(ws, out.device)
    if step == "all":
        check(lib().dd_forward(plan.handle, _ptr(x), _ptr(weights), _ptr(out), out.numel(),
                               _ptr(ws), wsb, _stream_ptr(stream)), "dd_forward")
    else:
        check(lib().dd_forward_sum(plan.handle, _ptr(out), out.numel(), _ptr(ws), wsb,
                                   _stream_ptr(stream)), "dd_forward_sum")
    return out


def dedisperse_noalloc(x, plan: Plan, out, weights=None, stream=None):
    """dd_forward_noalloc: the forward with the library's static workspace
    (no device allocation in the call).  `out` must be given; the plan must
    have been prepared on the device (plan.prepare())."""
    _check_input(x, plan)
    _check_weights(weights, plan, x.device)
    if out is None:
        raise ValueError("dedisperse_noalloc needs a preallocated `out`")
    out = _out_tensor(plan, out, x.device)
    check(lib().dd_forward_noalloc(plan.handle, _ptr(x), _ptr(weights), _ptr(out), out.numel(),
                                   _stream_ptr(stream)), "dd_forward_noalloc")
    return out


def bin_input(x, plan: Plan, ws, weights=None, stream=None):
    """The binning step alone (dd_forward_bin) into the workspace ws."""
    _check_input(x, plan)
    _check_weights(weights, plan, x.device)
    check(lib().dd_forward_bin(plan.handle, _ptr(x), _ptr(weights), _ptr(ws),
                               _ws_bytes(ws, x.device), _stream_ptr(stream)),
          "dd_forward_bin")
    return ws


def adjoint(grad_out, plan: Plan, x=None, weights=None, grad_in=True, grad_w=True, ws=None,
            stream=None):
    """Gradients of sum(grad_out * forward(x, w)) for an f32 plan
    (dd_adjoint).  Returns (dX or None, dw or None).  grad_in may be a
    contiguous device float32 [nchans, nsamp] tensor to write dX into."""
    import torch
    if plan.dtype != "f32":
        raise ValueError("the adjoint is defined for f32 plans")
    if (grad_out.dtype != torch.float32 or not grad_out.is_cuda or not grad_out.is_contiguous()
            or grad_out.numel() != plan.out_elems):
        raise ValueError(f"grad_out must be a contiguous device float32 tensor of {plan.out_elems}")
    dev = grad_out.device
    if grad_w:
        if x is None:
            raise ValueError("x is needed for the weight gradient")
    if x is not None:
        _check_input(x, plan)
        _on(x, dev, "x")
    _check_weights(weights, plan, dev)
    if isinstance(grad_in, torch.Tensor):
        if (grad_in.dtype != torch.float32 or grad_in.device != dev or not grad_in.is_contiguous()
                or tuple(grad_in.shape) != (plan.nchans, plan.nsamp)):
            raise ValueError(f"grad_in must be a contiguous float32 [{plan.nchans}, {plan.nsamp}] "
                             "tensor on grad_out's device")
        dx = grad_in
    else:
        dx = (torch.empty((plan.nchans, plan.nsamp), dtype=torch.float32, device=dev)
              if grad_in else None)
    dw = torch.empty(plan.nchans, dtype=torch.float32, device=dev) if grad_w else None
    if ws is None:
        ws = workspace(plan, dev)
    check(lib().dd_adjoint(plan.handle, _ptr(grad_out), _ptr(x), _ptr(weights), _ptr(dx),
                           _ptr(dw), _ptr(ws), _ws_bytes(ws, dev), _stream_ptr(stream)), "dd_adjoint")
    return dx, dw


def _check_beams(x, plan):
    import torch
    if (x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous()
            or x.shape[-2:] != (plan.nchans, plan.nsamp)):
        raise ValueError(f"x must be a contiguous device float32 [..., {plan.nchans}, "
                         f"{plan.nsamp}] tensor")
    return x.numel() // (plan.nchans * plan.nsamp)


def boxcar_loss(x, plan: Plan, weights=None, max_width: int = 32, ws=None, stream=None):
    """Sum over beams, DMs, widths 1..max_width (powers of two) and valid
    windows of squared boxcar sums of the dedispersed output, which is never
    stored (dd_boxcar_loss).  x: [nbeams, nchans, nsamp] or [nchans, nsamp]."""
    import torch
    nb = _check_beams(x, plan)
    _check_weights(weights, plan, x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    if ws is None:
        ws = workspace(plan, x.device)
    check(lib().dd_boxcar_loss(plan.handle, _ptr(x), nb, _ptr(weights), int(max_width),
                               _ptr(loss), _ptr(ws), _ws_bytes(ws, x.device), _stream_ptr(stream)),
          "dd_boxcar_loss")
    return loss[0]


def boxcar_backward(x, plan: Plan, weights=None, max_width: int = 32, grad_in=True,
                    grad_w=True, ws=None, stream=None):
    """(dL/dx, dL/dw) of boxcar_loss, recomputing the dedispersed output
    (dd_boxcar_backward)."""
    import torch
    nb = _check_beams(x, plan)
    _check_weights(weights, plan, x.device)
    dx = torch.empty_like(x) if grad_in else None
    dw = torch.empty(plan.nchans, dtype=torch.float32, device=x.device) if grad_w else None
    if ws is None:
        ws = workspace(plan, x.device)
    check(lib().dd_boxcar_backward(plan.handle, _ptr(x), nb, _ptr(weights), int(max_width),
                                   _ptr(dx), _ptr(dw), _ptr(ws), _ws_bytes(ws, x.device),
                                   _stream_ptr(stream)),
          "dd_boxcar_backward")
    return dx, dw


def batch_boxcar_workspace(batch: Batch, device=None):
    """A workspace for the batch boxcar calls (dd_batch_boxcar_workspace)."""
    import torch
    n = ctypes.c_size_t()
    check(lib().dd_batch_boxcar_workspace(batch.handle, ctypes.byref(n)), "dd_batch_boxcar_workspace")
    return torch.empty(max(1, n.value), dtype=torch.uint8, device=device or "cuda")


def _check_batch_input(x, batch: Batch):
    import torch
    if x.dtype != torch.uint8 or not x.is_cuda or not x.is_contiguous() or x.numel() < batch.in_bytes:
        raise ValueError("x must be the packed batch input (bytes) on the device")
    if batch.dtype != "f32":
        raise ValueError("the batch boxcar calls take f32 batches")


def _check_batch_weights(weights, batch: Batch, dev):
    import torch
    if weights is not None and (weights.dtype != torch.float32
                                or weights.numel() != sum(p.nchans for p in batch.plans)):
        raise ValueError("weights must be the packed float32 weights of every beam")
    _on(weights, dev, "weights")


def batch_boxcar_loss(x, batch: Batch, weights=None, max_width: int = 32, ws=None, stream=None):
    """Per-beam boxcar losses of a float32 batch (dd_batch_boxcar_loss): x
    and weights packed as for dedisperse_batch.  Returns [nbeams] float32."""
    import torch
    _check_batch_input(x, batch)
    _check_batch_weights(weights, batch, x.device)
    loss = torch.empty(len(batch.plans), dtype=torch.float32, device=x.device)
    if ws is None:
        ws = batch_boxcar_workspace(batch, x.device)
    check(lib().dd_batch_boxcar_loss(batch.handle, _ptr(x), _ptr(weights), int(max_width), _ptr(loss),
                                     _ptr(ws), _ws_bytes(ws, x.device), _stream_ptr(stream)),
          "dd_batch_boxcar_loss")
    return loss


def batch_boxcar_backward(x, batch: Batch, weights=None, max_width: int = 32, grad_in=True,
                          grad_w=True, ws=None, stream=None):
    """Gradients of the summed per-beam boxcar losses (dd_batch_boxcar_backward):
    dL/dx as a float32 buffer in the batch input's layout (beam b's block at
    in_offsets[b] // 4; see Batch.split_input) and dL/dw as every beam's
    weight gradient concatenated.  grad_in / grad_w: True (allocate), False
    (skip) or a float32 tensor to write into."""
    import torch
    _check_batch_input(x, batch)
    _check_batch_weights(weights, batch, x.device)
    nw = sum(p.nchans for p in batch.plans)

    def buf(arg, n):
        if isinstance(arg, torch.Tensor):
            if arg.dtype != torch.float32 or arg.numel() < n:
                raise ValueError(f"output buffers must be float32 tensors of {n} or more")
            return _on(arg, x.device, "an output buffer")
        return torch.zeros(n, dtype=torch.float32, device=x.device) if arg else None

    dx = buf(grad_in, batch.in_bytes // 4)
    dw = buf(grad_w, nw)
    if ws is None:
        ws = batch_boxcar_workspace(batch, x.device)
    check(lib().dd_batch_boxcar_backward(batch.handle, _ptr(x), _ptr(weights), int(max_width), _ptr(dx),
                                         _ptr(dw), _ptr(ws), _ws_bytes(ws, x.device), _stream_ptr(stream)),
          "dd_batch_boxcar_backward")
    return dx, dw


def _autograd_fn():
    import torch

    class DedispFn(torch.autograd.Function):
        """out = dedisperse(x, w) with a hand-written adjoint: backward runs
        dd_adjoint.  Saves (x, w), not the output."""

        @staticmethod
        def forward(ctx, x, weights, plan):
            ctx.plan = plan
            ctx.save_for_backward(x, weights)
            return dedisperse(x, plan, weights=weights)

        @staticmethod
        def backward(ctx, g):
            x, weights = ctx.saved_tensors
            need_x, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            dx, dw = adjoint(g.contiguous(), ctx.plan, x=x, weights=weights,
                             grad_in=need_x, grad_w=need_w)
            return dx, dw, None

    return DedispFn


def _boxcar_fn():
    import torch

    class BoxcarLossFn(torch.autograd.Function):
        """L = boxcar_loss(x, w) with a hand-written backward: forward runs
        dd_boxcar_loss and saves (x, w), never the dedispersed output;
        backward runs dd_boxcar_backward, which recomputes the output tiles
        it needs.  The upstream scalar gradient scales the result (autograd's
        chain rule; skipped when it is exactly 1)."""

        @staticmethod
        def forward(ctx, x, weights, plan, max_width):
            ctx.plan, ctx.max_width = plan, int(max_width)
            ctx.save_for_backward(x, weights)
            return boxcar_loss(x, plan, weights, ctx.max_width)

        @staticmethod
        def backward(ctx, gL):
            x, weights = ctx.saved_tensors
            need_x, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            dx, dw = boxcar_backward(x, ctx.plan, weights, ctx.max_width, grad_in=need_x,
                                     grad_w=need_w)
            if float(gL) != 1.0:
                dx = dx * gL if dx is not None else None
                dw = dw * gL if dw is not None else None
            return dx, dw, None, None

    return BoxcarLossFn


_FN = None
_BOX_FN = None


def boxcar_loss_autograd(x, weights, plan: Plan, max_width: int = 32):
    """Differentiable boxcar loss of the dedispersed output (the output is
    recomputed in the backward, never stored): gradients flow to x
    ([nbeams, nchans, nsamp] or [nchans, nsamp]) and to the shared
    per-channel weights (or None for unit weights)."""
    global _BOX_FN
    if _BOX_FN is None:
        _BOX_FN = _boxcar_fn()
    return _BOX_FN.apply(x, weights, plan, max_width)


def dedisperse_autograd(x, weights, plan: Plan):
    """Differentiable float32 dedispersion: gradients flow to x and to the
    per-channel weights through the hand-written HIP adjoint."""
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    return _FN.apply(x, weights, plan)

"""Python binding of libdop: argument marshalling only.

Every step of the propagation runs in the HIP library; this module checks
tensor shapes/dtypes/devices, passes raw device pointers and the current
HIP stream through the C ABI, and raises on any error status.  PyTorch is
used only for device memory and streams.
"""

import ctypes
import threading

import numpy as np
import torch

from . import _lib as L
from ._lib import DopError, DopProblem, DopServeStats, check, lib

OUT_MODES = {"crop": L.DOP_OUT_CROP, "full": L.DOP_OUT_FULL}


def _pair(v):
    if np.ndim(v) == 0:
        return int(v), int(v)
    a, b = v
    return int(a), int(b)


class Problem:
    """Problem description (paper Sec. 3.1): DOE grid n x n, padded grid
    m x m, pitch dx, distance z, wavelengths, refractive indices n(lambda_k)
    and PSF weights.  Lengths share one unit.  n and m may be (rows, columns)
    pairs for a rectangular DOE and grid (Table 2's 128,640 x 85,760); the
    attributes n and m are then the column counts.  With upsample = s >= 2
    the height map (and its gradient) is the coarse design of 1/s the rows
    and columns, nearest-neighbour upsampled inside the first pass."""

    def __init__(self, n, m, dx, z, lambdas, n_index, weights=None, out_mode="crop",
                 bandlimit=False, upsample=1):
        self.ny, self.nx = _pair(n)
        self.my, self.mx = _pair(m)
        self.n, self.m = self.nx, self.mx
        self.dx, self.z = float(dx), float(z)
        self.lambdas = np.ascontiguousarray(np.atleast_1d(lambdas), dtype=np.float64)
        self.n_index = np.ascontiguousarray(np.atleast_1d(n_index), dtype=np.float64)
        if self.lambdas.shape != self.n_index.shape:
            raise ValueError("lambdas and n_index must have the same length")
        self.weights = None if weights is None else np.ascontiguousarray(
            np.atleast_1d(weights), dtype=np.float32)
        if self.weights is not None and self.weights.shape != self.lambdas.shape:
            raise ValueError("weights must have one entry per wavelength")
        if out_mode not in OUT_MODES:
            raise ValueError("out_mode must be 'crop' or 'full'")
        self.out_mode = out_mode
        self.bandlimit = bool(bandlimit)
        self._c = DopProblem()
        c = self._c
        c.n, c.m, c.dx, c.z = self.nx, self.mx, self.dx, self.z
        c.ny, c.my = self.ny, self.my
        c.n_lambda = len(self.lambdas)
        c.lambda_ = self.lambdas.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.n_index = self.n_index.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.weight = (self.weights.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
                    if self.weights is not None else None)
        c.out_mode = OUT_MODES[out_mode]
        c.flags = L.DOP_BANDLIMIT if self.bandlimit else 0
        self.upsample = int(upsample)
        c.upsample = self.upsample

    @classmethod
    def from_dict(cls, d, out_mode="crop", bandlimit=False):
        return cls(d["n"], d["m"], d["dx"], d["z"], d["lams"], d["n_index"],
                   d.get("weights"), out_mode=out_mode, bandlimit=bandlimit)

    @property
    def k(self):
        return len(self.lambdas)

    @property
    def doe_shape(self):
        return (self.ny, self.nx)

    @property
    def grid_shape(self):
        return (self.my, self.mx)

    @property
    def h_shape(self):
        """Shape of the height map (the coarse design when upsampled)."""
        s = max(self.upsample, 1)
        return (self.ny // s, self.nx // s)

    @property
    def out_shape(self):
        return self.doe_shape if self.out_mode == "crop" else self.grid_shape

    def ptr(self):
        return ctypes.byref(self._c)


def workspace_size(prob, op=L.DOP_OP_PSF):
    out = ctypes.c_size_t(0)
    check(lib().dop_workspace_size(None, prob.ptr(), op, ctypes.byref(out)), "dop_workspace_size")
    return out.value


class Context:
    """A libdop context on one HIP device (owns the twiddle table)."""

    def __init__(self, device=None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        check(lib().dop_context_create(self.device, ctypes.byref(h)), "dop_context_create")
        self.handle = h
        self._ws = {}
        self._lock = threading.Lock()
        self.group_cap = {}  # field bytes -> largest wavelength group that fitted

    def workspace(self, nbytes, stream):
        """Cached device workspace of at least nbytes for this stream."""
        key = int(stream)
        with self._lock:
            buf = self._ws.get(key)
            if buf is None or buf.numel() < nbytes:
                buf = None
                self._ws.pop(key, None)
                buf = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
                self._ws[key] = buf
        return buf

    def workspace_bytes(self, stream):
        """Bytes of the workspace cached for this stream (0 if none)."""
        with self._lock:
            buf = self._ws.get(int(stream))
            return 0 if buf is None else buf.numel()

    def profile_enable(self, enable=True):
        """Start (clearing the totals) or stop per-pass HIP-event timing."""
        check(lib().dop_profile_enable(self.handle, 1 if enable else 0), "dop_profile_enable")

    def profile_read(self):
        """{pass name: (launches, total ms)} of the timed launches so far."""
        arr = (L.DopPassProfile * 8)()
        cnt = ctypes.c_int(0)
        check(lib().dop_profile_read(self.handle, arr, 8, ctypes.byref(cnt)), "dop_profile_read")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(cnt.value)}

    def release_workspaces(self):
        with self._lock:
            self._ws.clear()

    def close(self):
        if getattr(self, "handle", None):
            self._ws.clear()
            lib().dop_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def default_context(device=None):
    if device is None:
        device = torch.cuda.current_device()
    ctx = _contexts.get(device)
    if ctx is None:
        ctx = Context(device)
        _contexts[device] = ctx
    return ctx


def _stream_handle(device):
    return torch.cuda.current_stream(device).cuda_stream


def _need(t, name, dtype, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must live on cuda:{device}, got {t.device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def propagate(u_in, prob, k=0, ctx=None, out=None):
    """Eq. (3): propagate an n x n complex64 field by prob.z at wavelength
    prob.lambdas[k].  Returns n x n (crop) or m x m (full) complex64."""
    ctx = ctx or default_context(u_in.device.index)
    dev = ctx.device
    _need(u_in, "u_in", torch.complex64, prob.doe_shape, dev)
    if out is None:
        out = torch.empty(prob.out_shape, dtype=torch.complex64, device=u_in.device)
    _need(out, "out", torch.complex64, prob.out_shape, dev)
    stream = _stream_handle(dev)
    nbytes = workspace_size(prob, L.DOP_OP_PROPAGATE)
    ws = ctx.workspace(nbytes, stream)
    check(lib().dop_propagate(ctx.handle, prob.ptr(), int(k), _ptr(u_in), _ptr(out), _ptr(ws),
                              ws.numel(), ctypes.c_void_p(stream)), "dop_propagate")
    return out


def _psf_workspace(ctx, prob, stream, save_fields, group):
    """Workspace for dop_psf: one field, or room for a group of up to `group`
    wavelengths (the library then reads h and read-modify-writes the PSF once
    per group) when the fields are not saved and the memory is free."""
    field = workspace_size(prob, L.DOP_OP_PSF)
    g = 1 if save_fields else max(1, min(int(group), prob.k, ctx.group_cap.get(field, 4)))
    if g > 1:
        # what the device could hold: free memory, blocks torch keeps cached,
        # and this stream's workspace (replaced below), less a margin
        free, _ = torch.cuda.mem_get_info(ctx.device)
        spare = torch.cuda.memory_reserved(ctx.device) - torch.cuda.memory_allocated(ctx.device)
        budget = free + spare + ctx.workspace_bytes(stream) - (4 << 30)
        g = max(1, min(g, budget // field))
    while g > 1:
        try:
            return ctx.workspace(g * field, stream), g * field
        except torch.cuda.OutOfMemoryError:
            g -= 1
            ctx.group_cap[field] = g  # do not try the larger group again
    return ctx.workspace(field, stream), field


def psf(h, prob, amp=None, save_fields=False, ctx=None, out=None, group=4):
    """Eq. (1)-(4): wavelength-summed PSF of height map h (n x n float32).
    With save_fields=True also returns the K x n x n complex64 fields.
    `group` caps the wavelengths processed together (1 = one at a time;
    the result is bitwise the same)."""
    ctx = ctx or default_context(h.device.index)
    dev = ctx.device
    _need(h, "h", torch.float32, prob.h_shape, dev)
    if amp is not None:
        _need(amp, "amp", torch.float32, prob.doe_shape, dev)
    if out is None:
        out = torch.empty(prob.out_shape, dtype=torch.float32, device=h.device)
    _need(out, "out", torch.float32, prob.out_shape, dev)
    saved = None
    if save_fields:
        saved = torch.empty((prob.k,) + prob.doe_shape, dtype=torch.complex64, device=h.device)
    stream = _stream_handle(dev)
    ws, nbytes = _psf_workspace(ctx, prob, stream, save_fields, group)
    check(lib().dop_psf(ctx.handle, prob.ptr(), _ptr(h), _ptr(amp), _ptr(out), _ptr(saved),
                        _ptr(ws), nbytes, ctypes.c_void_p(stream)), "dop_psf")
    return (out, saved) if save_fields else out


def psf_noalloc(h, prob, amp=None, out=None, saved=None, ctx=None):
    """psf() through dop_psf_noalloc: the library's static device scratch is
    the workspace, so the call allocates no device memory inside the library
    (pass `out`, and `saved` for the fields, to allocate nothing here either).
    Grids up to 4096 x 4096; calls that overlap on one device race."""
    ctx = ctx or default_context(h.device.index)
    dev = ctx.device
    _need(h, "h", torch.float32, prob.h_shape, dev)
    if amp is not None:
        _need(amp, "amp", torch.float32, prob.doe_shape, dev)
    if out is None:
        out = torch.empty(prob.out_shape, dtype=torch.float32, device=h.device)
    _need(out, "out", torch.float32, prob.out_shape, dev)
    if saved is not None:
        _need(saved, "saved", torch.complex64, (prob.k,) + prob.doe_shape, dev)
    check(lib().dop_psf_noalloc(ctx.handle, prob.ptr(), _ptr(h), _ptr(amp), _ptr(out), _ptr(saved),
                                ctypes.c_void_p(_stream_handle(dev))), "dop_psf_noalloc")
    return out


def psf_backward(h, prob, saved_u, grad_psf, amp=None, ctx=None, out=None):
    """dL/dh given dL/dPSF (crop) and the fields saved by psf(); dL/dh has
    the shape of h (the coarse design when upsampled)."""
    ctx = ctx or default_context(h.device.index)
    dev = ctx.device
    _need(h, "h", torch.float32, prob.h_shape, dev)
    _need(saved_u, "saved_u", torch.complex64, (prob.k,) + prob.doe_shape, dev)
    _need(grad_psf, "grad_psf", torch.float32, prob.doe_shape, dev)
    if amp is not None:
        _need(amp, "amp", torch.float32, prob.doe_shape, dev)
    if out is None:
        out = torch.empty(prob.h_shape, dtype=torch.float32, device=h.device)
    _need(out, "out", torch.float32, prob.h_shape, dev)
    stream = _stream_handle(dev)
    nbytes = workspace_size(prob, L.DOP_OP_PSF_BACKWARD)
    ws = ctx.workspace(nbytes, stream)
    check(lib().dop_psf_backward(ctx.handle, prob.ptr(), _ptr(h), _ptr(amp), _ptr(saved_u),
                                 _ptr(grad_psf), _ptr(out), _ptr(ws), ws.numel(),
                                 ctypes.c_void_p(stream)), "dop_psf_backward")
    return out


class DopPSF(torch.autograd.Function):
    """PSF(h) with the hand-written adjoint as its backward (crop output)."""

    @staticmethod
    def forward(fctx, h, prob, amp=None):
        out, saved = psf(h.detach().contiguous(), prob, amp=amp, save_fields=True)
        fctx.prob = prob
        fctx.amp = amp
        fctx.save_for_backward(h, saved)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        h, saved = fctx.saved_tensors
        g = psf_backward(h.detach().contiguous(), fctx.prob, saved,
                         grad_out.contiguous().to(torch.float32), amp=fctx.amp)
        return g, None, None


def psf_autograd(h, prob, amp=None):
    return DopPSF.apply(h, prob, amp)


PROBE_KINDS = {"read": L.DOP_PROBE_READ, "write": L.DOP_PROBE_WRITE, "copy": L.DOP_PROBE_COPY,
               "inplace": L.DOP_PROBE_INPLACE, "passc": L.DOP_PROBE_PASSC}


def probe_bandwidth(kind, buf, nbytes=None, m=0, ctx=None):
    """Enqueue one bandwidth probe (dop_probe_bandwidth) over the first
    nbytes of the device tensor buf (its contents are overwritten) on the
    current stream; returns the bytes the kernel moves."""
    ctx = ctx or default_context(buf.device.index)
    nbytes = buf.numel() * buf.element_size() if nbytes is None else int(nbytes)
    if nbytes > buf.numel() * buf.element_size():
        raise ValueError("nbytes exceeds the buffer")
    moved = ctypes.c_size_t(0)
    check(lib().dop_probe_bandwidth(ctx.handle, PROBE_KINDS[kind], _ptr(buf), nbytes, int(m),
                                    ctypes.byref(moved),
                                    ctypes.c_void_p(_stream_handle(ctx.device))),
          "dop_probe_bandwidth")
    return moved.value


UPSAMPLE_KINDS = {"nearest": L.DOP_UPSAMPLE_NEAREST, "lanczos3": L.DOP_UPSAMPLE_LANCZOS3}


def upsample(coarse, s, kind="nearest", ctx=None, out=None):
    """Super-resolved front end: the (ncy s) x (ncx s) map Wy coarse Wx^T of
    an ncy x ncx float32 design (nearest or Lanczos-3 interpolation)."""
    ctx = ctx or default_context(coarse.device.index)
    dev = ctx.device
    if coarse.dim() != 2:
        raise ValueError("coarse must be a 2-D map")
    ncy, ncx = int(coarse.shape[0]), int(coarse.shape[1])
    _need(coarse, "coarse", torch.float32, (ncy, ncx), dev)
    fine = (ncy * int(s), ncx * int(s))
    if out is None:
        out = torch.empty(fine, dtype=torch.float32, device=coarse.device)
    _need(out, "out", torch.float32, fine, dev)
    check(lib().dop_upsample_rect(ctx.handle, UPSAMPLE_KINDS[kind], ncy, ncx, int(s),
                                  _ptr(coarse), _ptr(out), ctypes.c_void_p(_stream_handle(dev))),
          "dop_upsample_rect")
    return out


def upsample_adjoint(grad_fine, s, kind="nearest", ctx=None, out=None):
    """Wy^T grad_fine Wx: a fine-grid gradient carried back to the design."""
    ctx = ctx or default_context(grad_fine.device.index)
    dev = ctx.device
    if grad_fine.dim() != 2:
        raise ValueError("grad_fine must be a 2-D map")
    nfy, nfx = int(grad_fine.shape[0]), int(grad_fine.shape[1])
    if nfy % int(s) or nfx % int(s):
        raise ValueError(f"fine size {nfy} x {nfx} is not a multiple of {s}")
    _need(grad_fine, "grad_fine", torch.float32, (nfy, nfx), dev)
    ncy, ncx = nfy // int(s), nfx // int(s)
    if out is None:
        out = torch.empty((ncy, ncx), dtype=torch.float32, device=grad_fine.device)
    _need(out, "out", torch.float32, (ncy, ncx), dev)
    check(lib().dop_upsample_adjoint_rect(ctx.handle, UPSAMPLE_KINDS[kind], ncy, ncx, int(s),
                                          _ptr(grad_fine), _ptr(out),
                                          ctypes.c_void_p(_stream_handle(dev))),
          "dop_upsample_adjoint_rect")
    return out


class DopUpsample(torch.autograd.Function):
    """upsample() with upsample_adjoint() as its backward."""

    @staticmethod
    def forward(fctx, coarse, s, kind="nearest"):
        fctx.s, fctx.kind = s, kind
        return upsample(coarse.detach().contiguous(), s, kind)

    @staticmethod
    def backward(fctx, grad_out):
        return upsample_adjoint(grad_out.contiguous().to(torch.float32), fctx.s, fctx.kind), None, None


class Server:
    """Continuous-batching PSF server over a device arena (see dop.h)."""

    POLICIES = {"fifo": L.DOP_SERVE_FIFO, "size_aware": L.DOP_SERVE_SIZE_AWARE,
                "chunked": L.DOP_SERVE_CHUNKED}

    def __init__(self, arena_bytes, max_slots=4, ctx=None, mock_us_per_mpix=None,
                 policy="chunked", share_ratio=0.25, age_bound_s=0.25):
        self.mock = mock_us_per_mpix is not None
        h = ctypes.c_void_p()
        if self.mock:
            self._arena = None
            check(lib().dop_serve_create_mock(ctypes.c_void_p(256), int(arena_bytes),
                                              int(max_slots), float(mock_us_per_mpix),
                                              ctypes.byref(h)), "dop_serve_create_mock")
        else:
            self.ctx = ctx or default_context()
            self._arena = torch.empty(int(arena_bytes), dtype=torch.uint8,
                                      device=f"cuda:{self.ctx.device}")
            torch.cuda.synchronize(self.ctx.device)
            check(lib().dop_serve_create(self.ctx.handle, _ptr(self._arena), int(arena_bytes),
                                         int(max_slots), ctypes.byref(h)), "dop_serve_create")
        self.handle = h
        self._keep = {}
        self.set_policy(policy, share_ratio=share_ratio, age_bound_s=age_bound_s)

    def set_policy(self, policy, share_ratio=0.25, age_bound_s=0.25):
        """Scheduling policy: "chunked" (its age bound in seconds), "fifo" or
        "size_aware" (its share ratio); see dop_serve_set_policy."""
        param = {"chunked": age_bound_s, "size_aware": share_ratio}.get(policy, 0.0)
        check(lib().dop_serve_set_policy(self.handle, self.POLICIES[policy], float(param)),
              "dop_serve_set_policy")

    def submit(self, prob, h, out, amp=None):
        """Queue a PSF request; h/amp/out are device tensors (or, for a mock
        server, any integers standing in for addresses).  Returns the
        ticket."""
        t = ctypes.c_uint64(0)
        if self.mock:
            hp, ap, op = ctypes.c_void_p(int(h)), None, ctypes.c_void_p(int(out))
        else:
            dev = self.ctx.device
            _need(h, "h", torch.float32, prob.h_shape, dev)
            _need(out, "out", torch.float32, prob.out_shape, dev)
            if amp is not None:
                _need(amp, "amp", torch.float32, prob.doe_shape, dev)
            hp, ap, op = _ptr(h), _ptr(amp), _ptr(out)
            # the server's streams are not ordered after the caller's: let the
            # work that produced h / amp (and last used out) finish first
            torch.cuda.current_stream(dev).synchronize()
        check(lib().dop_serve_submit(self.handle, prob.ptr(), hp, ap, op, ctypes.byref(t)),
              "dop_serve_submit")
        self._keep[t.value] = (prob, h, out, amp)
        return t.value

    def poll(self, ticket):
        return lib().dop_serve_poll(self.handle, ticket)

    def wait(self, ticket, timeout_s=-1.0):
        st = lib().dop_serve_wait(self.handle, ticket, float(timeout_s))
        if st != L.DOP_OK:
            raise DopError(st, "dop_serve_wait", L.last_error())
        self._keep.pop(ticket, None)
        return st

    def latency_ms(self, ticket):
        v = ctypes.c_double(0)
        check(lib().dop_serve_latency(self.handle, ticket, ctypes.byref(v)), "dop_serve_latency")
        return v.value

    def stats(self):
        s = DopServeStats()
        check(lib().dop_serve_stats_get(self.handle, ctypes.byref(s)), "dop_serve_stats_get")
        return {f: getattr(s, f) for f, _ in DopServeStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().dop_serve_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

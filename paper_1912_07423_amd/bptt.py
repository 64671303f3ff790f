"""Surrogate-gradient BPTT of a recurrent LIF network as a torch.autograd.Function over
the C ABI (snn_bptt_* in include/snn.h).  The forward pass and the hand-written adjoint
run in the library's HIP kernels; this module only passes device pointers.

    plan = RecurrentLIF(in_mask, rec_mask, n_out, batch, steps)      # structure
    loss = plan.loss(x, w_in, w_rec, w_out, labels)                   # autograd-aware
    loss.backward()                                                   # grads of w_*

`w_in` / `w_rec` are the values of the sparse weights in CSR order (rows = presynaptic
neuron, targets ascending), as returned by `plan.csr_values(dense)`.
"""
import ctypes as C
import math

import numpy as np

from . import _lib as L


def _csr(mask):
    mask = np.asarray(mask, bool)
    rows, cols = np.nonzero(mask)           # row-major: rows ascending, columns ascending
    ptr = np.zeros(mask.shape[0] + 1, np.uint64)
    np.cumsum(np.bincount(rows, minlength=mask.shape[0]), out=ptr[1:])
    return ptr, cols.astype(np.int32), (rows, cols)


class RecurrentLIF:
    """Plan (structure + workspace) of the recurrent LIF network on one GPU.  The per-step
    kernels of each pass are replayed from HIP graphs captured at the first call, or
    launched one by one with eager=True (same kernels, same results)."""

    def __init__(self, in_mask, rec_mask, n_out, batch, steps, checkpoint=25, tau_ms=20.0,
                 tau_out_ms=20.0, dt_ms=1.0, theta=1.0, slope=25.0, smooth=False, eager=False,
                 device=0):
        import torch
        self._lib = L.load()
        self._h = None
        self.device = torch.device("cuda", device)
        in_mask, rec_mask = np.asarray(in_mask, bool), np.asarray(rec_mask, bool)
        self.n_in, self.n_hidden = in_mask.shape
        assert rec_mask.shape == (self.n_hidden, self.n_hidden)
        self.n_out, self.batch, self.steps = int(n_out), int(batch), int(steps)
        self.smooth = bool(smooth)
        self._in_ptr, self._in_col, self._in_idx = _csr(in_mask)
        self._rec_ptr, self._rec_col, self._rec_idx = _csr(rec_mask)
        d = L.BpttDesc(batch=self.batch, steps=self.steps, n_in=self.n_in, n_hidden=self.n_hidden,
                       n_out=self.n_out, checkpoint=int(checkpoint),
                       beta=math.exp(-dt_ms / tau_ms), beta_out=math.exp(-dt_ms / tau_out_ms),
                       theta=theta, slope=slope, smooth=1 if smooth else 0, eager=1 if eager else 0)
        self.desc = d
        stream = torch.cuda.current_stream(self.device)

        alloc_fn = torch.cuda.caching_allocator_alloc
        delete_fn = torch.cuda.caching_allocator_delete

        def _alloc(nbytes, s, ctx):
            try:
                return alloc_fn(int(nbytes), device, stream)
            except Exception:
                return None

        def _free(ptr, nbytes, s, ctx):
            try:
                delete_fn(ptr)
            except Exception:
                pass  # interpreter shutdown: the process is releasing the device anyway

        self._keep = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
        self._alloc = L.Allocator(self._keep[0], self._keep[1], None)
        h = C.c_void_p()
        L.check(self._lib.snn_bptt_create(
            C.byref(d), self._in_ptr.ctypes.data, self._in_col.ctypes.data,
            self._rec_ptr.ctypes.data, self._rec_col.ctypes.data, C.byref(self._alloc),
            stream.cuda_stream or None, C.byref(h)))
        self._h = h
        self.nnz_in, self.nnz_rec = len(self._in_col), len(self._rec_col)

    def close(self):
        if self._h:
            self._lib.snn_bptt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- weights in CSR order ---------------------------------------------------------
    def csr_values(self, w_in_dense, w_rec_dense):
        """Dense [n_in, n_hidden] / [n_hidden, n_hidden] -> CSR-ordered value vectors."""
        return (np.ascontiguousarray(np.asarray(w_in_dense)[self._in_idx], np.float32),
                np.ascontiguousarray(np.asarray(w_rec_dense)[self._rec_idx], np.float32))

    def dense(self, v_in, v_rec):
        """CSR-ordered value vectors -> dense matrices (zeros off the masks)."""
        a = np.zeros((self.n_in, self.n_hidden), np.asarray(v_in).dtype)
        b = np.zeros((self.n_hidden, self.n_hidden), np.asarray(v_rec).dtype)
        a[self._in_idx] = v_in
        b[self._rec_idx] = v_rec
        return a, b

    # -- calls ------------------------------------------------------------------------
    def _stream(self):
        import torch
        return torch.cuda.current_stream(self.device).cuda_stream or None

    def _check(self, x, w_in, w_rec, w_out, labels):
        import torch
        for t, shape, dt in ((x, (self.batch, self.steps, self.n_in), torch.float32),
                             (w_in, (self.nnz_in,), torch.float32),
                             (w_rec, (self.nnz_rec,), torch.float32),
                             (w_out, (self.n_hidden, self.n_out), torch.float32),
                             (labels, (self.batch,), torch.int32)):
            if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"expected a contiguous {dt} tensor of shape {shape} on {self.device}")

    def forward(self, x, w_in, w_rec, w_out, labels):
        import torch
        self._check(x, w_in, w_rec, w_out, labels)
        loss = torch.empty((), dtype=torch.float32, device=self.device)
        L.check(self._lib.snn_bptt_forward(self._h, x.data_ptr(), w_in.data_ptr(), w_rec.data_ptr(),
                                           w_out.data_ptr(), labels.data_ptr(), loss.data_ptr(),
                                           self._stream()))
        return loss

    def backward(self, w_in, w_rec, w_out, g_loss=None):
        import torch
        g_in = torch.empty_like(w_in)
        g_rec = torch.empty_like(w_rec)
        g_out = torch.empty_like(w_out)
        L.check(self._lib.snn_bptt_backward(self._h, w_in.data_ptr(), w_rec.data_ptr(), w_out.data_ptr(),
                                            g_loss.data_ptr() if g_loss is not None else None,
                                            g_in.data_ptr(), g_rec.data_ptr(), g_out.data_ptr(),
                                            self._stream()))
        return g_in, g_rec, g_out

    def trace(self):
        """Host copies of the latest forward pass: spikes [T, B, H], membrane
        checkpoints [n_seg, B, H], readout maxima and argmax steps [B, O]."""
        T, H, B, O = self.steps, self.n_hidden, self.batch, self.n_out
        n_seg = -(-T // self.desc.checkpoint)
        s = np.zeros((T, H, 64), np.float32)
        v = np.zeros((n_seg, H, 64), np.float32)
        m = np.zeros((B, O), np.float32)
        tm = np.zeros((B, O), np.int32)
        L.check(self._lib.snn_bptt_get_trace(self._h, s.ctypes.data, v.ctypes.data, m.ctypes.data,
                                             tm.ctypes.data, self._stream()))
        return (s[:, :, :B].transpose(0, 2, 1), v[:, :, :B].transpose(0, 2, 1), m, tm)

    def loss(self, x, w_in, w_rec, w_out, labels):
        return _Function.apply(w_in, w_rec, w_out, self, x, labels)


def _function():
    import torch

    class RecurrentLIFFunction(torch.autograd.Function):
        """loss = f(w_in, w_rec, w_out); backward = the library's adjoint pass.  The
        backward pass uses the trajectory of the plan's latest forward pass."""

        @staticmethod
        def forward(ctx, w_in, w_rec, w_out, plan, x, labels):
            loss = plan.forward(x, w_in, w_rec, w_out, labels)
            ctx.plan = plan
            ctx.generation = getattr(plan, "_generation", 0) + 1
            plan._generation = ctx.generation
            ctx.save_for_backward(w_in, w_rec, w_out)
            return loss

        @staticmethod
        def backward(ctx, g):
            plan = ctx.plan
            if getattr(plan, "_generation", None) != ctx.generation:
                raise RuntimeError("the plan ran another forward pass since this one; "
                                   "backward needs the latest forward's trajectory")
            w_in, w_rec, w_out = ctx.saved_tensors
            g = g.detach().to(torch.float32).contiguous()
            g_in, g_rec, g_out = plan.backward(w_in, w_rec, w_out, g)
            return g_in, g_rec, g_out, None, None, None

    return RecurrentLIFFunction


class _Lazy:
    def __init__(self):
        self._f = None

    def apply(self, *args):
        if self._f is None:
            self._f = _function()
        return self._f.apply(*args)


_Function = _Lazy()

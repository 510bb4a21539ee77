"""Weighted-quadrature formation of isogeometric Galerkin matrices on MI355X.

``Plan`` is a thin convenience wrapper over the C-ABI (include/wq.h, bound in
``_wq``): it allocates the device workspace and the CSR outputs with PyTorch
(device memory and streams only) and forwards every call to libwq.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _wq
from ._wq import (WQ_BASIS_BSPLINE, WQ_BASIS_NURBS, WQ_FP32, WQ_FP64, WQ_MASS, WQ_STATIC_SCRATCH_BYTES, WQ_STIFF,
                  WQError, check)

__all__ = ["Batch", "Plan", "WQError", "WQ_BASIS_BSPLINE", "WQ_BASIS_NURBS", "WQ_FP32", "WQ_FP64", "WQ_MASS",
           "WQ_STATIC_SCRATCH_BYTES", "WQ_STIFF"]


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Plan:
    """One single-patch problem (3D, or 2D given two knot vectors) on the
    current CUDA (HIP) device."""

    def __init__(self, knots3: Sequence[np.ndarray], p: int, precision: int = WQ_FP64):
        self._h = C.c_void_p()
        ks = [np.ascontiguousarray(k, dtype=np.float64) for k in knots3]
        self._keep = ks
        n_knots = (C.c_int64 * len(ks))(*[len(k) for k in ks])
        ptrs = (C.POINTER(C.c_double) * len(ks))(*[k.ctypes.data_as(C.POINTER(C.c_double)) for k in ks])
        check(_wq.wq_plan_create(len(ks), p, n_knots, ptrs, precision, C.byref(self._h)))
        self.d = len(ks)
        self.p = p
        self.precision = precision
        s = _wq.wq_sizes_t()
        check(_wq.wq_sizes(self._h, C.byref(s)), self._h)
        self.sizes = s
        self.n = tuple(s.n)
        self.n_qp = tuple(s.n_qp)
        self.n_rows = s.n_rows
        self.nnz = s.nnz
        self.n_qp_total = s.n_qp_total
        self.workspace = None

    @property
    def value_dtype(self):
        import torch
        return torch.float64 if self.precision == WQ_FP64 else torch.float32

    def qpoints(self, d: int) -> np.ndarray:
        x = np.zeros(self.n_qp[d], dtype=np.float64)
        check(_wq.wq_qpoints(self._h, d, x.ctypes.data_as(C.POINTER(C.c_double))), self._h)
        return x

    def bind(self, stream=None, workspace=None):
        import torch
        if workspace is None:
            workspace = torch.empty(self.sizes.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
        off = (-workspace.data_ptr()) % 256
        self.workspace = workspace
        check(_wq.wq_bind(self._h, workspace.data_ptr() + off, workspace.numel() - off, _stream(stream)), self._h)

    def setup(self, ctrl, coef=None, stream=None):
        """ctrl: device float64 tensor (n3, n2, n1, 3), or (n2, n1, 2) in 2D;
        coef: device float64
        tensor with n_qp_total entries (q1 fastest) or None for a = 1."""
        if ctrl.numel() != self.n_rows * self.d:
            raise ValueError(f"control net must hold {self.n_rows} x {self.d} values")
        if coef is not None and coef.numel() != self.n_qp_total:
            raise ValueError(f"coefficient must hold {self.n_qp_total} values")
        check(_wq.wq_setup(self._h, _ptr(ctrl), _ptr(coef), _stream(stream)), self._h)

    def setup_nurbs(self, ctrl, weights, coef=None, basis: int = 0, stream=None):
        """wq_setup_nurbs: a rational map with the control points' weights
        (device float64, n_rows values); basis WQ_BASIS_BSPLINE (0) or
        WQ_BASIS_NURBS (1, mass only)."""
        if ctrl.numel() != self.n_rows * self.d:
            raise ValueError(f"control net must hold {self.n_rows} x {self.d} values")
        if weights.numel() != self.n_rows:
            raise ValueError(f"weights must hold {self.n_rows} values")
        if coef is not None and coef.numel() != self.n_qp_total:
            raise ValueError(f"coefficient must hold {self.n_qp_total} values")
        check(_wq.wq_setup_nurbs(self._h, _ptr(ctrl), _ptr(weights), _ptr(coef), basis, _stream(stream)), self._h)

    def set_geometry(self, ctrl, coef=None, stream=None):
        """wq_set_geometry: a new control net on the same knots (rules kept)."""
        if ctrl.numel() != self.n_rows * self.d:
            raise ValueError(f"control net must hold {self.n_rows} x {self.d} values")
        if coef is not None and coef.numel() != self.n_qp_total:
            raise ValueError(f"coefficient must hold {self.n_qp_total} values")
        check(_wq.wq_set_geometry(self._h, _ptr(ctrl), _ptr(coef), _stream(stream)), self._h)

    def set_coefficient(self, coef, stream=None):
        if coef is not None and coef.numel() != self.n_qp_total:
            raise ValueError(f"coefficient must hold {self.n_qp_total} values")
        check(_wq.wq_set_coefficient(self._h, _ptr(coef), _stream(stream)), self._h)

    def qp_physical(self, stream=None):
        import torch
        shape = {3: (self.n_qp[2], self.n_qp[1], self.n_qp[0], 3),
                 2: (self.n_qp[1], self.n_qp[0], 2),
                 1: (self.n_qp[0], 1)}[self.d]
        x = torch.empty(shape, dtype=torch.float64, device="cuda")
        check(_wq.wq_qp_physical(self._h, _ptr(x), _stream(stream)), self._h)
        return x

    def pattern(self, row_ptr=None, col_idx=None, stream=None):
        import torch
        if row_ptr is None:
            row_ptr = torch.empty(self.n_rows + 1, dtype=torch.int64, device="cuda")
        if col_idx is None:
            col_idx = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        check(_wq.wq_pattern(self._h, _ptr(row_ptr), _ptr(col_idx), _stream(stream)), self._h)
        return row_ptr, col_idx

    def assemble(self, which: int, mass=None, stiff=None, stream=None):
        import torch
        if (which & WQ_MASS) and mass is None:
            mass = torch.empty(self.nnz, dtype=self.value_dtype, device="cuda")
        if (which & WQ_STIFF) and stiff is None:
            stiff = torch.empty(self.nnz, dtype=self.value_dtype, device="cuda")
        check(_wq.wq_assemble(self._h, which, _ptr(mass) if which & WQ_MASS else None,
                              _ptr(stiff) if which & WQ_STIFF else None, _stream(stream)), self._h)
        return mass, stiff

    def request_bytes(self) -> int:
        n = C.c_size_t()
        check(_wq.wq_request_bytes(self._h, C.byref(n)), self._h)
        return n.value

    def assemble_request(self, ctx, coef, which: int, mass=None, stiff=None, stream=None):
        """Matrices for coefficient ``coef`` (device float64, n_qp_total, or
        None for a = 1) into a request context ``ctx`` (device uint8 tensor
        of at least request_bytes() + 256 bytes)."""
        import torch
        if coef is not None and coef.numel() != self.n_qp_total:
            raise ValueError(f"coefficient must hold {self.n_qp_total} values")
        if (which & WQ_MASS) and mass is None:
            mass = torch.empty(self.nnz, dtype=self.value_dtype, device="cuda")
        if (which & WQ_STIFF) and stiff is None:
            stiff = torch.empty(self.nnz, dtype=self.value_dtype, device="cuda")
        off = (-ctx.data_ptr()) % 256
        check(_wq.wq_assemble_request(self._h, ctx.data_ptr() + off, ctx.numel() - off, _ptr(coef), which,
                                      _ptr(mass) if which & WQ_MASS else None,
                                      _ptr(stiff) if which & WQ_STIFF else None, _stream(stream)), self._h)
        return mass, stiff

    def weights(self, d: int, pair: int, stream=None):
        import torch
        qcap = 3 * self.p + 1
        w = torch.empty((self.n[d], qcap), dtype=torch.float64, device="cuda")
        qs = torch.empty(self.n[d], dtype=torch.int32, device="cuda")
        qc = torch.empty(self.n[d], dtype=torch.int32, device="cuda")
        check(_wq.wq_weights(self._h, d, pair, _ptr(w), _ptr(qs), _ptr(qc), _stream(stream)), self._h)
        return w, qs, qc

    def field(self, stream=None):
        import torch
        f = torch.empty((7, self.n_qp[2], self.n_qp[1], self.n_qp[0]), dtype=self.value_dtype, device="cuda")
        check(_wq.wq_field(self._h, _ptr(f), _stream(stream)), self._h)
        return f

    def sync(self, stream=None):
        check(_wq.wq_sync(self._h, _stream(stream)), self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        # at interpreter exit the binding may already be torn down
        destroy = getattr(_wq, "wq_plan_destroy", None) if _wq is not None else None
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = C.c_void_p()


def _bcheck(status: int, batch) -> None:
    if status != _wq.WQ_OK:
        raise WQError(status, _wq.wq_batch_last_error(batch).decode() if batch else "")


class Batch:
    """Many patches (bound ``Plan`` objects) formed together: one persistent
    launch per class of equal (p, d, precision), schedules picked by the
    library's autotuner, optionally replayed from a captured HIP graph."""

    def __init__(self, plans: Sequence[Plan]):
        self.plans = list(plans)
        n = len(self.plans)
        arr = (C.c_void_p * n)(*[p._h.value for p in self.plans])
        self._h = C.c_void_p()
        _bcheck(_wq.wq_batch_create(n, arr, C.byref(self._h)), None)
        nb, nc = C.c_size_t(), C.c_int()
        _bcheck(_wq.wq_batch_sizes(self._h, C.byref(nb), C.byref(nc)), self._h)
        self.workspace_bytes, self.n_classes = nb.value, nc.value
        self.workspace = None
        self.mass = self.stiff = None

    def bind(self, mass=None, stiff=None, stream=None):
        """mass, stiff: per-patch device value tensors (or None)."""
        import torch
        n = len(self.plans)
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.workspace.data_ptr()) % 256
        self.mass, self.stiff = mass, stiff
        m = (C.c_void_p * n)(*[t.data_ptr() if t is not None else None for t in mass]) if mass else None
        s = (C.c_void_p * n)(*[t.data_ptr() if t is not None else None for t in stiff]) if stiff else None
        _bcheck(_wq.wq_batch_bind(self._h, self.workspace.data_ptr() + off, self.workspace.numel() - off,
                                  m, s, _stream(stream)), self._h)

    def tune(self, which: int, stream=None):
        _bcheck(_wq.wq_batch_tune(self._h, which, _stream(stream)), self._h)

    def assemble(self, which: int, use_graph: bool = False, stream=None):
        _bcheck(_wq.wq_batch_assemble(self._h, which, int(use_graph), _stream(stream)), self._h)

    def schedule(self):
        """Per class: degree, dimension, precision, patch count and the
        schedule (work-item target and persistent workgroups per compute unit;
        wgs_per_cu 0: the single-patch kernels, patch after patch)."""
        out = []
        info = (C.c_int * 6)()
        for k in range(self.n_classes):
            _bcheck(_wq.wq_batch_schedule(self._h, k, info), self._h)
            out.append(dict(zip(("p", "d", "precision", "patches", "work_target", "wgs_per_cu"), list(info))))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(_wq, "wq_batch_destroy", None) if _wq is not None else None
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = C.c_void_p()

"""An EnKF handle (include/hikf_enkf.h) whose device memory is owned by torch.

Marshalling only: the resident region and the outputs are torch tensors,
their pointers and the current stream go to libhikf.so, where every step of
the filter runs.
"""

import ctypes

import torch

from . import hikf as H
from .filter import _stream_handle


def enkf_problem(rowptr, col, val, r_diag, m, n_ens, timing=False, tile_rows=0, device="cuda"):
    """(hikf_enkf_problem, keepalive): device copies of H (CSR) and R;
    tile_rows: rows per workgroup of the transform (0 = automatic)."""
    t_rowptr = torch.as_tensor(rowptr, dtype=torch.int64).to(device).contiguous()
    t_col = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
    t_val = torch.as_tensor(val, dtype=torch.float64).to(device).contiguous()
    t_r = torch.as_tensor(r_diag, dtype=torch.float64).to(device).contiguous()
    pr = H.hikf_enkf_problem()
    pr.m, pr.p, pr.n_ens = int(m), int(len(t_rowptr) - 1), int(n_ens)
    pr.nnz = int(t_col.numel())
    pr.h_rowptr_dev = t_rowptr.data_ptr()
    pr.h_col_dev = t_col.data_ptr() if t_col.numel() else None
    pr.h_val_dev = t_val.data_ptr() if t_val.numel() else None
    pr.r_diag_dev = t_r.data_ptr()
    pr.timing = 1 if timing else 0
    pr.tile_rows = int(tile_rows)
    return pr, (t_rowptr, t_col, t_val, t_r)


def enkf_plan(problem):
    info = H.hikf_enkf_plan_info()
    H.check(H.hikf_enkf_plan(ctypes.byref(problem), ctypes.byref(info)), "hikf_enkf_plan")
    return info


class EnkfFilter:
    """Owns the resident region of one ensemble filter.  x0: (m, N) FP64
    device tensor, the initial ensemble (row = grid cell, members in
    columns)."""

    def __init__(self, problem, x0, keepalive=(), stream=None):
        self.problem = problem
        self.info = enkf_plan(problem)
        self.m, self.p, self.n = int(problem.m), int(problem.p), int(problem.n_ens)
        self.ld = int(self.info.ld)
        x0 = x0.contiguous()
        assert x0.dtype == torch.float64 and tuple(x0.shape) == (self.m, self.n) and x0.is_cuda
        self.resident = torch.empty(int(self.info.resident_bytes), dtype=torch.uint8,
                                    device=x0.device)
        self._keep = keepalive
        self.handle = ctypes.c_void_p()
        H.check(H.hikf_enkf_init(ctypes.byref(problem), ctypes.c_void_p(x0.data_ptr()),
                                 ctypes.c_void_p(self.resident.data_ptr()),
                                 self.info.resident_bytes, _stream_handle(stream),
                                 ctypes.byref(self.handle)), "hikf_enkf_init")
        if stream is not None:
            self.resident.record_stream(stream)

    def step(self, e, y, v, mean_out=None, var_out=None, stream=None):
        """Queue one step.  e: (m, ld) model-error draws or None; y: (p,);
        v: (p, N) observation perturbations (FP64 device tensors)."""
        if e is not None:
            assert e.dtype == torch.float64 and tuple(e.shape) == (self.m, self.ld)
            assert e.is_contiguous() and e.is_cuda
        for t, shape in ((y, (self.p,)), (v, (self.p, self.n))):
            assert t.dtype == torch.float64 and tuple(t.shape) == shape
            assert t.is_contiguous() and t.is_cuda
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None
               else ctypes.c_void_p(None))
        H.check(H.hikf_enkf_step(self.handle, ptr(e), ptr(y), ptr(v), ptr(mean_out),
                                 ptr(var_out), _stream_handle(stream)),
                "hikf_enkf_step", self.handle)

    def query(self):
        st = H.hikf_enkf_stats()
        H.check(H.hikf_enkf_query(self.handle, ctypes.byref(st)), "hikf_enkf_query", self.handle)
        return st

    def export(self, stream=None):
        x = torch.empty(self.m, self.n, dtype=torch.float64, device=self.resident.device)
        H.check(H.hikf_enkf_export(self.handle, ctypes.c_void_p(x.data_ptr()),
                                   _stream_handle(stream)), "hikf_enkf_export", self.handle)
        return x

    def import_(self, x, stream=None):
        xc = x.contiguous()
        assert xc.dtype == torch.float64 and tuple(xc.shape) == (self.m, self.n)
        if stream is not None and xc is not x:
            xc.record_stream(stream)          # a temporary read on `stream`
        H.check(H.hikf_enkf_import(self.handle, ctypes.c_void_p(xc.data_ptr()),
                                   _stream_handle(stream)), "hikf_enkf_import", self.handle)

    def close(self):
        if self.handle:
            H.hikf_enkf_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""A filter handle whose device memory is owned by torch.

Marshalling only: tensors are allocated with torch on the current CUDA (HIP)
device, their pointers and the current stream are handed to libhikf.so, and
every computation runs there.
"""

import ctypes

import torch

from . import hikf as H

PRECISIONS = {"f32": H.HIKF_FMM_F32, "f64": H.HIKF_FMM_F64, "bf16x3": H.HIKF_FMM_BF16X3,
              "bf16": H.HIKF_FMM_BF16}
PRIORS = {"zero": H.HIKF_PRIOR_ZERO, "scaled_i": H.HIKF_PRIOR_SCALED_I,
          "kernel": H.HIKF_PRIOR_KERNEL}
FAMILIES = {"powexp": H.HIKF_KERNEL_POWEXP, "r2": H.HIKF_KERNEL_TEST_R2}


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def problem_from_csr(dim, n, rowptr, col, val, r_diag, family="powexp", theta=1.0,
                     ell=1.0, gamma=1.0, prior="kernel", alpha=0.0, x0=None,
                     device="cuda"):
    """Device copies of the problem arrays plus the hikf_problem struct.

    Returns (problem, keepalive) where keepalive holds the tensors the struct
    points to.
    """
    t_rowptr = torch.as_tensor(rowptr, dtype=torch.int64).to(device).contiguous()
    t_col = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
    t_val = torch.as_tensor(val, dtype=torch.float64).to(device).contiguous()
    t_r = torch.as_tensor(r_diag, dtype=torch.float64).to(device).contiguous()
    t_x0 = None if x0 is None else torch.as_tensor(x0, dtype=torch.float64).to(device).contiguous()
    pr = H.hikf_problem()
    pr.dim, pr.n = int(dim), int(n)
    pr.kernel_family = FAMILIES[family]
    pr.prior_kind = PRIORS[prior]
    pr.theta, pr.ell, pr.gamma, pr.alpha = float(theta), float(ell), float(gamma), float(alpha)
    pr.p = int(len(t_rowptr) - 1)
    pr.nnz = int(t_col.numel())
    pr.h_rowptr_dev = t_rowptr.data_ptr()
    pr.h_col_dev = t_col.data_ptr() if t_col.numel() else None
    pr.h_val_dev = t_val.data_ptr() if t_val.numel() else None
    pr.r_diag_dev = t_r.data_ptr()
    pr.x0_dev = None if t_x0 is None else t_x0.data_ptr()
    return pr, (t_rowptr, t_col, t_val, t_r, t_x0)


def make_options(n_c=4, precision="f32", direct=False, timing=False, graph=False, riccati=0,
                 history=0, sparse=False, rowpass_variant=None, tune_cache=None,
                 psd_guard=False, m2l_eps=0.0):
    """hikf_options; rowpass_variant None = automatic (tuning cache or the
    built-in default), else the variant 0..7 to force."""
    op = H.hikf_options()
    op.n_c = int(n_c)
    op.fmm_precision = PRECISIONS[precision]
    op.direct = 1 if direct else 0
    op.timing = 1 if timing else 0
    op.graph = 1 if graph else 0
    op.riccati = int(riccati)
    op.history = int(history)
    op.sparse = 1 if sparse else 0
    op.rowpass_variant = 0 if rowpass_variant is None else 1 + int(rowpass_variant)
    op.tune_cache = tune_cache.encode() if tune_cache else None
    op.psd_guard = 1 if psd_guard else 0
    op.m2l_eps = float(m2l_eps)
    return op


def plan(problem, options):
    info = H.hikf_plan_info()
    H.check(H.hikf_plan(ctypes.byref(problem), ctypes.byref(options), ctypes.byref(info)),
            "hikf_plan")
    return info


class HikfFilter:
    """Owns the resident (and, until released, scratch) workspace of one filter."""

    def __init__(self, problem, options, keepalive=(), device="cuda", stream=None,
                 keep_scratch=False):
        self.problem, self.options = problem, options
        self.info = plan(problem, options)
        self.m = int(self.info.m)
        self.p = int(problem.p)
        self.resident = torch.empty(int(self.info.resident_bytes), dtype=torch.uint8, device=device)
        self.scratch = torch.empty(int(self.info.scratch_bytes), dtype=torch.uint8, device=device)
        self._keep = keepalive
        self.handle = ctypes.c_void_p()
        st = H.hikf_init(ctypes.byref(problem), ctypes.byref(options),
                         ctypes.c_void_p(self.resident.data_ptr()), self.info.resident_bytes,
                         ctypes.c_void_p(self.scratch.data_ptr()), self.info.scratch_bytes,
                         _stream_handle(stream), ctypes.byref(self.handle))
        H.check(st, "hikf_init")
        if stream is not None:
            # init's work is queued on `stream`: tell torch's allocator, so the
            # regions are not handed out for other streams' work before it ends
            self.scratch.record_stream(stream)
            self.resident.record_stream(stream)
        if not keep_scratch:
            # the scratch region may be reused once init's work has finished;
            # torch's allocator orders the reuse after `stream` (or the
            # current stream) has passed this point
            self.scratch = None

    def step(self, y, x_out=None, var_out=None, stream=None):
        """Queue one assimilation step with measurement y (p doubles on the device)."""
        yc = y.contiguous()
        assert yc.dtype == torch.float64 and yc.numel() == self.p and yc.is_cuda
        if stream is not None and yc is not y:
            yc.record_stream(stream)          # a temporary read on `stream`
        st = H.hikf_step(self.handle, ctypes.c_void_p(yc.data_ptr()),
                         ctypes.c_void_p(x_out.data_ptr() if x_out is not None else None),
                         ctypes.c_void_p(var_out.data_ptr() if var_out is not None else None),
                         _stream_handle(stream))
        H.check(st, "hikf_step", self.handle)

    def query(self):
        stats = H.hikf_stats()
        H.check(H.hikf_query(self.handle, ctypes.byref(stats)), "hikf_query", self.handle)
        return stats

    def export_state(self, stream=None):
        dev = self.resident.device
        x = torch.empty(self.m, dtype=torch.float64, device=dev)
        v = torch.empty(self.m, dtype=torch.float64, device=dev)
        c = torch.empty(self.m, self.p, dtype=torch.float64, device=dev)
        H.check(H.hikf_export_state(self.handle, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                    _stream_handle(stream)), "hikf_export_state", self.handle)
        return x, v, c

    def import_state(self, x=None, var=None, c=None, stream=None):
        ts = [None if t is None else t.contiguous() for t in (x, var, c)]
        if stream is not None:
            for t, orig in zip(ts, (x, var, c)):
                if t is not None and t is not orig:
                    t.record_stream(stream)   # temporaries read on `stream`
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None
               else ctypes.c_void_p(None))
        H.check(H.hikf_import_state(self.handle, ptr(ts[0]), ptr(ts[1]), ptr(ts[2]),
                                    _stream_handle(stream)), "hikf_import_state", self.handle)

    def export_checkpoint(self, stream=None):
        """(x, var, C, [G | h], info) device tensors and the checkpoint info."""
        dev = self.resident.device
        x = torch.empty(self.m, dtype=torch.float64, device=dev)
        v = torch.empty(self.m, dtype=torch.float64, device=dev)
        c = torch.empty(self.m, self.p, dtype=torch.float64, device=dev)
        ps = torch.empty(self.p * self.p + self.p, dtype=torch.float64, device=dev)
        info = H.hikf_checkpoint_info()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        H.check(H.hikf_export_checkpoint(self.handle, ptr(x), ptr(v), ptr(c), ptr(ps),
                                         ctypes.byref(info), _stream_handle(stream)),
                "hikf_export_checkpoint", self.handle)
        return x, v, c, ps, info

    def import_checkpoint(self, x, var, c, pspace, info, stream=None):
        ts = [t.contiguous() if t is not None else None for t in (x, var, c, pspace)]
        if stream is not None:
            for t, orig in zip(ts, (x, var, c, pspace)):
                if t is not None and t is not orig:
                    t.record_stream(stream)
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None
               else ctypes.c_void_p(None))
        H.check(H.hikf_import_checkpoint(self.handle, ptr(ts[0]), ptr(ts[1]), ptr(ts[2]),
                                         ptr(ts[3]), ctypes.byref(info), _stream_handle(stream)),
                "hikf_import_checkpoint", self.handle)

    def cov_apply(self, v, stream=None):
        """P_{t|t} v for the current step t (needs options.history >= t)."""
        v = v.contiguous()
        assert v.dtype == torch.float64 and v.numel() == self.m and v.is_cuda
        out = torch.empty_like(v)
        nbytes = int(self.info.query_bytes)
        scratch = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=v.device)
        H.check(H.hikf_cov_apply(self.handle, ctypes.c_void_p(v.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(scratch.data_ptr()), nbytes,
                                 _stream_handle(stream)), "hikf_cov_apply", self.handle)
        return out

    def cov_apply_noalloc(self, v, out=None, stream=None):
        """P_{t|t} v through the entry point that allocates nothing (its
        workspace is the library's fixed device array); out may be given so
        that this call allocates nothing on the torch side either."""
        assert v.dtype == torch.float64 and v.numel() == self.m and v.is_cuda and v.is_contiguous()
        if out is None:
            out = torch.empty_like(v)
        H.check(H.hikf_cov_apply_noalloc(self.handle, ctypes.c_void_p(v.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
                "hikf_cov_apply_noalloc", self.handle)
        return out

    def export_cq(self, stream=None):
        out = torch.empty(self.m, self.p, dtype=torch.float64, device=self.resident.device)
        H.check(H.hikf_export_cq(self.handle, ctypes.c_void_p(out.data_ptr()),
                                 _stream_handle(stream)), "hikf_export_cq", self.handle)
        return out

    def close(self):
        if self.handle:
            H.hikf_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(filters, ys, x_outs=None, var_outs=None, stream=None):
    """One hikf_step_batch call: step filters[i] with ys[i] (p_i doubles on the
    device each), writing x_outs[i] / var_outs[i] when given."""
    n = len(filters)
    assert len(ys) == n
    for f, y in zip(filters, ys):
        assert y.dtype == torch.float64 and y.is_cuda and y.is_contiguous() and y.numel() == f.p
    arr = ctypes.c_void_p * n

    def ptrs(ts):
        return arr(*[t.data_ptr() if t is not None else None for t in ts])

    fh = arr(*[f.handle.value for f in filters])
    st = H.hikf_step_batch(fh, ptrs(ys), ptrs(x_outs) if x_outs is not None else None,
                           ptrs(var_outs) if var_outs is not None else None, n,
                           _stream_handle(stream))
    H.check(st, "hikf_step_batch")

"""Host-side checks of the C ABI (no GPU calls).

The library must load, export every function include/hikf.h and
include/hikf_enkf.h declare, and hikf_plan / hikf_enkf_plan (host only) must
validate shapes and report the workspace they need.
"""

import ctypes
import os
import re

import pytest

import synth
from oracle import bbfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for header in ("hikf.h", "hikf_enkf.h"):
        src = open(os.path.join(ROOT, "include", header)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(hikf_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_1404_3816_amd import hikf as H
    lib = ctypes.CDLL(H.LIB_PATH)
    declared = _declared_functions()
    assert "hikf_init" in declared and "hikf_step" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(H.EXPORTED) == declared


def _problem(dim=2, n=32, p=16, nnz=100, **kw):
    from paper_1404_3816_amd import hikf as H
    pr = H.hikf_problem()
    pr.dim, pr.n, pr.p, pr.nnz = dim, n, p, nnz
    pr.kernel_family = kw.get("family", H.HIKF_KERNEL_POWEXP)
    pr.prior_kind = kw.get("prior", H.HIKF_PRIOR_KERNEL)
    pr.theta, pr.ell, pr.gamma = kw.get("theta", 1.0), kw.get("ell", 0.3), kw.get("gamma", 1.0)
    pr.alpha = kw.get("alpha", 0.0)
    fake = 256  # any non-NULL value; hikf_plan never dereferences them
    pr.h_rowptr_dev = pr.h_col_dev = pr.h_val_dev = pr.r_diag_dev = fake
    pr.x0_dev = None
    return pr


def _plan(pr, n_c=4, precision=0, direct=0, sparse=0):
    from paper_1404_3816_amd import hikf as H
    op = H.hikf_options()
    op.n_c, op.fmm_precision, op.direct, op.sparse = n_c, precision, direct, sparse
    info = H.hikf_plan_info()
    st = H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info))
    return st, info


@pytest.mark.parametrize("dim,n", [(2, 32), (2, 256), (2, 1024), (3, 128), (3, 16),
                                   (2, 33), (2, 59), (2, 1000), (3, 12), (3, 100)])
def test_plan_tree_counts_match_oracle(dim, n):
    from paper_1404_3816_amd import hikf as H
    st, info = _plan(_problem(dim=dim, n=n, p=64))
    assert st == H.HIKF_OK
    leaf = 8 if dim == 2 else 4
    near, far = bbfmm.interaction_counts(dim, n, leaf)
    assert info.near_pairs == near
    assert info.far_pairs == far
    assert info.m == n ** dim
    assert leaf << info.depth == bbfmm.padded_size(n, leaf)
    assert info.r == 4 ** dim
    # resident state holds at least C (FP64) and C_Q (FP32): 12 m p bytes
    assert info.resident_bytes >= 12 * info.m * 64


def test_plan_rejects_bad_input():
    from paper_1404_3816_amd import hikf as H
    assert _plan(_problem(dim=4))[0] == H.HIKF_E_INVALID
    assert _plan(_problem(theta=0.0))[0] == H.HIKF_E_INVALID
    assert _plan(_problem(ell=-1.0))[0] == H.HIKF_E_INVALID
    assert _plan(_problem(gamma=2.5))[0] == H.HIKF_E_INVALID
    assert _plan(_problem(), n_c=0)[0] == H.HIKF_E_INVALID
    assert _plan(_problem(), n_c=9)[0] == H.HIKF_E_INVALID
    assert _plan(_problem(), precision=7)[0] == H.HIKF_E_INVALID
    assert _plan(_problem(p=0))[0] == H.HIKF_E_INVALID
    assert _plan(_problem(nnz=-1))[0] == H.HIKF_E_INVALID
    assert _plan(_problem(prior=9))[0] == H.HIKF_E_INVALID
    pr = _problem()
    pr.h_rowptr_dev = None
    assert _plan(pr)[0] == H.HIKF_E_INVALID


def test_plan_reports_unsupported_shapes():
    from paper_1404_3816_amd import hikf as H
    assert _plan(_problem(dim=3, n=1300))[0] == H.HIKF_E_UNSUPPORTED   # 2048^3-cell tree
    assert _plan(_problem(p=20))[0] == H.HIKF_E_UNSUPPORTED      # not a multiple of 16
    assert _plan(_problem(p=528))[0] == H.HIKF_E_UNSUPPORTED     # above 512
    assert _plan(_problem(dim=3, n=16), n_c=6)[0] == H.HIKF_E_UNSUPPORTED  # r = 216 > 64


def test_plan_direct_mode_has_no_far_field():
    from paper_1404_3816_amd import hikf as H
    st, info = _plan(_problem(n=32), direct=1)
    assert st == H.HIKF_OK
    assert info.far_pairs == 0
    assert info.near_pairs == 16 * 16


def test_status_strings():
    from paper_1404_3816_amd import hikf as H
    for s in range(6):
        assert H.hikf_status_string(s)
    assert H.hikf_last_error(None) == b""


def test_ray_operator_fits_abi_layout():
    rp, col, val = synth.crosswell_h(2, 32, 16)
    assert rp.dtype.name == "int64" and col.dtype.name == "int32" and val.dtype.name == "float64"


def test_step_batch_rejects_bad_arguments_without_a_device():
    # argument checks happen before any device call
    from paper_1404_3816_amd import hikf as H
    assert H.hikf_step_batch(None, None, None, None, -1, None) == H.HIKF_E_INVALID
    assert H.hikf_step_batch(None, None, None, None, 0, None) == H.HIKF_OK
    arr = ctypes.c_void_p * 2
    assert H.hikf_step_batch(arr(None, None), arr(None, None), None, None, 2,
                             None) == H.HIKF_E_INVALID
    # the same filter twice (the handles are never dereferenced: the check
    # comes first)
    fake, y = 4096, 8192
    assert H.hikf_step_batch(arr(fake, fake), arr(y, y), None, None, 2,
                             None) == H.HIKF_E_INVALID


def test_plan_bf16_modes_add_split_operands():
    # BF16 modes keep FP32 storage and add hi/lo copies of W, M and the M2L tables
    from paper_1404_3816_amd import hikf as H
    st32, i32 = _plan(_problem(dim=3, n=32, p=64), precision=H.HIKF_FMM_F32)
    st3, i3 = _plan(_problem(dim=3, n=32, p=64), precision=H.HIKF_FMM_BF16X3)
    st1, i1 = _plan(_problem(dim=3, n=32, p=64), precision=H.HIKF_FMM_BF16)
    assert st32 == st3 == st1 == H.HIKF_OK
    assert i3.resident_bytes == i32.resident_bytes == i1.resident_bytes
    assert i3.scratch_bytes == i1.scratch_bytes > i32.scratch_bytes
    # W split: 2 copies x 2 bytes per entry of the m x p matrix
    assert i3.scratch_bytes - i32.scratch_bytes >= 2 * 2 * 32 ** 3 * 64


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_plan_sparse_mode_drops_dense_w(precision):
    # the sparse mode keeps the nonzeros by leaf (a few words per nonzero and
    # per leaf) instead of the dense W over the tree's cells (and, in the BF16
    # modes, its hi / lo copies); the resident state is the same
    from paper_1404_3816_amd import hikf as H
    pr = _problem(dim=2, n=1000, p=256)
    st_d, i_d = _plan(pr, precision=precision)
    st_s, i_s = _plan(pr, precision=precision, sparse=1)
    assert st_d == st_s == H.HIKF_OK
    assert i_s.resident_bytes == i_d.resident_bytes
    word = 8 if precision == H.HIKF_FMM_F64 else 4
    dense_w = 1024 * 1024 * 256 * word + (1024 * 1024 * 256 * 4 if precision == 2 else 0)
    bucket = 128 * 128 * 8 + pr.nnz * (8 + word) + 4096
    assert i_d.scratch_bytes - i_s.scratch_bytes >= dense_w - bucket
    # direct mode has no tree lists to bucket by: the option is ignored
    st_x, i_x = _plan(_problem(dim=2, n=64, p=32), direct=1, sparse=1)
    st_y, i_y = _plan(_problem(dim=2, n=64, p=32), direct=1)
    assert st_x == st_y == H.HIKF_OK and i_x.scratch_bytes == i_y.scratch_bytes


def test_plan_query_bytes_only_with_history():
    from paper_1404_3816_amd import hikf as H
    pr = _problem(dim=2, n=64, p=32)
    op = H.hikf_options()
    op.n_c, op.fmm_precision, op.history = 4, H.HIKF_FMM_F32, 0
    info = H.hikf_plan_info()
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    base, q0 = info.resident_bytes, info.query_bytes
    op.history = 5
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    assert q0 == 0 and info.query_bytes > 64 * 64 * 16 * 4
    # the history holds C_prior (m p doubles) and S^-1 (p^2 doubles) per step
    assert info.resident_bytes - base >= 5 * (64 * 64 * 32 + 32 * 32) * 8
    op.history = -1
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_E_INVALID
    assert H.hikf_cov_apply(None, None, None, None, 0, None) == H.HIKF_E_INVALID


def test_plan_rowpass_variant_range():
    from paper_1404_3816_amd import hikf as H
    pr = _problem(dim=2, n=64, p=32)
    op = H.hikf_options()
    op.n_c, op.fmm_precision = 4, H.HIKF_FMM_F32
    info = H.hikf_plan_info()
    for v in range(9):
        op.rowpass_variant = v
        assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    for v in (-1, 9):
        op.rowpass_variant = v
        assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op),
                           ctypes.byref(info)) == H.HIKF_E_INVALID


def test_plan_reads_tuning_cache(tmp_path):
    # the tuning cache entry with the same p and C_Q type and the nearest m
    # chooses the variant; a forced variant wins; no match -> default 0
    import json
    from paper_1404_3816_amd import hikf as H
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({"device": "x", "rowpass": [
        {"p": 32, "cq": "f32", "m": 4096, "variant": 3, "ms": [1, 1, 1, 0.5]},
        {"p": 32, "cq": "f32", "m": 10 ** 6, "variant": 1, "ms": [1, 0.5, 1, 1]},
        {"p": 32, "cq": "f64", "m": 4096, "variant": 2, "ms": [1, 1, 0.5, None]},
        {"p": 64, "cq": "f32", "m": 4096, "variant": 1, "ms": [1, 0.5, 1, 1]}]}, indent=1))

    def variant(n, p, prec, forced=0, path=str(cache)):
        pr = _problem(dim=2, n=n, p=p)
        op = H.hikf_options()
        op.n_c, op.fmm_precision, op.rowpass_variant = 4, prec, forced
        op.tune_cache = path.encode() if path else None
        info = H.hikf_plan_info()
        assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
        return info.rowpass_variant

    assert variant(64, 32, H.HIKF_FMM_F32) == 3           # m = 4096
    assert variant(1024, 32, H.HIKF_FMM_F32) == 1         # m = 1M: nearest entry
    assert variant(64, 32, H.HIKF_FMM_F64) == 2
    assert variant(64, 64, H.HIKF_FMM_F32) == 1
    assert variant(64, 48, H.HIKF_FMM_F32) == 0           # no entry for p = 48
    assert variant(64, 32, H.HIKF_FMM_F32, forced=3) == 2  # forced variant 2
    assert variant(64, 32, H.HIKF_FMM_F32, path=None) == 0
    assert variant(64, 32, H.HIKF_FMM_F32, path=str(tmp_path / "missing.json")) == 0


def test_checkpoint_calls_check_arguments_without_a_device():
    from paper_1404_3816_amd import hikf as H
    info = H.hikf_checkpoint_info()
    assert H.hikf_export_checkpoint(None, None, None, None, None, ctypes.byref(info),
                                    None) == H.HIKF_E_INVALID
    assert H.hikf_import_checkpoint(None, None, None, None, None, ctypes.byref(info),
                                    None) == H.HIKF_E_INVALID
    assert H.hikf_export_checkpoint(4096, None, None, None, None, None, None) == H.HIKF_E_INVALID
    assert H.hikf_import_checkpoint(4096, None, None, None, None, None, None) == H.HIKF_E_INVALID


def test_plan_psd_guard_flag():
    from paper_1404_3816_amd import hikf as H
    pr = _problem(dim=2, n=64, p=32)
    op = H.hikf_options()
    op.n_c, op.fmm_precision = 4, H.HIKF_FMM_F64
    info = H.hikf_plan_info()
    op.psd_guard = 0
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    base = info.scratch_bytes
    op.psd_guard = 1
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    assert info.scratch_bytes >= base + 3 * 32 * 32 * 8      # three p x p work matrices
    op.psd_guard = 2
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_E_INVALID


def test_plan_lowrank_m2l_threshold():
    from paper_1404_3816_amd import hikf as H
    pr = _problem(dim=2, n=256, p=32)
    op = H.hikf_options()
    op.n_c, op.fmm_precision = 5, H.HIKF_FMM_F32
    info = H.hikf_plan_info()
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    base = info.scratch_bytes
    op.m2l_eps = 1e-5
    assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op), ctypes.byref(info)) == H.HIKF_OK
    # compressed M and L of the finest level: 2 x 1024 leaves x 25 nodes x 32 columns
    assert info.scratch_bytes >= base + 2 * 1024 * 25 * 32 * 4
    for bad in (-1e-3, 1.0, float("nan")):
        op.m2l_eps = bad
        assert H.hikf_plan(ctypes.byref(pr), ctypes.byref(op),
                           ctypes.byref(info)) == H.HIKF_E_INVALID


def _enkf_problem(m=1000, p=32, n_ens=40, nnz=500):
    from paper_1404_3816_amd import hikf as H
    pr = H.hikf_enkf_problem()
    pr.m, pr.p, pr.n_ens, pr.nnz = m, p, n_ens, nnz
    fake = 256  # never dereferenced by the plan
    pr.h_rowptr_dev = pr.h_col_dev = pr.h_val_dev = pr.r_diag_dev = fake
    return pr


@pytest.mark.parametrize("n_ens,ld", [(2, 16), (16, 16), (17, 32), (40, 48), (81, 96), (100, 128),
                                      (400, 400), (401, 448), (512, 512)])
def test_enkf_plan_pads_the_ensemble_to_a_tile_width(n_ens, ld):
    from paper_1404_3816_amd import hikf as H
    info = H.hikf_enkf_plan_info()
    pr = _enkf_problem(n_ens=n_ens)
    assert H.hikf_enkf_plan(ctypes.byref(pr), ctypes.byref(info)) == H.HIKF_OK
    assert info.ld == ld
    # the ensemble alone: m rows of ld doubles
    assert info.resident_bytes >= pr.m * ld * 8


@pytest.mark.parametrize("field,value,code", [("n_ens", 1, 1), ("n_ens", 513, 2), ("p", 0, 1),
                                              ("p", 513, 2), ("m", 0, 1), ("nnz", -1, 1)])
def test_enkf_plan_rejects_bad_shapes(field, value, code):
    from paper_1404_3816_amd import hikf as H
    pr = _enkf_problem()
    setattr(pr, field, value)
    info = H.hikf_enkf_plan_info()
    assert H.hikf_enkf_plan(ctypes.byref(pr), ctypes.byref(info)) == code


def test_enkf_plan_rejects_null_arrays():
    from paper_1404_3816_amd import hikf as H
    pr = _enkf_problem()
    pr.r_diag_dev = None
    info = H.hikf_enkf_plan_info()
    assert H.hikf_enkf_plan(ctypes.byref(pr), ctypes.byref(info)) == H.HIKF_E_INVALID
    assert H.hikf_enkf_step(None, None, None, None, None, None, None) == H.HIKF_E_INVALID

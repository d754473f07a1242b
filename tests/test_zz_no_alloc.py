"""hikf_cov_apply_noalloc (the covariance query whose workspace is the
library's fixed device array) against hikf_cov_apply (caller workspace) on
the same filters: two calls in a row, the second on a smaller filter, so the
second query runs in an array the first one filled with larger data.  Both
entry points run the same kernels, so the outputs must agree bit for bit."""

import numpy as np
import pytest

from helpers import Case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_3816_amd import hikf  # noqa: F401  (fails loudly without libhikf.so)


def _stepped_filter(case, precision, steps):
    import torch
    from paper_1404_3816_amd import filter as F
    pr, keep = F.problem_from_csr(case.dim, case.n, case.rowptr, case.col, case.val,
                                  case.r_diag, **case.kparams())
    f = F.HikfFilter(pr, F.make_options(4, precision, False, history=8), keep)
    y = torch.as_tensor(case.ys, device="cuda")
    for k in range(steps):
        f.step(y[k])
    return f


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_query_matches_workspace_query(precision):
    import torch
    big = Case(2, 128, 64, ell=0.1, steps=3)
    small = Case(2, 32, 16, ell=0.3, steps=2)
    fb = _stepped_filter(big, precision, 3)
    fs = _stepped_filter(small, precision, 2)
    assert fb.info.query_bytes > fs.info.query_bytes
    vb = torch.as_tensor(np.random.default_rng(1).standard_normal(big.m), device="cuda")
    vs = torch.as_tensor(np.random.default_rng(2).standard_normal(small.m), device="cuda")
    ref_b = fb.cov_apply(vb)
    ref_s = fs.cov_apply(vs)
    out_b = torch.full_like(vb, float("nan"))
    out_s = torch.full_like(vs, float("nan"))
    got_b = fb.cov_apply_noalloc(vb, out_b)            # first: the larger query
    got_s = fs.cov_apply_noalloc(vs, out_s)            # then a smaller one
    torch.cuda.synchronize()
    assert torch.isfinite(got_b).all() and torch.isfinite(got_s).all()
    assert torch.equal(got_b, ref_b)
    assert torch.equal(got_s, ref_s)
    # a repeated small query after the large one still matches
    assert torch.equal(fs.cov_apply_noalloc(vs), ref_s)
    fb.close()
    fs.close()


def test_noalloc_query_rejects_oversized_workspace():
    import torch
    from paper_1404_3816_amd import hikf as H
    case = Case(2, 512, 64, ell=0.1, steps=1)
    f = _stepped_filter(case, "f32", 0)
    assert f.info.query_bytes > H.HIKF_NOALLOC_SCRATCH_BYTES
    v = torch.zeros(case.m, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HikfError) as err:
        f.cov_apply_noalloc(v)
    assert err.value.status == H.HIKF_E_NOMEM
    f.close()

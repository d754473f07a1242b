"""GPU tests of the runtime around the step: the captured step graph, the
grouped step of the serving loop, and the negative-variance counter.  All
go through the C ABI; results are compared bitwise with plain hikf_step
calls, whose parity with the oracle is covered in test_gpu_parity.py."""

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


def _filter(case, graph=False, n_c=4, precision="f32", riccati=0):
    from paper_1404_3816_amd import filter as F
    pr, keep = F.problem_from_csr(case.dim, case.n, case.rowptr, case.col, case.val,
                                  case.r_diag, **case.kparams())
    return F.HikfFilter(pr, F.make_options(n_c, precision, False, graph=graph, riccati=riccati),
                        keep)


@pytest.mark.parametrize("dim,n,p", [(2, 64, 32), (3, 16, 64)])
def test_graph_replays_match_eager(dim, n, p):
    # every replay is compared with the eager step, with unrelated eager work
    # and a synchronisation between replays
    import torch
    case = Case(dim, n, p, ell=0.2, steps=5, planes=2)
    y = torch.as_tensor(case.ys, device="cuda")
    fe, fg = _filter(case), _filter(case, graph=True)
    xe = torch.empty(case.m, dtype=torch.float64, device="cuda")
    ve, xg, vg = torch.empty_like(xe), torch.empty_like(xe), torch.empty_like(xe)
    junk = torch.randn(1 << 20, device="cuda")
    for k in range(case.steps):
        fe.step(y[k], xe, ve)
        fg.step(y[k], xg, vg)
        junk = (junk * 1.0001).sin_()
        torch.cuda.synchronize()
        assert torch.equal(xe, xg) and torch.equal(ve, vg), k
    se, sg = fe.query(), fg.query()
    assert sg.steps_applied == se.steps_applied == case.steps
    assert sg.last_status == 0 and sg.min_pivot == se.min_pivot
    ce, cg = fe.export_state()[2], fg.export_state()[2]
    assert torch.equal(ce, cg)
    fe.close()
    fg.close()


def test_graph_failed_step_is_transactional():
    # a NaN measurement through the graph leaves the state as it was
    import torch
    case = Case(2, 32, 16, ell=0.3, steps=2)
    f = _filter(case, graph=True)
    y = torch.as_tensor(case.ys, device="cuda")
    f.step(y[0])
    x0, v0, c0 = f.export_state()
    bad = y[1].clone()
    bad[3] = float("nan")
    f.step(bad)
    x1, v1, c1 = f.export_state()
    st = f.query()
    f.close()
    assert st.last_status == 1 and st.steps_applied == 1
    assert torch.equal(x0, x1) and torch.equal(v0, v1) and torch.equal(c0, c1)


def test_step_batch_matches_solo_steps():
    import torch
    from paper_1404_3816_amd import filter as F
    cases = [Case(2, 32, 16, ell=0.3, steps=3), Case(2, 64, 48, ell=0.1, steps=3),
             Case(3, 16, 32, ell=0.2, steps=3)]
    solo = [_filter(c) for c in cases]
    grouped = [_filter(c, graph=(i == 1)) for i, c in enumerate(cases)]
    ys = [torch.as_tensor(c.ys, device="cuda") for c in cases]
    for k in range(3):
        xs = [torch.empty(c.m, dtype=torch.float64, device="cuda") for c in cases]
        vs = [torch.empty_like(x) for x in xs]
        F.step_batch(grouped, [y[k].contiguous() for y in ys], xs, [vs[0], None, vs[2]])
        for i, f in enumerate(solo):
            xo = torch.empty_like(xs[i])
            vo = torch.empty_like(xs[i])
            f.step(ys[i][k], xo, vo)
            torch.cuda.synchronize()
            assert torch.equal(xo, xs[i]), (i, k)
            if i != 1:
                assert torch.equal(vo, vs[i]), (i, k)
    for f, g in zip(solo, grouped):
        assert torch.equal(f.export_state()[2], g.export_state()[2])
        assert g.query().steps_applied == 3
        f.close()
        g.close()


def test_negative_variance_counter():
    import torch
    case = Case(2, 32, 16, ell=0.3, steps=2)
    f = _filter(case, precision="f64")
    y = torch.as_tensor(case.ys, device="cuda")
    f.step(y[0])
    assert f.query().negative_variances == 0
    # a checkpoint whose variances are -10 everywhere: one step adds
    # K(0) = 1 and subtracts a non-negative term, so every entry stays negative
    x, v, c = f.export_state()
    f.import_state(x, torch.full_like(v, -10.0), c)
    f.step(y[1])
    st = f.query()
    _, v2, _ = f.export_state()
    f.close()
    assert int((v2 < 0).sum()) == case.m
    assert st.negative_variances == case.m


def _trajectory(f, y, m, steps):
    import torch
    x = torch.empty(m, dtype=torch.float64, device="cuda")
    v = torch.empty_like(x)
    xs, vs = [], []
    for k in range(steps):
        f.step(y[k], x, v)
        xs.append(x.cpu().numpy().copy())
        vs.append(v.cpu().numpy().copy())
    return np.array(xs), np.array(vs)


@pytest.mark.parametrize("riccati,graph", [(1, False), (4, False), (1000, False), (4, True)])
def test_riccati_recursion_matches_gather(riccati, graph):
    # G <- G S^-1 R + H C_Q and h <- h + G S^-1 nu are exact identities of the
    # update; carried over many steps they drift only by rounding
    import torch
    from helpers import max_step_rel
    case = Case(2, 64, 32, ell=0.2, steps=12)
    y = torch.as_tensor(case.ys, device="cuda")
    fa, fb = _filter(case, precision="f64"), _filter(case, precision="f64", riccati=riccati,
                                                     graph=graph)
    xa, va = _trajectory(fa, y, case.m, case.steps)
    xb, vb = _trajectory(fb, y, case.m, case.steps)
    sa, sb = fa.query(), fb.query()
    fa.close()
    fb.close()
    assert sb.last_status == 0 and sb.steps_applied == case.steps
    assert max_step_rel(xb, xa) < 1e-9
    assert max_step_rel(vb, va) < 1e-10


def test_riccati_import_forces_a_gather():
    # after import_state the carried G, h would describe the old state: the
    # next step must form them from C again
    import torch
    case = Case(2, 32, 16, ell=0.3, steps=4)
    y = torch.as_tensor(case.ys, device="cuda")
    fa, fb = _filter(case, precision="f64"), _filter(case, precision="f64", riccati=1000)
    for k in range(2):
        fa.step(y[k])
    fb.step(y[0])
    x, v, c = fa.export_state()
    fb.import_state(x, v, c)                 # fb jumps to fa's state after 2 steps
    fa.step(y[2])
    fb.step(y[2])
    xa, va, ca = fa.export_state()
    xb, vb, cb = fb.export_state()
    fa.close()
    fb.close()
    assert float(((xb - xa).norm() / xa.norm())) < 1e-12
    assert float(((vb - va).norm() / va.norm())) < 1e-12


@pytest.mark.parametrize("p", [64, 96, 256, 512])
def test_rowpass_variants_agree(p):
    # every launch form of the row pass: K, hence C_post, is summed in the
    # same order in all of them (bitwise equal); x_hat and the variance add
    # the column parts' dot products in two or four groups (rounding only);
    # a persistent form equals its one-tile-per-workgroup twin bitwise
    import torch
    from paper_1404_3816_amd import filter as F
    case = Case(2, 96, p, ell=0.2, steps=3)
    y = torch.as_tensor(case.ys, device="cuda")
    out = {}
    for v in range(8):
        pr, keep = F.problem_from_csr(2, case.n, case.rowptr, case.col, case.val, case.r_diag,
                                      **case.kparams())
        f = F.HikfFilter(pr, F.make_options(4, "f64", False, rowpass_variant=v,
                                            graph=(v % 2 == 1)), keep)
        for k in range(case.steps):
            f.step(y[k])
        st = f.query()
        assert st.last_status == 0 and st.steps_applied == case.steps
        assert st.rowpass_variant == v
        out[v] = f.export_state()
        f.close()
    x0, v0, c0 = out[0]
    for v in range(1, 8):
        x, var, c = out[v]
        assert torch.equal(c, c0), v
        assert torch.allclose(x, x0, rtol=1e-12, atol=1e-14 * x0.abs().max().item()), v
        assert torch.allclose(var, v0, rtol=1e-12, atol=1e-14), v
    for v in range(8):
        assert all(torch.equal(a, b) for a, b in zip(out[v], out[v ^ 1])), v


def test_tune_cache_is_read_by_init(tmp_path):
    # hikf_init takes the row-pass variant from the tuning cache entry with
    # the same p and C_Q type and the nearest m
    import json
    import torch
    from paper_1404_3816_amd import filter as F
    case = Case(2, 64, 32, ell=0.2, steps=1)
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({"device": "x", "rowpass": [
        {"p": 32, "cq": "f32", "m": 4096, "variant": 3, "ms": [1, 1, 1, 0.5]},
        {"p": 32, "cq": "f32", "m": 10 ** 6, "variant": 1, "ms": [1, 0.5, 1, 1]},
        {"p": 32, "cq": "f64", "m": 4096, "variant": 2, "ms": [1, 1, 0.5, 1]},
        {"p": 64, "cq": "f32", "m": 4096, "variant": 1, "ms": [1, 0.5, 1, 1]}]}))
    got = {}
    for prec in ("f32", "f64"):
        pr, keep = F.problem_from_csr(2, case.n, case.rowptr, case.col, case.val, case.r_diag,
                                      **case.kparams())
        f = F.HikfFilter(pr, F.make_options(4, prec, False, tune_cache=str(cache)), keep)
        f.step(torch.as_tensor(case.ys[0], device="cuda"))
        got[prec] = f.query().rowpass_variant
        f.close()
    assert got == {"f32": 3, "f64": 2}
    # no cache, or a cache without a matching entry: the built-in default (0)
    pr, keep = F.problem_from_csr(2, case.n, case.rowptr, case.col, case.val, case.r_diag,
                                  **case.kparams())
    f = F.HikfFilter(pr, F.make_options(4, "f32", False, tune_cache=str(tmp_path / "none")),
                     keep)
    assert f.query().rowpass_variant == 0
    f.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("riccati", [1, 3])
def test_recursion_matches_oracle_and_reports_drift(precision, riccati):
    # G and h carried by the exact p-space recursion between gathers (period
    # `riccati`): the filter still matches the oracle's literal cross-
    # covariance filter on the same C_Q (the oracle's FP64 bbFMM product, so
    # FP32 mode is held to its C_Q bound times the sensitivity ceiling), and
    # every gather after the first measures the drift of the carried values,
    # which is rounding only
    from helpers import CQ_TOL, KAPPA, max_step_rel, rel
    case = Case(2, 64, 32, ell=0.1, gamma=2.0, steps=4)
    cq, xs, vs, stats = case.gpu_run(n_c=5, precision=precision, riccati=riccati)
    ref = case.cq_bbfmm(5)
    xb, vb = case.tier_b(ref)
    ex, ev = max_step_rel(xs, xb), max_step_rel(vs, vb)
    print(f"recursion period {riccati} ({precision}): x {ex:.3e} var {ev:.3e}, drift "
          f"G {stats.riccati_drift_g:.3e} h {stats.riccati_drift_h:.3e} "
          f"over {stats.riccati_checks} checks")
    assert stats.last_status == 0 and stats.steps_applied == case.steps
    assert stats.riccati_checks == (case.steps - 1) // riccati
    assert stats.riccati_drift_g < 1e-10 and stats.riccati_drift_h < 1e-10
    if precision == "f64":
        assert ex < 1e-9 and ev < 1e-10
    else:
        kx, kv = KAPPA[("fmm", 64, 32, 5)]
        assert rel(cq, ref) < CQ_TOL["f32"]
        assert ex < kx * CQ_TOL["f32"] and ev < kv * CQ_TOL["f32"]


def test_recursion_drift_is_not_checked_after_import():
    # an imported state has nothing carried: the next gather is no check
    import torch
    case = Case(2, 64, 32, ell=0.1, steps=4)
    f = _filter(case, riccati=2)
    y = torch.as_tensor(case.ys, device="cuda")
    f.step(y[0])
    f.step(y[1])
    x, v, c = f.export_state()
    f.import_state(x, v, c)
    f.step(y[2])                          # forced gather: no check
    st = f.query()
    assert st.riccati_checks == 0 and st.steps_applied == 3
    f.step(y[3])                          # carried, not gathered (period 2)
    assert f.query().riccati_checks == 0
    f.close()

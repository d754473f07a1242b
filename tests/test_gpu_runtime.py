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

"""Serving on the GPU: every result in the concurrent mix equals the same
request run alone (bitwise), every result states its error against FP64, and
the results are checked against the oracle: the first requests, every
Pfaffian labelled FP32, and every solve by its backward error."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import serve
    return serve.GpuExecutor("cuda:0")


@pytest.mark.parametrize("count,nmax", [(64, 1024), (96, 4096)])
def test_serve_alone_equals_mix(ex, oracle_mod, count, nmax):
    """The serving mix (Pfaffian and solve jobs, FP64 and FP32 labels, a quarter
    reusing an earlier matrix) with n log-uniform up to 1024 and up to 4096,
    the order range of the serving workload."""
    import torch
    from paper_2408_05238_amd import serve
    reqs, mids = serve.make_workload(count, rate_hz=0.0, seed=8, nmin=64, nmax=nmax)
    serve.materialize(reqs, mids, seed=8)
    print(f"serve mix count={count} nmax={nmax}", flush=True)
    sch = serve.Scheduler(ex, budget_bytes=64 << 30, workers=4)
    mix = sch.run_trace(reqs)
    st = sch.stats(min(r.arrival for r in reqs))
    assert st["completed"] == len(reqs) and st["batched"] > 0 and st["cache_hits"] > 0
    assert st["errors_stated"] == len(reqs)
    assert sch.reserved == 0 and sch.tokens_used == 0
    for r in reqs:
        alone = ex.run([r], None)[0][0]
        m = mix[r.rid]
        assert m.info == alone.info == 0, (r, m.info, alone.info)
        assert m.err_kind == ("berr" if r.kind == "solve" else "logpf_rel_bound")
        if r.kind == "pf":
            assert (m.logabs, m.sign) == (alone.logabs, alone.sign), r
        else:
            assert torch.equal(m.X, alone.X), r
            assert m.iters == alone.iters and m.berr == alone.berr == m.err
            assert m.err <= 1e-13
    checked = 0
    for i, r in enumerate(reqs):
        if r.kind == "solve":
            if r.n > 2048 and i >= 24:
                continue
            A = r.A.cpu().numpy()
            X = mix[r.rid].X.cpu().numpy()
            assert oracle_mod.backward_error(A, X, r.B.cpu().numpy()) <= 1e-13
        elif i < 24 or r.prec == "f32":
            A = r.A.cpu().numpy()
            la, sg, _ = oracle_mod.logpf(A, nthreads=8)
            m = mix[r.rid]
            assert m.sign == sg and oracle_mod.isclose_log(m.logabs, la) <= m.err, (r, m.logabs, la)
            checked += 1
    assert checked > 0


def test_serve_ratio_requests(ex, oracle_mod):
    """Pfaffian ratios through the serving loop: served from the resident FP64
    factors of a matrix an earlier solve factored (cache hits), or factoring a
    new one; each against the oracle's quotient of two Pfaffians within the
    conditioning bound of the ratio tests, with its stated error bound."""
    from test_gpu_ratio import ratio_tol

    from paper_2408_05238_amd import serve
    R = serve.Request
    reqs = [R(rid=0, kind="solve", n=1000, prec="f64", matrix_id=0, arrival=0.0, nrhs=2),
            R(rid=1, kind="ratio", n=1000, prec="f64", matrix_id=0, arrival=0.0, r=3),
            R(rid=2, kind="ratio", n=1000, prec="f32", matrix_id=0, arrival=0.0, r=1),
            R(rid=3, kind="ratio", n=600, prec="f64", matrix_id=1, arrival=0.0, r=5)]
    serve.materialize(reqs, [(0, 1000), (1, 600)], seed=8)
    sch = serve.Scheduler(ex, budget_bytes=16 << 30, workers=1)
    res = sch.run_trace(reqs)
    assert res[0].info == 0 and not res[0].cached
    assert res[1].cached and res[2].cached and not res[3].cached
    for q in reqs[1:]:
        m = res[q.rid]
        A, U, V = q.A.cpu().numpy(), q.U.cpu().numpy(), q.V.cpu().numpy()
        la_r, s_r, info_r = oracle_mod.pf_ratio(A, U, V, nthreads=8)
        tol = ratio_tol(oracle_mod.full_from_lower(A), U, V, la_r)
        print(f"ratio n={q.n} r={q.r}: {m.logabs!r} vs {la_r!r}, stated {m.err:.3e}, bound {tol:.3e}", flush=True)
        assert m.info == info_r == 0 and m.sign == s_r
        assert abs(m.logabs - la_r) <= tol
        assert m.err_kind == "log_ratio_bound" and 0.0 < m.err < 1e-8

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

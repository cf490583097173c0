"""Serving on the GPU: every result in the concurrent mix equals the same
request run alone (bitwise), and a subset matches the oracle."""
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


def test_serve_alone_equals_mix(ex, oracle_mod):
    import torch
    from paper_2408_05238_amd import serve
    reqs, mids = serve.make_workload(64, rate_hz=0.0, seed=8, nmin=64, nmax=1024)
    serve.materialize(reqs, mids, seed=8)
    sch = serve.Scheduler(ex, budget_bytes=64 << 30, workers=4)
    mix = sch.run_trace(reqs)
    st = sch.stats(min(r.arrival for r in reqs))
    assert st["completed"] == len(reqs) and st["batched"] > 0 and st["cache_hits"] > 0
    assert sch.reserved == 0 and sch.tokens_used == 0
    for r in reqs:
        alone = ex.run([r], None)[0][0]
        m = mix[r.rid]
        assert m.info == alone.info == 0, (r, m.info, alone.info)
        if r.kind == "pf":
            assert (m.logabs, m.sign) == (alone.logabs, alone.sign), r
        else:
            assert torch.equal(m.X, alone.X), r
            if r.prec == "f32":
                assert m.iters == alone.iters and m.berr == alone.berr
    # a subset against the oracle
    for r in reqs[:24]:
        A = r.A.cpu().numpy()
        if r.kind == "pf":
            la, sg, _ = oracle_mod.logpf(A)
            assert mix[r.rid].sign == sg and oracle_mod.isclose_log(mix[r.rid].logabs, la) <= 1e-12
        else:
            X = mix[r.rid].X.cpu().numpy()
            assert oracle_mod.backward_error(A, X, r.B.cpu().numpy()) <= 1e-13

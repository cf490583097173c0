"""Serving scheduler logic on the CPU: a fake executor that sleeps a modelled time
and records what ran concurrently."""
from __future__ import annotations

import threading
import time

import pytest

from paper_2408_05238_amd import serve


class FakeExecutor:
    def __init__(self, num_cus=256, scale=2e-10, ws=lambda n: 8 * n * n):
        self.num_cus = num_cus
        self.scale = scale
        self._ws = ws
        self.lock = threading.Lock()
        self.tok = 0
        self.max_tok = 0
        self.calls = []
        self.running = 0
        self.max_running = 0

    def ltlt_ws(self, n, prec):
        return self._ws(n)

    def solve_ws(self, n, nrhs):
        return 8 * n * nrhs

    def refine_ws(self, n, nrhs):
        return 8 * n * nrhs * 4

    def ratio_ws(self, n, r):
        return 8 * n * 2 * r * 2

    def run(self, reqs, factors):
        tk = sum(serve.tokens(r, factors is not None) for r in reqs)
        with self.lock:
            self.tok += tk
            self.max_tok = max(self.max_tok, self.tok)
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.calls.append(([r.rid for r in reqs], factors is not None))
        work = sum(0 if factors is not None else r.n ** 3 / 3 for r in reqs)
        time.sleep(min(0.02, 1e-4 + work * self.scale))
        out = []
        for r in reqs:
            # deterministic per-matrix "result"
            out.append(serve.Result(r.rid, r.arrival, logabs=float(r.matrix_id * 1000 + r.n), sign=1,
                                    cached=factors is not None, batched=len(reqs) > 1))
        with self.lock:
            self.tok -= tk
            self.running -= 1
        new = None if (factors is not None or len(reqs) > 1 or (reqs[0].kind == "pf" and reqs[0].n <= 512)) \
            else ("factors", reqs[0].matrix_id)
        return out, new


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serve.percentile(v, 50) == 50 and serve.percentile(v, 99) == 99 and serve.percentile(v, 100) == 100
    assert serve.percentile([3.0], 99) == 3.0


def test_workload_recipe():
    reqs, mids = serve.make_workload(2000, rate_hz=100.0, seed=8)
    again, _ = serve.make_workload(2000, rate_hz=100.0, seed=8)
    assert [(r.n, r.kind, r.prec, r.matrix_id, r.arrival) for r in reqs] == \
        [(r.n, r.kind, r.prec, r.matrix_id, r.arrival) for r in again]
    ns = [r.n for r in reqs]
    assert all(n % 2 == 0 and 64 <= n <= 4096 for n in ns)
    f32 = sum(r.prec == "f32" for r in reqs) / len(reqs)
    solves = sum(r.kind == "solve" for r in reqs) / len(reqs)
    assert 0.26 < f32 < 0.34 and 0.45 < solves < 0.55
    # log-uniform: about half the draws below the geometric mean sqrt(64*4096) = 512
    fresh = [n for _, n in mids]
    assert 0.45 < sum(n < 512 for n in fresh) / len(fresh) < 0.55
    # Poisson: mean gap 1/rate
    gaps = [b.arrival - a.arrival for a, b in zip(reqs, reqs[1:])]
    assert abs(sum(gaps) / len(gaps) - 0.01) < 0.001
    assert len(mids) < len(reqs)           # some requests reuse a matrix


def test_scheduler_completes_and_respects_limits():
    reqs, _ = serve.make_workload(300, rate_hz=3000.0, seed=8, nmax=2048)
    ex = FakeExecutor(num_cus=64)
    budget = 1 << 30
    sch = serve.Scheduler(ex, budget_bytes=budget, workers=6)
    t0 = time.perf_counter()
    res = sch.run_trace(reqs, t0=t0)
    st = sch.stats(t0)
    assert st["completed"] == 300 and st["rejected"] == 0
    assert sch.high_water <= budget
    assert ex.max_tok <= 64
    assert ex.max_running > 1                       # work overlapped
    assert sch.reserved == 0 and sch.tokens_used == 0 and not sch.cache.pins
    for r in reqs:
        assert res[r.rid].logabs == r.matrix_id * 1000 + r.n and res[r.rid].end >= r.arrival
    assert st["batched"] > 0 and st["cache_hits"] > 0
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_scheduler_rejects_oversized_and_evicts():
    ex = FakeExecutor()
    budget = 3 * serve.factor_bytes(1000) + 3 * 8 * 1000 * 1000
    sch = serve.Scheduler(ex, budget_bytes=budget, workers=2)
    reqs = [serve.Request(rid=i, kind="solve", n=1000, prec="f64", matrix_id=i, arrival=0.0) for i in range(5)]
    reqs.append(serve.Request(rid=5, kind="pf", n=4000, prec="f64", matrix_id=99, arrival=0.0))
    res = sch.run_trace(reqs)
    assert res[5].info == -100 and sch.rejected == 1
    assert all(res[i].info == 0 for i in range(5))
    assert sch.evictions >= 1 and sch.high_water <= budget and sch.cache.bytes <= budget


def test_tokens_limit_serialises_large_factorizations():
    ex = FakeExecutor(num_cus=40)
    sch = serve.Scheduler(ex, budget_bytes=1 << 40, workers=4)
    reqs = [serve.Request(rid=i, kind="pf", n=2048, prec="f64", matrix_id=i, arrival=0.0) for i in range(4)]
    sch.run_trace(reqs)
    assert ex.max_tok <= 40 and ex.max_running == 1      # 32 tokens each: never two at once


def test_cached_factors_skip_factorization():
    ex = FakeExecutor()
    sch = serve.Scheduler(ex, budget_bytes=1 << 40, workers=1)
    reqs = [serve.Request(rid=0, kind="solve", n=1000, prec="f64", matrix_id=7, arrival=0.0),
            serve.Request(rid=1, kind="pf", n=1000, prec="f64", matrix_id=7, arrival=0.05),
            serve.Request(rid=2, kind="pf", n=1000, prec="f32", matrix_id=7, arrival=0.1),
            serve.Request(rid=3, kind="solve", n=1000, prec="f32", matrix_id=7, arrival=0.15),
            serve.Request(rid=4, kind="solve", n=1000, prec="f32", matrix_id=7, arrival=0.2)]
    res = sch.run_trace(reqs)
    # Pfaffians of either label are taken from the FP64 factors; an FP32 solve
    # needs FP32-trailing factors of its own, which the next FP32 solve reuses
    assert not res[0].cached and res[1].cached and res[2].cached
    assert not res[3].cached and res[4].cached


def test_small_solves_hold_tokens_next_to_large_factorizations():
    """A solve of order <= 512 without resident factors runs a factorization, so
    it holds its panel's tokens like any other; batched Pfaffians hold none."""
    ex = FakeExecutor(num_cus=40)
    sch = serve.Scheduler(ex, budget_bytes=1 << 40, workers=4)
    reqs = [serve.Request(rid=0, kind="pf", n=2048, prec="f64", matrix_id=0, arrival=0.0)]
    reqs += [serve.Request(rid=1 + i, kind="solve", n=500, prec="f64", matrix_id=1 + i, arrival=0.0)
             for i in range(6)]
    reqs += [serve.Request(rid=10 + i, kind="pf", n=300, prec="f64", matrix_id=10 + i, arrival=0.0)
             for i in range(6)]
    sch.run_trace(reqs)
    assert serve.tokens(reqs[1], False) == 8 and serve.tokens(reqs[1], True) == 0
    assert serve.tokens(reqs[-1], False) == 0
    assert ex.max_tok <= 40 and sch.tokens_used == 0


def test_ratio_requests_share_the_fp64_factors():
    """A ratio request is served from the resident FP64 factors of its matrix: a
    Pfaffian of order > 512 leaves them, the ratios (and an FP32-labelled
    Pfaffian) reuse them; a ratio on a new matrix factors it first."""
    ex = FakeExecutor()
    sch = serve.Scheduler(ex, budget_bytes=1 << 40, workers=1)
    reqs = [serve.Request(rid=0, kind="pf", n=1000, prec="f64", matrix_id=3, arrival=0.0),
            serve.Request(rid=1, kind="ratio", n=1000, prec="f64", matrix_id=3, arrival=0.05, r=4),
            serve.Request(rid=2, kind="ratio", n=1000, prec="f32", matrix_id=3, arrival=0.1, r=1),
            serve.Request(rid=3, kind="ratio", n=800, prec="f64", matrix_id=4, arrival=0.15, r=2),
            serve.Request(rid=4, kind="ratio", n=800, prec="f64", matrix_id=4, arrival=0.2, r=2)]
    res = sch.run_trace(reqs)
    assert serve.factor_prec(reqs[2]) == "f64"
    assert not res[0].cached and res[1].cached and res[2].cached
    assert not res[3].cached and res[4].cached
    assert sch.reserved == 0 and sch.tokens_used == 0
    # the bytes a ratio holds: its workspace, [U V], the solve behind its error bound
    b = serve.request_bytes(reqs[1], ex, True)
    assert b == ex.ratio_ws(1000, 4) + 2 * 8 * 1000 * 8 + ex.refine_ws(1000, 8)


def test_workload_ratio_share_and_ranks():
    reqs, mids = serve.make_workload(400, rate_hz=100.0, seed=3, ratio_frac=0.5, ratio_rmax=6)
    ratios = [r for r in reqs if r.kind == "ratio"]
    assert ratios and all(1 <= r.r <= 6 and r.prec == "f64" for r in ratios)
    seen = set()
    for r in reqs:   # a ratio always refers to a matrix that appeared before it
        if r.kind == "ratio":
            assert r.matrix_id in seen
        seen.add(r.matrix_id)
    base, _ = serve.make_workload(400, rate_hz=100.0, seed=3)
    assert not any(r.kind == "ratio" for r in base)
    assert [(r.n, r.matrix_id, r.arrival) for r in base] == [(r.n, r.matrix_id, r.arrival) for r in reqs]


def test_ratio_error_bound_terms():
    """The stated ratio error: r = 0 leaves the rounding term alone; otherwise the
    first-order term grows linearly in eta and in ||A||_inf, and the Gram form
    ||R K^-1 R^T||_2 (X^T X = R^T R) equals ||X K^-1 X^T||_2."""
    import math

    import numpy as np
    u = 2.0 ** -53
    assert serve.ratio_error_bound(100, 0, 5.0, None, None, 0.0, 0.0) == 64 * u * 5.0
    rng = np.random.default_rng(0)
    n, r = 40, 3
    S = np.tril(rng.standard_normal((n, n)), -1)
    A = S - S.T
    W = rng.standard_normal((n, 2 * r))
    X = np.linalg.solve(A, W)
    J = np.block([[np.zeros((r, r)), np.eye(r)], [-np.eye(r), np.zeros((r, r))]])
    K = W.T @ X - J
    direct = np.linalg.norm(X @ np.linalg.solve(K, X.T), 2)
    eta, an = 1e-16, np.abs(A).sum(1).max()
    got = serve.ratio_error_bound(n, r, 0.0, X.T @ X, W.T @ X, eta, an) - 64 * u
    assert math.isclose(got, 0.5 * 2 * r * direct * math.sqrt(n) * eta * an, rel_tol=1e-9)
    got2 = serve.ratio_error_bound(n, r, 0.0, X.T @ X, W.T @ X, 2 * eta, an) - 64 * u
    assert math.isclose(got2, 2 * got, rel_tol=1e-9)

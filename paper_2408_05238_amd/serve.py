"""Continuous-batching request loop for Pfaffian and solve jobs on one GPU.

Requests arrive over time; the scheduler admits them as workers, HBM budget and
compute tokens free up, so work of different requests overlaps on the device
(one HIP stream per worker):

* HBM budget: every admitted request reserves the bytes it will hold (working
  copy of A, factorization workspace, right-hand sides, the original matrix for
  refinement); factors of finished requests stay resident in an LRU cache keyed
  by (matrix id, precision) and are evicted when an admission needs the room.
  A request whose factors are resident skips the factorization.
* compute tokens: a factorization launches persistent panel kernels of
  ceil((n-1)/64) workgroups that must be co-resident; the scheduler only runs
  factorizations whose token sum fits the device's CU count, so two of them can
  never wait on each other for residency.  Batched launches and requests served
  from resident factors hold no tokens.
* continuous batching: small Pfaffian requests (n <= 512) waiting together are
  factored by one persistent batched launch.
* Pfaffian ratios: a "ratio" request asks for Pf(A + U V^T - V U^T) / Pf(A)
  with U, V of rank r <= 32; it is served from the resident FP64 factors of A
  (factoring A first when they are not resident), one solve with 2r
  right-hand sides instead of a factorization of the updated matrix.
* precision: a request labelled FP32 means an FP32-trailing factorization plus
  iterative refinement to FP64 backward error; refinement corrects solves only,
  so Pfaffian and ratio requests are always taken from FP64 factors.  Every
  result states its error against FP64: the backward error eta of its solution
  for a solve, the relative log|Pf| bound of the FP64 reduction for a Pfaffian,
  and for a ratio a first-order bound on the error of log|ratio| from the
  measured backward error of its solve (see ratio_error_bound).
* FIFO with overtaking: a request that does not fit yet does not block smaller
  ones behind it.

The scheduling core (`Scheduler`) is independent of the GPU: it drives an
executor object and a clock, so its admission, eviction and accounting logic can
be exercised with a fake executor and a fake clock.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Dict, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    kind: str            # "pf", "solve" or "ratio"
    n: int
    prec: str            # "f64" or "f32" (FP32 trailing update + refinement for solves)
    matrix_id: int
    arrival: float       # seconds from the start of the trace
    nrhs: int = 16
    A: object = None     # client-owned device tensor (column-major), read-only
    B: object = None     # client-owned right-hand sides for solves
    r: int = 0           # rank of a ratio request's update
    U: object = None     # client-owned n x r device tensors of a ratio request
    V: object = None


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    start: float = 0.0
    end: float = 0.0
    logabs: float = float("nan")
    sign: int = 0
    info: int = 0
    X: object = None
    iters: int = 0
    berr: float = 0.0
    cached: bool = False
    batched: bool = False
    err: float = float("nan")   # stated error against FP64 (see the module docstring)
    err_kind: str = ""          # "berr" (solve), "logpf_rel_bound" (Pfaffian) or "log_ratio_bound" (ratio)

    @property
    def latency(self) -> float:
        return self.end - self.arrival


def percentile(values: List[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not values:
        return float("nan")
    v = sorted(values)
    r = max(1, int(math.ceil(q / 100.0 * len(v))))
    return v[min(r, len(v)) - 1]


SMALL_N = 512
# Relative error bound of log|Pf| from the FP64 reductions, |d| / max(1, |log|Pf||),
# the bound their parity tests verify against the oracle.
PF_REL_BOUND = 1e-12


U_RND = 2.0 ** -53


def ratio_error_bound(n: int, r: int, logabs: float, XtX, WtX, eta: float, anorm_inf: float) -> float:
    """First-order bound on the error of log|ratio| for a ratio served through
    the identity ratio = Pf(K) / Pf(-J), K = W^T X - J, X = A^-1 W, W = [U V]
    (J = [[0, I_r], [-I_r, 0]]).  A backward error dA of the solve perturbs K by
    X^T dA X (A skew), and d log|Pf(K)| = tr(K^-1 dK) / 2, so
      |d| <= (2r / 2) ||X K^-1 X^T||_2 ||dA||_2,
    with ||X K^-1 X^T||_2 = ||R K^-1 R^T||_2 (X^T X = R^T R) and
    ||dA||_2 <= sqrt(n) eta ||A||_inf (eta: the measured componentwise-normwise
    backward error of the solve with W); plus 64 u max(1, |log|ratio||) for the
    2r x 2r Pfaffian, the logarithms and their sums.  XtX, WtX: 2r x 2r host arrays."""
    import numpy as np
    tail = 64 * U_RND * max(1.0, abs(logabs))
    if r == 0:
        return tail
    m = 2 * r
    J = np.block([[np.zeros((r, r)), np.eye(r)], [-np.eye(r), np.zeros((r, r))]])
    K = np.asarray(WtX, dtype=np.float64) - J
    w, Q = np.linalg.eigh(0.5 * (XtX + XtX.T))
    Rt = Q * np.sqrt(np.clip(w, 0.0, None))          # X^T X = Rt Rt^T
    c = np.linalg.norm(Rt.T @ np.linalg.solve(K, Rt), 2)
    return 0.5 * m * c * math.sqrt(n) * eta * anorm_inf + tail


def factor_prec(req: Request) -> str:
    """Precision of the factors a request uses: Pfaffians and ratios always FP64."""
    return "f64" if req.kind in ("pf", "ratio") else req.prec


def factor_key(req: Request):
    return (req.matrix_id, factor_prec(req))


def factor_bytes(n: int) -> int:
    """Resident factors: the factored array, ipiv and T."""
    return 8 * n * n + 4 * n + 8 * n


def request_bytes(req: Request, ex, have_factors: bool) -> int:
    """Device bytes a request holds while it runs (besides cached factors).

    `ex` supplies the library's workspace queries (ltlt_ws, solve_ws, refine_ws,
    ratio_ws).
    """
    n = req.n
    b = 0
    if not have_factors:
        b += factor_bytes(n) + ex.ltlt_ws(n, 0 if factor_prec(req) == "f64" else 1)
    if req.kind == "solve":
        b += 2 * 8 * n * req.nrhs          # right-hand sides and solution
        b += ex.refine_ws(n, req.nrhs)     # every solve states its backward error
    elif req.kind == "ratio":
        m = 2 * req.r
        b += ex.ratio_ws(n, req.r)         # the ratio itself
        b += 2 * 8 * n * m + ex.refine_ws(n, m)  # its error bound: [U V] and the solve
    return b


def batchable(req: Request, have_factors: bool) -> bool:
    """Small Pfaffian requests without resident factors go to the batched launch."""
    return req.kind == "pf" and req.n <= SMALL_N and not have_factors


def tokens(req: Request, have_factors: bool) -> int:
    """CUs a dispatch needs co-resident: the panel workgroups of a factorization."""
    if have_factors or batchable(req, have_factors) or req.n < 2:
        return 0
    return (req.n - 1 + 63) // 64


class FactorCache:
    """LRU of resident factors under the shared budget.  Entries in use by a
    running request are pinned and never evicted."""

    def __init__(self):
        self.entries: "collections.OrderedDict[tuple, tuple]" = collections.OrderedDict()
        self.pins: Dict[tuple, int] = {}
        self.bytes = 0

    def get(self, key):
        if key in self.entries:
            self.entries.move_to_end(key)
            return self.entries[key][0]
        return None

    def put(self, key, value, nbytes):
        if key in self.entries:
            self.bytes -= self.entries.pop(key)[1]
        self.entries[key] = (value, nbytes)
        self.bytes += nbytes

    def pin(self, key):
        self.pins[key] = self.pins.get(key, 0) + 1

    def unpin(self, key):
        self.pins[key] -= 1
        if not self.pins[key]:
            del self.pins[key]

    def evict_lru(self, protect=None) -> bool:
        """Drop the least recently used unpinned entry; False if there is none."""
        for key in self.entries:
            if key != protect and key not in self.pins:
                _, nb = self.entries.pop(key)
                self.bytes -= nb
                return True
        return False


class Scheduler:
    """Admission and dispatch; `executor.run(batch, have)` does the work of one dispatch.

    executor interface:
      run(reqs: List[Request], factors: Optional[object]) -> (List[Result], new_factors or None)
      ltlt_ws(n, prec), solve_ws(n, nrhs), refine_ws(n, nrhs) -> bytes
      num_cus -> int
    """

    def __init__(self, executor, budget_bytes: int = 64 << 30, workers: int = 8, clock=time.perf_counter,
                 batch_small: bool = True, max_batch: int = 64):
        self.ex = executor
        self.budget = budget_bytes
        self.workers = workers
        self.clock = clock
        self.batch_small = batch_small
        self.max_batch = max_batch
        self.cache = FactorCache()
        self.lock = threading.Condition()
        self.reserved = 0          # bytes held by running requests
        self.tokens_used = 0
        self.high_water = 0
        self.busy = 0
        self.queue: List[Request] = []
        self.results: Dict[int, Result] = {}
        self.evictions = 0
        self.rejected = 0
        self._stop = False

    # -- accounting -----------------------------------------------------------
    def _need(self, req: Request):
        have = self.cache.get(factor_key(req)) is not None
        return request_bytes(req, self.ex, have), tokens(req, have), have

    def _fits(self, nbytes: int, protect=None) -> bool:
        while self.reserved + self.cache.bytes + nbytes > self.budget:
            if not self.cache.evict_lru(protect):
                return False
            self.evictions += 1
        return True

    def _pick(self):
        """Next dispatch (list of requests) that fits, FIFO with overtaking."""
        for qi, req in enumerate(self.queue):
            nb, tk, have = self._need(req)
            if nb > self.budget:
                self.queue.pop(qi)
                self.rejected += 1
                res = Result(req.rid, req.arrival, info=-100)
                res.start = res.end = self.clock()
                self.results[req.rid] = res
                return None
            if self.tokens_used + tk > self.ex.num_cus:
                continue
            if not self._fits(nb, factor_key(req) if have else None):
                continue
            batch = [req]
            if self.batch_small and batchable(req, have):
                total = nb
                for other in self.queue[qi + 1:]:
                    if len(batch) >= self.max_batch:
                        break
                    if other.kind == "pf" and other.n <= SMALL_N:
                        nb2, _, have2 = self._need(other)
                        if batchable(other, have2) and self._fits(total + nb2):
                            batch.append(other)
                            total += nb2
                nb = total
            for r in batch:
                self.queue.remove(r)
            if have:
                self.cache.pin(factor_key(req))
            self.reserved += nb
            self.tokens_used += tk
            self.high_water = max(self.high_water, self.reserved + self.cache.bytes)
            return batch, nb, tk, have
        return None

    # -- worker ---------------------------------------------------------------
    def _worker(self):
        while True:
            with self.lock:
                pick = None
                while True:
                    if self._stop and not self.queue:
                        return
                    pick = self._pick()
                    if pick:
                        break
                    self.lock.wait(0.005)
                batch, nb, tk, have = pick
                self.busy += 1
                factors = self.cache.get(factor_key(batch[0])) if have else None
            start = self.clock()
            results, new_factors = self.ex.run(batch, factors)
            end = self.clock()
            with self.lock:
                for req, res in zip(batch, results):
                    res.arrival = req.arrival
                    res.start, res.end = start, end
                    self.results[req.rid] = res
                self.reserved -= nb
                self.tokens_used -= tk
                self.busy -= 1
                if have:
                    self.cache.unpin(factor_key(batch[0]))
                if new_factors is not None:
                    req = batch[0]
                    self.cache.put(factor_key(req), new_factors, factor_bytes(req.n))
                    self.high_water = max(self.high_water, self.reserved + self.cache.bytes)
                self.lock.notify_all()

    def run_trace(self, requests: List[Request], t0: Optional[float] = None) -> Dict[int, Result]:
        """Replay `requests` (arrival times relative to t0) through `workers` threads."""
        self._stop = False
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock() if t0 is None else t0
        for r in reqs:
            r.arrival = t0 + r.arrival
        threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(self.workers)]
        for t in threads:
            t.start()
        i = 0
        while i < len(reqs):
            now = self.clock()
            with self.lock:
                while i < len(reqs) and reqs[i].arrival <= now:
                    self.queue.append(reqs[i])
                    i += 1
                self.lock.notify_all()
            if i < len(reqs):
                dt = reqs[i].arrival - self.clock()
                if dt > 0:
                    time.sleep(min(dt, 0.001))
        with self.lock:
            self._stop = True
            self.lock.notify_all()
        for t in threads:
            t.join()
        return self.results

    def stats(self, t_begin: float) -> dict:
        res = [r for r in self.results.values() if r.info != -100]
        lat = [r.latency for r in res]
        berr = [r.err for r in res if r.err_kind == "berr"]
        t_end = max((r.end for r in res), default=t_begin)
        return {
            "completed": len(res),
            "rejected": self.rejected,
            "p50_ms": percentile(lat, 50) * 1e3,
            "p99_ms": percentile(lat, 99) * 1e3,
            "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else float("nan"),
            "req_per_s": len(res) / max(t_end - t_begin, 1e-9),
            "hbm_high_water_gb": self.high_water / 2 ** 30,
            "evictions": self.evictions,
            "cache_hits": sum(1 for r in res if r.cached),
            "batched": sum(1 for r in res if r.batched),
            "solve_berr_max": max(berr) if berr else float("nan"),
            "pf_logabs_rel_bound": PF_REL_BOUND,
            "errors_stated": sum(1 for r in res if r.err_kind),
            # numerical outcomes other than 0 (a singular or odd-order input's
            # info, SKF_ENONFINITE, SKF_ETIMEOUT), by code
            "outcomes": {str(k): v for k, v in sorted(collections.Counter(r.info for r in res if r.info).items())},
        }


# ---------------------------------------------------------------------------
# GPU executor (HIP library through the binding)
# ---------------------------------------------------------------------------

class GpuExecutor:
    """Runs one dispatch on the calling worker thread's own stream."""

    def __init__(self, device="cuda:0"):
        import torch

        from . import skf
        self.skf = skf
        self.torch = torch
        self.device = torch.device(device)
        skf.lib()
        self.num_cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        self._tls = threading.local()

    def ltlt_ws(self, n: int, prec: int) -> int:
        return self.skf.ltlt_workspace(n, prec)

    def solve_ws(self, n: int, nrhs: int) -> int:
        return self.skf.solve_workspace(n, nrhs)

    def refine_ws(self, n: int, nrhs: int) -> int:
        return self.skf.refine_workspace(n, nrhs)

    def ratio_ws(self, n: int, r: int) -> int:
        return self.skf.pf_ratio_workspace(n, r)

    def _stream(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream(device=self.device)
            self._tls.stream = s
        return s

    def run(self, reqs: List[Request], factors):
        skf, torch = self.skf, self.torch
        s = self._stream()
        with torch.cuda.stream(s):
            if len(reqs) > 1 or batchable(reqs[0], factors is not None):
                mats = []
                for r in reqs:
                    w = skf.colmajor(r.n, r.n, device=self.device)
                    w.copy_(r.A)
                    mats.append(w)
                la, sg, info = skf.logpf_batched(mats, stream=s)
                s.synchronize()
                la, sg, info = la.cpu().tolist(), sg.cpu().tolist(), info.cpu().tolist()
                out = [Result(r.rid, r.arrival, logabs=la[i], sign=sg[i], info=info[i], batched=len(reqs) > 1,
                              err=PF_REL_BOUND, err_kind="logpf_rel_bound")
                       for i, r in enumerate(reqs)]
                return out, None
            r = reqs[0]
            prec = skf.PREC_F64 if factor_prec(r) == "f64" else skf.PREC_F32_TRAILING
            new = None
            if factors is None:
                LT = skf.colmajor(r.n, r.n, device=self.device)
                LT.copy_(r.A)
                ipiv = torch.empty(max(r.n, 1), dtype=torch.int32, device=self.device)
                T = torch.empty(max(r.n - 1, 1), dtype=torch.float64, device=self.device)
                work = skf.workspace(skf.ltlt_workspace(r.n, prec), self.device)
                dinfo = torch.zeros(1, dtype=torch.int32, device=self.device)
                skf.ltlt(LT, ipiv, T, prec, work, dinfo, stream=s)
                del work
                factors = new = (LT, ipiv, T, dinfo)
            LT, ipiv, T, dinfo = factors
            res = Result(r.rid, r.arrival, cached=new is None)
            if r.kind == "pf":
                la, sg = skf.logpf_from_factors(r.n, ipiv[:r.n], T[:max(r.n - 1, 0)], stream=s)
                s.synchronize()
                res.logabs, res.sign, res.info = float(la.item()), int(sg.item()), int(dinfo.item())
                res.err, res.err_kind = PF_REL_BOUND, "logpf_rel_bound"
            elif r.kind == "ratio":
                Tn = T[:max(r.n - 1, 0)]
                la, sg, info = skf.pf_ratio(LT, ipiv[:r.n], Tn, r.U, r.V, stream=s)
                res.logabs, res.sign = float(la.item()), int(sg.item())
                res.info = int(dinfo.item()) or int(info)
                eta, anorm, XtX, WtX = 0.0, 0.0, None, None
                if r.r > 0 and res.info == 0:
                    # the stated error: the solve with W = [U V] through the same
                    # factors, its measured backward error and the 2r x 2r Gram products
                    W = skf.colmajor(r.n, 2 * r.r, device=self.device)
                    W[:, :r.r].copy_(r.U)
                    W[:, r.r:].copy_(r.V)
                    X, _, _, eta = skf.solve_refine(r.A, LT, ipiv[:r.n], Tn, W, maxit=0, stream=s)
                    S = torch.tril(r.A, -1).abs()
                    anorm = float((S.sum(0) + S.sum(1)).max().item())
                    Xh, Wh = X.cpu().numpy(), W.cpu().numpy()
                    XtX, WtX = Xh.T @ Xh, Wh.T @ Xh
                s.synchronize()
                res.err = ratio_error_bound(r.n, r.r, res.logabs, XtX, WtX, float(eta), anorm)
                res.err_kind = "log_ratio_bound"
            else:
                # FP64 factors: one solve, then the backward error (no correction
                # when it already meets the tolerance); FP32-trailing factors:
                # refinement until it does
                X, st, it, be = skf.solve_refine(r.A, LT, ipiv[:r.n], T[:max(r.n - 1, 0)], r.B, stream=s)
                res.X, res.info, res.iters, res.berr = X, st, it, be
                res.err, res.err_kind = be, "berr"
                s.synchronize()
            return [res], new


def make_workload(count: int, rate_hz: float, seed: int = 8, nmin: int = 64, nmax: int = 4096,
                  f32_frac: float = 0.3, solve_frac: float = 0.5, reuse_frac: float = 0.25,
                  ratio_frac: float = 0.0, ratio_rmax: int = 8):
    """The serving trace: Poisson arrivals at `rate_hz`; n = 2 round(exp(U(ln nmin, ln nmax))/2);
    70/30 FP64/FP32+refine; Pfaffian:solve 50:50; 25% of requests reuse an earlier matrix.
    With ratio_frac > 0, that share of the requests that reuse a matrix ask for a
    Pfaffian ratio of a rank-r update (r uniform in 1..ratio_rmax) instead."""
    from . import inputs
    reqs = []
    t = 0.0
    ctr = 0
    mids = []
    for i in range(count):
        u = [inputs.uniform(seed, inputs.STREAM_SERVE, ctr + c) for c in range(6)]
        ctr += 6
        t += -math.log(max(u[0], 1e-300)) / rate_hz if rate_hz > 0 else 0.0
        reuse = bool(mids) and u[1] < reuse_frac
        if reuse:
            mid, n = mids[int(u[2] * len(mids)) % len(mids)]
        else:
            n = int(2 * round(math.exp(math.log(nmin) + u[2] * (math.log(nmax) - math.log(nmin))) / 2))
            n = max(nmin, min(nmax, n))
            mid = len(mids)
            mids.append((mid, n))
        kind = "solve" if u[3] < solve_frac else "pf"
        prec = "f32" if u[4] < f32_frac else "f64"
        rk = 0
        if reuse and u[5] < ratio_frac:
            kind, prec = "ratio", "f64"
            rk = 1 + min(ratio_rmax - 1, int(u[4] * ratio_rmax))
        reqs.append(Request(rid=i, kind=kind, n=n, prec=prec, matrix_id=mid, arrival=t, r=rk))
    return reqs, mids


def materialize(reqs: List[Request], mids, seed: int = 8, device="cuda:0", threads: int = 8):
    """Client-side inputs on the device: matrix `mid` is the skew Gaussian matrix of
    its order from stream STREAM_BATCH0 + mid; a solve's right-hand sides come from
    stream STREAM_BATCH0 + 1_000_000 + rid (Gaussian, nrhs columns)."""
    from . import inputs, skf
    mats = {}
    for mid, n in mids:
        a = inputs.skew_gaussian(n, seed, inputs.STREAM_BATCH0 + mid, threads=threads)
        mats[mid] = skf.to_device_colmajor(a, device)
    for r in reqs:
        r.A = mats[r.matrix_id]
        if r.kind == "solve":
            r.B = skf.to_device_colmajor(inputs.gaussian(r.n, r.nrhs, seed, inputs.STREAM_BATCH0 + 1_000_000 + r.rid),
                                         device)
        elif r.kind == "ratio":
            # U and V of the update: Gaussian, scaled by 1/sqrt(n) so the update
            # is of the size of A's entries
            w = inputs.gaussian(r.n, 2 * r.r, seed, inputs.STREAM_BATCH0 + 1_000_000 + r.rid) / math.sqrt(r.n)
            r.U = skf.to_device_colmajor(w[:, :r.r], device)
            r.V = skf.to_device_colmajor(w[:, r.r:], device)
    return mats

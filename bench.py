#!/usr/bin/env python3
"""Benchmark: blocked skew LTL^T on one MI355X, GFLOP/s on the nominal n^3/3.

One step = one full factorization P A P^T = L T L^T (panel kernels, trailing
skew rank-2k updates, final row permutation of L) of a seeded Gaussian skew
matrix of order n = 16384 in FP64, inputs resident in HBM (every step factors
its own pre-loaded copy, so no copy sits in the timed region).

Prints ONE JSON line.  Besides the contract fields it carries
  roofline     the trailing-update kernel (nearly all flops) against MI355X's
               FP64 matrix peak, from HIP events recorded around each of its
               launches during the timed steps;
  cpu_baseline the CPU oracle (unblocked, FP64) on a bounded sample of the same
               matrix: its first S elimination steps, nominal flops sum (n-k-1)^2;
  panel        the panel kernel's share and microseconds per elimination step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "skr2k_perm_n16384_traffic.txt"))
    ap.add_argument("--workload", choices=["ltlt", "mixed", "batched", "serve", "complex"], default="ltlt",
                    help="ltlt: the headline factorization; mixed: FP32-trailing + refinement vs FP64 solves "
                         "(n=16384, 32768, 16 RHS); batched: 8192 small matrices in one launch; serve: "
                         "2000-request Poisson trace; complex: complex128 Pfaffian-only reduction (n=4096)")
    ap.add_argument("--sizes", default="16384,32768", help="orders for --workload mixed")
    ap.add_argument("--count", type=int, default=0, help="matrices (batched) or requests (serve); 0 = default")
    ap.add_argument("--no-side", action="store_true",
                    help="ltlt workload: skip the Pfaffian-only and low-rank ratio measurements after the timed steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run three plain device copies of 1 GiB (reference for HBM counters)")
    return ap.parse_args()


def read_traffic(path: str):
    """HBM bytes per trailing-update launch from a committed counter summary, or None.

    The summary records the sha256 of the kernel source it was measured on; a
    changed source voids it.
    """
    import hashlib
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        src = os.path.join(ROOT, "paper_2408_05238_amd", "csrc", "skr2k.hip")
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if kv.get("source_sha256") != h:
            return None
        return float(kv["bytes_per_launch"])
    except Exception:
        return None


def _oracle_sample(A_host, n: int, target_s: float, threads: int):
    """Oracle on the first S elimination steps of the matrix, S grown until the
    run takes about target_s: (S, seconds, nominal flops sum (n-k-1)^2)."""
    import numpy as np
    import oracle
    S = 4
    while True:
        Ac = np.array(A_host, order="F", copy=True)
        t0 = time.perf_counter()
        oracle.ltlt(Ac, nthreads=threads, nsteps=S, want_gap=False, inplace=True)
        dt = time.perf_counter() - t0
        del Ac
        if dt >= 0.5 * target_s or S >= n - 2:
            break
        S = min(n - 2, max(S * 2, int(S * target_s / max(dt, 1e-3))))
    return S, dt, float(sum((n - k - 1) ** 2 for k in range(S)))


def cpu_baseline(A_host, n: int, target_s: float):
    """Oracle on a bounded sample of the same matrix (its first S elimination
    steps), with the host's threads (at most 16) and with one thread."""
    threads = max(1, min(16, os.cpu_count() or 1))
    S, dt, flops = _oracle_sample(A_host, n, target_s, threads)
    S1, dt1, flops1 = _oracle_sample(A_host, n, 0.5 * target_s, 1)
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {S} elimination steps of the n={n} matrix (unblocked FP64 oracle), "
                      f"nominal flops sum_k (n-k-1)^2 = {flops:.3e}, {dt:.2f} s",
            "single_thread": {"value": round(flops1 / dt1 / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": f"first {S1} elimination steps, nominal flops {flops1:.3e}, {dt1:.2f} s"}}


def _device():
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2408_05238_amd import skf
    skf.lib()  # raises if libskf.so is missing: there is no fallback path
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    return dev


def _sig(v):
    """Floats to 4 significant digits (error figures such as 1e-15 stay visible)."""
    return float(f"{v:.4g}") if isinstance(v, float) else v


def _line(metric, value, unit, ms_per_step, args, dtype, workload, higher=True, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": {"workload": workload}}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_mixed(args):
    """FP64 factor + solve against FP32-trailing factor + refined solve, 16 RHS.

    A: seed 5; B: seed 6.  Each step factors a pre-loaded copy and solves.
    """
    import numpy as np
    import torch

    from paper_2408_05238_amd import inputs, skf
    dev = _device()
    nrhs = 16
    rows = []
    for n in [int(x) for x in args.sizes.split(",") if x]:
        A = inputs.skew_gaussian(n, 5, inputs.STREAM_A, threads=16)
        Bh = inputs.gaussian(n, nrhs, 6, inputs.STREAM_B)
        A0 = skf.to_device_colmajor(A, device=dev)
        del A
        B = skf.to_device_colmajor(Bh, device=dev)
        res = {}
        for prec_name, prec in (("f64", skf.PREC_F64), ("f32_refine", skf.PREC_F32_TRAILING)):
            LT = skf.colmajor(n, n, device=dev)
            ipiv = torch.empty(n, dtype=torch.int32, device=dev)
            T = torch.empty(n - 1, dtype=torch.float64, device=dev)
            wl = skf.workspace(skf.ltlt_workspace(n, prec), dev)
            dinfo = torch.zeros(1, dtype=torch.int32, device=dev)
            X = skf.colmajor(n, nrhs, device=dev)
            ws = skf.workspace(max(skf.solve_workspace(n, nrhs), skf.refine_workspace(n, nrhs)), dev)
            times, tf = [], []
            for it in range(args.warmup + args.steps):
                LT.copy_(A0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                skf.ltlt(LT, ipiv, T, prec, wl, dinfo)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                if prec == skf.PREC_F64:
                    X.copy_(B)
                    skf.solve(LT, ipiv, T, X, work=ws, dinfo=dinfo)
                    st, iters = 0, 0
                else:
                    _, st, iters, berr = skf.solve_refine(A0, LT, ipiv, T, B, X=X, tol=1e-13, maxit=10, work=ws)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if it >= args.warmup:
                    times.append(t2 - t0)
                    tf.append(t1 - t0)
            assert int(dinfo.item()) == 0
            Xh = X.cpu().numpy()
            # backward error max_j |b_j - A x_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf), FP64 on the device
            F = _full_skew(A0)
            R = B - torch.matmul(F, X)
            eta = float((R.abs().amax(0) / (F.abs().sum(1).amax() * X.abs().amax(0)
                                            + B.abs().amax(0))).amax().item())
            del F, R
            la, sg = skf.logpf_from_factors(n, ipiv, T)
            res[prec_name] = {"ms": round(1e3 * float(np.median(times)), 2),
                              "factor_ms": round(1e3 * float(np.median(tf)), 2),
                              "factor_gflops": round(n ** 3 / 3 / float(np.median(tf)) / 1e9, 1),
                              "iters": iters, "status": st, "backward_error": eta,
                              "logabs_pf": float(la.item()), "sign": int(sg.item()),
                              "ipiv": ipiv.cpu().numpy()}
            del LT, wl, ws, X, Xh
            torch.cuda.empty_cache()
        p64, p32 = res["f64"], res["f32_refine"]
        rows.append({"n": n, "f64": {k: v for k, v in p64.items() if k != "ipiv"},
                     "f32_refine": {k: v for k, v in p32.items() if k != "ipiv"},
                     "speedup_total": round(p64["ms"] / p32["ms"], 3),
                     "speedup_factor": round(p64["factor_ms"] / p32["factor_ms"], 3),
                     "pivot_mismatches_vs_f64": int((p64["ipiv"] != p32["ipiv"]).sum()),
                     "logpf_rel_diff_vs_f64": abs(p32["logabs_pf"] - p64["logabs_pf"]) /
                     max(1.0, abs(p64["logabs_pf"]))})
        del A0, B
        torch.cuda.empty_cache()
    head = rows[0]
    _line("LTL^T factor + 16-RHS solve, FP32-trailing + refinement vs FP64 (speedup)",
          head["speedup_total"], "x", head["f32_refine"]["ms"], args, "f64 storage, f32 trailing products",
          f"skew Gaussian n={','.join(str(r['n']) for r in rows)} (seed 5), B 16 Gaussian columns (seed 6), "
          f"refine to backward error 1e-13", results=rows)


def _full_skew(L):
    """Full skew matrix from the strict lower triangle of a device matrix (torch)."""
    import torch
    low = torch.tril(L, -1)
    return low - low.T


def bench_batched(args):
    """8192 matrices, even n uniform on [32, 512] (seed 7), log|Pf| and sign in one launch
    (the Pfaffian-only reduction); the full batched factorization is timed beside it."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    from paper_2408_05238_amd import inputs, skf
    dev = _device()
    count = args.count or 8192
    n_list = inputs.even_sizes(count, 32, 512, 7).astype(np.int64)
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum(n_list * n_list)
    host = torch.empty(int(offs[-1]), dtype=torch.float64).pin_memory()
    hv = host.numpy()

    def fill(b):
        n = int(n_list[b])
        hv[offs[b]:offs[b + 1]] = inputs.batch_matrix(n, 7, b).ravel(order="F")
    with cf.ThreadPoolExecutor(16) as pool:
        list(pool.map(fill, range(count)))
    src = host.to(dev)
    del host, hv
    nrun = args.warmup + args.steps
    copies = [src.clone() for _ in range(nrun)]
    work = skf.workspace(skf.batched_workspace(n_list), dev)
    torch.cuda.synchronize()
    outs = []
    for i in range(args.warmup):
        outs.append(skf.logpf_batched_packed(copies[i], offs[:-1], n_list, work=work))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, nrun):
        outs.append(skf.logpf_batched_packed(copies[i], offs[:-1], n_list, work=work))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    la, sg, info, _ = outs[-1]
    assert int(info.abs().sum().item()) == 0
    same = all(torch.equal(o[0], la) and torch.equal(o[1], sg) for o in outs)
    # the same batch through the full factorization (paired steps, L left in place)
    copies[0].copy_(src)
    ptrs = [copies[0][int(offs[b]):int(offs[b + 1])].view(int(n_list[b]), int(n_list[b])).T
            for b in range(count)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    la_f, sg_f, info_f, _, _ = skf.ltlt_batched(ptrs, with_factors=False, work=work)
    torch.cuda.synchronize()
    dt_full = time.perf_counter() - t1
    flops = float((n_list.astype(np.float64) ** 3).sum() / 3)
    bytes_ = float((n_list * (n_list - 1) // 2).sum() * 8)
    extra = {"gflops_nominal": round(flops / dt / 1e9, 1), "hbm_gbs_min_bytes": round(bytes_ / dt / 1e9, 1),
             "runs_bitwise_identical": same, "sum_n3_over_3": flops,
             "full_factorization": {"pf_per_s": round(count / dt_full, 1), "ms": round(dt_full * 1e3, 3),
                                    "signs_equal": bool(torch.equal(sg_f, sg)),
                                    "max_rel_logpf_diff": float(((la_f - la).abs() / la.abs().clamp(min=1.0)).max())}}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        k = 0
        while time.perf_counter() - t < min(args.cpu_seconds, 10.0) and k < count:
            n = int(n_list[k])
            oracle.logpf_pfonly(inputs.batch_matrix(n, 7, k))
            k += 1
        ct = time.perf_counter() - t
        extra["cpu_baseline"] = {"value": round(k / ct, 1), "unit": "Pf/s", "cores": 1, "kind": "oracle",
                                 "sample": f"first {k} matrices of the batch, one at a time"}
    _line("batched Pf/s (8192 skew matrices, even n uniform on [32,512])", round(count / dt, 1), "Pf/s",
          round(dt * 1e3, 3), args, "f64", f"{count} skew Gaussian matrices, even n uniform on [32,512] (seed 7), "
          f"log|Pf| and sign in one persistent launch (Pfaffian-only reduction)", **extra)


def bench_complex(args):
    """Complex128 Pfaffian-only reduction of one n x n complex skew Gaussian matrix
    (real part seed/stream A, imaginary part seed/stream IMAG); n defaults to 4096.
    The blocked reduction: complex panel kernel plus the real trailing update run
    on the real and imaginary planes (FP64 matrix cores)."""
    import ctypes

    import numpy as np
    import torch

    from paper_2408_05238_amd import inputs, skf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lib = skf.lib()
    n = args.n if args.n != 16384 else 4096
    dev = torch.device("cuda:0")
    A = inputs.skew_gaussian_c128(n, args.seed)
    dA = skf.to_device_colmajor(A, device=dev)
    work = skf.workspace(int(lib.skf_pfonly_c128_workspace(n)), dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    T = torch.empty(max(n - 1, 1), dtype=torch.complex128, device=dev)
    dinfo = torch.zeros(1, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        skf.pfonly_c128(dA, ipiv, T, work, dinfo)
    torch.cuda.synchronize()
    lib.skf_profile_read(None, None, None, 1)
    lib.skf_profile_enable(1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        skf.pfonly_c128(dA, ipiv, T, work, dinfo)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    lib.skf_profile_enable(0)
    pms = (ctypes.c_double * 2)()
    pfl = (ctypes.c_double * 2)()
    pcnt = (ctypes.c_int64 * 2)()
    lib.skf_profile_read(pms, pfl, pcnt, 1)
    assert int(dinfo.item()) == 0
    la, ph = skf.logpf_c128_from_factors(n, ipiv, T)
    # nominal work: n/2 complex rank-2 trailing updates = 4 n^3/3 real flops
    flops = 4.0 * n ** 3 / 3.0
    upd_tf = pfl[1] / (pms[1] * 1e-3) / 1e12 if pms[1] > 0 else 0.0
    blocked = pcnt[0] > 0  # only the blocked form records panel launches
    out = {"metric": f"complex128 Pfaffian-only reduction time at n={n}", "value": round(ms, 3), "unit": "ms",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
           "data": "synthetic",
           "config": {"workload": f"dense complex skew-symmetric Gaussian matrix n={n} (seed {args.seed}), "
                                  "blocked Pfaffian-only reduction" if blocked else "unblocked Pfaffian-only reduction",
                      "n": n},
           "gflops_nominal": round(flops / (ms * 1e-3) / 1e9, 1),
           "roofline": {"bound": "mfma", "kernel": "skr2k_perm on the real and imaginary planes (trailing update)",
                        "achieved": round(upd_tf, 3), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(upd_tf / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                        "launches": int(2 * pcnt[1]) // max(args.steps, 1),
                        "ms_per_reduction": round(pms[1] / max(args.steps, 1), 3)},
           "panel": {"ms_per_reduction": round(pms[0] / max(args.steps, 1), 3),
                     "us_per_step": round(pms[0] * 1e3 / max(args.steps, 1) / max(n // 2, 1), 3),
                     "share": round(pms[0] / max(args.steps, 1) / ms, 3)},
           "logabs_pf": float(la.item()), "phase": [float(ph.real.item()), float(ph.imag.item())]}
    if not args.no_side:
        out["ltlt"] = _complex_ltlt_side(args, n, dA, lib)
    if not args.no_cpu_baseline:
        import oracle
        m = min(n, 1024)
        t1 = time.perf_counter()
        oracle.pfonly_c128(inputs.skew_gaussian_c128(m, args.seed))
        ct = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(ct * 1e3 * (n / m) ** 3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"numpy oracle on the n={m} leading case of the same recipe, {ct:.2f} s, "
                                         f"scaled by (n/{m})^3"}
    print(json.dumps(out), flush=True)


def _complex_ltlt_side(args, n, dA, lib):
    """The complex LTL^T of the same matrix (in place on a copy restored before
    each timed call; HIP events around the call only) and the solve with its
    factors for one right-hand side.  Nominal work: n unpaired complex rank-2
    updates, 8 n^3 / 3 real flops."""
    import ctypes

    import numpy as np
    import torch

    from paper_2408_05238_amd import skf
    dev = dA.device
    if int(lib.skf_ltlt_c128_workspace(n)) == 0:
        return {"skipped": "order beyond the complex LTL^T panel"}
    work = skf.workspace(int(lib.skf_ltlt_c128_workspace(n)), dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    T = torch.empty(max(n - 1, 1), dtype=torch.complex128, device=dev)
    dinfo = torch.zeros(1, dtype=torch.int32, device=dev)
    W = dA.clone()
    reps, times = max(1, min(args.steps, 5)), []
    for r in range(reps + 1):
        W.copy_(dA)
        if r == reps:
            lib.skf_profile_read(None, None, None, 1)
            lib.skf_profile_enable(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        skf.ltlt_c128(W, ipiv, T, work, dinfo)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1))
    lib.skf_profile_enable(0)
    pms = (ctypes.c_double * 2)()
    pfl = (ctypes.c_double * 2)()
    pcnt = (ctypes.c_int64 * 2)()
    lib.skf_profile_read(pms, pfl, pcnt, 1)
    assert int(dinfo.item()) == 0
    ms = float(np.median(times))
    b = torch.ones((n, 1), dtype=torch.complex128, device=dev)
    B = skf.colmajor(n, 1, device=dev, dtype=torch.complex128)
    swork = skf.workspace(int(lib.skf_solve_c128_workspace(n, 1)), dev)
    st = []
    for _ in range(3):
        B.copy_(b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        skf.solve_c128(W, ipiv, T, B, swork, dinfo)
        e1.record()
        torch.cuda.synchronize()
        st.append(e0.elapsed_time(e1))
    upd_tf = pfl[1] / (pms[1] * 1e-3) / 1e12 if pms[1] > 0 else 0.0
    return {"ms": round(ms, 3), "gflops_nominal": round(8.0 * n ** 3 / 3.0 / (ms * 1e-3) / 1e9, 1),
            "panel_us_per_step": round(pms[0] * 1e3 / max(n - 1, 1), 3),
            "update_tflops": round(upd_tf, 3), "update_frac_fp64_peak": round(upd_tf / FP64_MFMA_PEAK_TFLOPS, 4),
            "solve_ms_1rhs": round(float(np.median(st)), 3)}


def bench_serve(args):
    """2000-request Poisson trace (seed 8): saturation run, then 0.7 x saturation."""
    import torch

    from paper_2408_05238_amd import serve
    dev = _device()
    count = args.count or 2000
    ex = serve.GpuExecutor(str(dev))
    reqs, mids = serve.make_workload(count, rate_hz=0.0, seed=8)
    serve.materialize(reqs, mids, seed=8, device=dev, threads=16)
    torch.cuda.synchronize()
    # warm the code paths (one request of each kind)
    for r in reqs[:8]:
        ex.run([r], None)
    sch = serve.Scheduler(ex, budget_bytes=64 << 30, workers=8)
    t0 = time.perf_counter()
    sch.run_trace(reqs, t0=t0)
    sat = sch.stats(t0)
    rate = 0.7 * sat["req_per_s"]
    reqs2, _ = serve.make_workload(count, rate_hz=rate, seed=8)
    for a, b in zip(reqs2, reqs):
        a.A, a.B = b.A, b.B
    sch2 = serve.Scheduler(ex, budget_bytes=64 << 30, workers=8)
    t0 = time.perf_counter()
    sch2.run_trace(reqs2, t0=t0)
    st = sch2.stats(t0)
    _line("serving p99 latency at 0.7x saturation (2000 Poisson requests)", round(st["p99_ms"], 3), "ms",
          round(st["mean_ms"], 3), args, "f64 / f32-trailing+refine",
          f"{count} Poisson requests, n log-uniform on [64,4096] (seed 8), 70% FP64 / 30% FP32+refine, "
          f"Pf:solve 50:50, 16 RHS, 64 GB budget", higher=False,
          saturation={k: _sig(v) for k, v in sat.items()},
          at_rate_hz=round(rate, 2),
          serving={k: _sig(v) for k, v in st.items()})


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the factorization is not "
              f"sharded across GPUs in this build.", file=sys.stderr)
        sys.exit(2)
    if args.workload != "ltlt":
        return {"mixed": bench_mixed, "batched": bench_batched, "serve": bench_serve,
                "complex": bench_complex}[args.workload](args)
    import numpy as np
    import torch

    from paper_2408_05238_amd import inputs, skf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lib = skf.lib()  # raises if libskf.so is missing: there is no fallback path
    n = args.n
    prec = skf.PREC_F64 if args.prec == "f64" else skf.PREC_F32_TRAILING
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t_gen = time.perf_counter()
    A = inputs.skew_gaussian(n, args.seed, inputs.STREAM_A)
    t_gen = time.perf_counter() - t_gen
    d0 = skf.to_device_colmajor(A, device=dev)
    nrun = args.warmup + args.steps
    copies = []
    for _ in range(nrun):
        c = skf.colmajor(n, n, device=dev)
        c.copy_(d0)
        copies.append(c)
    work = skf.workspace(skf.ltlt_workspace(n, prec), dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    T = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    dinfo = torch.zeros(nrun, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        skf.ltlt(copies[i], ipiv, T, prec, work, dinfo[i:i + 1])
    torch.cuda.synchronize()

    lib.skf_profile_read(None, None, None, 1)
    lib.skf_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, nrun):
        skf.ltlt(copies[i], ipiv, T, prec, work, dinfo[i:i + 1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.skf_profile_enable(0)
    import ctypes
    ms = (ctypes.c_double * 2)()
    fl = (ctypes.c_double * 2)()
    cnt = (ctypes.c_int64 * 2)()
    lib.skf_profile_read(ms, fl, cnt, 1)

    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    infos = dinfo.cpu().tolist()
    assert all(v == 0 for v in infos), f"factorization reported info {infos}"

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gflops = (n ** 3 / 3.0) / (ms_per_step * 1e-3) / 1e9

    # the Pfaffian-only reduction of the same matrix (outside the timed region):
    # one warm-up, then the median of three event-timed runs
    pf_only = None
    if prec == skf.PREC_F64 and not args.no_side:
        ipiv2 = torch.empty_like(ipiv)
        T2 = torch.empty_like(T)
        dinfo2 = torch.zeros(1, dtype=torch.int32, device=dev)
        times = []
        for r in range(4):
            copies[0].copy_(d0)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            skf.pfonly(copies[0], ipiv2, T2, prec, work, dinfo2)
            e1.record()
            torch.cuda.synchronize()
            if r > 0:
                times.append(e0.elapsed_time(e1))
        la_f, sg_f = skf.logpf_from_factors(n, ipiv, T)
        la_p, sg_p = skf.logpf_from_factors(n, ipiv2, T2)
        la_f, la_p = float(la_f.item()), float(la_p.item())
        pf_ms = sorted(times)[1]
        pf_only = {"ms": round(pf_ms, 3), "speedup_vs_ltlt": round(ms_per_step / pf_ms, 3),
                   "info": int(dinfo2.item()), "sign_equal_ltlt": int(sg_f.item()) == int(sg_p.item()),
                   "logabs_rel_diff_vs_ltlt": abs(la_p - la_f) / max(1.0, abs(la_f))}

    # Pfaffian ratio of a rank-2r skew update through the resident factors of the
    # last timed step (outside the timed region): median of three event-timed
    # calls per r after one warm-up; at r = 1 the ratio is checked against the
    # Pfaffian-only reductions of the updated and the original matrix
    pf_ratio = None
    if prec == skf.PREC_F64 and pf_only is not None:
        LT = copies[nrun - 1]
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed)
        pf_ratio = {}
        for r in (1, 16):
            Ud = torch.randn(r, n, device=dev, dtype=torch.float64, generator=g).t()
            Vd = torch.randn(r, n, device=dev, dtype=torch.float64, generator=g).t()
            wk = skf.workspace(skf.pf_ratio_workspace(n, r), dev)
            di = torch.zeros(1, dtype=torch.int32, device=dev)
            times = []
            for rep in range(4):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                la_r, sg_r, _ = skf.pf_ratio(LT, ipiv, T, Ud, Vd, work=wk, dinfo=di)
                e1.record()
                torch.cuda.synchronize()
                if rep > 0:
                    times.append(e0.elapsed_time(e1))
            ent = {"ms": round(sorted(times)[1], 3), "info": int(di.item()),
                   "speedup_vs_refactorization": round(ms_per_step / sorted(times)[1], 1)}
            if r == 1:
                Bm = copies[0]
                Bm.copy_(d0)
                Bm.add_(Ud @ Vd.t() - Vd @ Ud.t())
                skf.pfonly(Bm, ipiv2, T2, prec, work, dinfo2)
                la_b, sg_b = skf.logpf_from_factors(n, ipiv2, T2)
                direct = float(la_b.item()) - la_p
                ent["logabs"] = float(la_r.item())
                ent["logabs_via_two_pfaffians"] = direct
                ent["abs_diff"] = abs(float(la_r.item()) - direct)
                ent["sign_equal"] = int(sg_r.item()) == int(sg_b.item()) * int(sg_p.item())
            pf_ratio[f"r{r}"] = ent
    del d0

    # parity spot check of the last step against the oracle's stored pivots (same seed)
    parity = None
    gpath = os.path.join(ROOT, "tests", "golden", f"ltlt_n{n}_s{args.seed}.npz")
    if os.path.exists(gpath) and prec == skf.PREC_F64:
        g = np.load(gpath)
        parity = {"pivots_equal_oracle": bool(np.array_equal(ipiv.cpu().numpy(), g["ipiv"])),
                  "max_rel_T_diff": float(np.abs(T[:n - 1].cpu().numpy() - g["T"]).max() / np.abs(g["T"]).max())}

    tr_ms = ms[1] / max(cnt[1], 1)
    tr_tflops = (fl[1] / (ms[1] * 1e-3) / 1e12) if ms[1] > 0 else 0.0
    peak = FP64_MFMA_PEAK_TFLOPS if prec == skf.PREC_F64 else 157.3
    traffic = read_traffic(args.traffic)
    roofline = {"bound": "mfma", "kernel": "skr2k_perm (trailing skew rank-2k update)",
                "achieved": round(tr_tflops, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tr_tflops / peak, 4), "traffic": traffic,
                "launches": int(cnt[1]), "avg_launch_ms": round(tr_ms, 4),
                "flops_per_launch_avg": fl[1] / max(cnt[1], 1)}
    panel = {"ms_per_factorization": round(ms[0] / args.steps, 3),
             "us_per_elimination_step": round(ms[0] * 1e3 / args.steps / max(n - 1, 1), 3),
             "share": round(ms[0] / args.steps / ms_per_step, 3)}

    out = {
        "metric": "LTL^T GFLOP/s (n^3/3) at n=16384 FP64",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == skf.PREC_F64 else "f64 storage, f32 trailing products",
        "data": "synthetic",
        "config": {"workload": f"dense skew-symmetric Gaussian matrix n={n} (seed {args.seed}), blocked "
                               f"partially pivoted LTL^T, {'FP64' if prec == skf.PREC_F64 else 'FP32-trailing'}",
                   "n": n, "prec": args.prec},
        "tuning": {"ltlt_nb": skf.tune_get("ltlt_nb", n), "pfonly_nb": skf.tune_get("pfonly_nb", n),
                   "skr2k_band": skf.tune_get("skr2k_band", n),
                   "table": os.path.relpath(skf.TUNING_PATH, ROOT) if os.path.exists(skf.TUNING_PATH) else None},
        "fraction_of_fp64_peak": round(gflops / 1e3 / FP64_MFMA_PEAK_TFLOPS, 4),
        "roofline": roofline,
        "panel": panel,
        "parity": parity,
        "pfaffian_only": pf_only,
        "pf_ratio_resident_factors": pf_ratio,
        "input_generation_s": round(t_gen, 2),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, n, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

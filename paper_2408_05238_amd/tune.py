"""Tuner: measures the library's block-size and tile-walk choices on the device
and persists the fastest as the tuning table the binding loads
(``paper_2408_05238_amd/tuning/mi355x.json``).

Parameters swept (every candidate runs the same kernels' other code; results
are identical up to rounding, the interchanges bit for bit on generic inputs):
  ltlt_nb     panel width of the full factorization: 64 or 128 (a width of
              256 needs 192 KB of LDS per panel workgroup, more than a CU has)
  pfonly_nb   panel width of the Pfaffian-only reduction: 64 or 128
  skr2k_band  block rows per band of the trailing update's tile walk

Each candidate is timed on a resident seeded Gaussian skew matrix (restored
from a pristine device copy before every repetition, outside the timed region)
with HIP events on the calling stream: one warm-up, then the median of
``reps`` runs.  The table maps ranges of orders to the winner: the boundary
between two measured orders is their geometric mean.

    python -m paper_2408_05238_amd.tune [--sizes 1024,2048,...] [--reps 3] [--out path]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_MAX = 1 << 40
DEFAULT_SIZES = (512, 1024, 2048, 4096, 8192, 16384, 32768)
BANDS = (2, 4, 8, 16, 32)


def _time_call(fn, A0, work, reps):
    """Median milliseconds of fn(A) over reps runs, A restored from A0 before each."""
    import torch
    A = work
    ts = []
    for r in range(reps + 1):
        A.copy_(A0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(A)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def _ranges(choices):
    """[(n, value), ...] sorted by n -> [(lo, hi, value)] covering 0..N_MAX,
    the boundaries at the geometric means of neighbouring measured orders."""
    out = []
    for i, (n, v) in enumerate(choices):
        lo = 0 if i == 0 else int(math.sqrt(choices[i - 1][0] * n)) + 1
        hi = N_MAX if i == len(choices) - 1 else int(math.sqrt(n * choices[i + 1][0]))
        if out and out[-1][2] == v:
            out[-1] = (out[-1][0], hi, v)
        else:
            out.append((lo, hi, v))
    return out


def sweep(sizes=DEFAULT_SIZES, reps=3, band_n=16384, log=print):
    import torch

    from paper_2408_05238_amd import inputs, skf

    lib = skf.lib()
    skf.load_tuning(path="off")        # measure against the built-in rules only
    meas = {"ltlt_nb": {}, "pfonly_nb": {}, "skr2k_band": {}}
    choice = {"ltlt_nb": [], "pfonly_nb": [], "skr2k_band": []}
    os.environ.pop("SKF_NB", None)
    for n in sizes:
        A0 = skf.to_device_colmajor(inputs.skew_gaussian(n, 2, inputs.STREAM_A))
        A = A0.clone()
        for param, call in (("ltlt_nb", skf.ltlt), ("pfonly_nb", skf.pfonly)):
            pid = skf.TUNE_PARAMS[param]
            res = {}
            for nb in (64, 128, 256):
                lib.skf_tune_clear()
                lib.skf_tune_set(pid, 0, N_MAX, nb)
                if lib.skf_tune_get(pid, n) != nb:
                    continue                   # infeasible for this n on this device
                ms = _time_call(lambda X: call(X), A0, A, reps)
                res[nb] = ms
                log(f"{param} n={n} nb={nb}: {ms:.3f} ms")
            lib.skf_tune_clear()
            if res:
                meas[param][str(n)] = {str(k): round(v, 4) for k, v in res.items()}
                choice[param].append((n, min(res, key=res.get)))
        del A, A0
        torch.cuda.empty_cache()
    # band of the trailing update's tile walk, at one order, with the chosen widths
    A0 = skf.to_device_colmajor(inputs.skew_gaussian(band_n, 2, inputs.STREAM_A))
    A = A0.clone()
    res = {}
    pid = skf.TUNE_PARAMS["skr2k_band"]
    for b in BANDS:
        lib.skf_tune_clear()
        for param in ("ltlt_nb",):
            for lo, hi, v in _ranges(choice[param]):
                lib.skf_tune_set(skf.TUNE_PARAMS[param], lo, hi, v)
        lib.skf_tune_set(pid, 0, N_MAX, b)
        ms = _time_call(lambda X: skf.ltlt(X), A0, A, reps)
        res[b] = ms
        log(f"skr2k_band n={band_n} band={b}: {ms:.3f} ms")
    lib.skf_tune_clear()
    meas["skr2k_band"][str(band_n)] = {str(k): round(v, 4) for k, v in res.items()}
    choice["skr2k_band"].append((band_n, min(res, key=res.get)))
    entries = []
    for param in ("ltlt_nb", "pfonly_nb", "skr2k_band"):
        for lo, hi, v in _ranges(choice[param]):
            entries.append({"param": param, "n_lo": lo, "n_hi": hi, "value": int(v)})
    return entries, meas


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default=",".join(str(n) for n in DEFAULT_SIZES))
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--band-n", type=int, default=16384)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "mi355x.json"))
    a = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the tuner measures on the GPU"
    sizes = [int(x) for x in a.sizes.split(",") if x]
    t0 = time.time()
    entries, meas = sweep(sizes, a.reps, a.band_n, log=lambda m: print(m, flush=True))
    table = {"device": torch.cuda.get_device_name(0), "generated_by": "python -m paper_2408_05238_amd.tune "
             + " ".join(argv if argv is not None else sys.argv[1:]),
             "reps": a.reps, "seconds": round(time.time() - t0, 1), "entries": entries,
             "measured_ms": meas}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(f"wrote {a.out}: {len(entries)} entries", flush=True)


if __name__ == "__main__":
    main()

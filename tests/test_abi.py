"""The C ABI library loads and exports every symbol include/skf.h declares;
argument checks that run on the host before any launch (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "skf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(skf_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2408_05238_amd import skf
    if not os.path.exists(skf.LIB_PATH):
        from paper_2408_05238_amd import build
        build.build()
    return skf.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_2408_05238_amd import skf
    decl = _declared()
    assert len(decl) >= 15
    missing = [s for s in decl if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(skf.EXPORTS) == decl


def test_version(lib):
    assert lib.skf_version().decode().startswith("skf")


def test_argument_errors_before_any_launch(lib):
    vp = ctypes.c_void_p
    # skf_ltlt: n < 0, lda < n, null A, bad precision
    assert lib.skf_ltlt(-1, vp(0), 1, vp(0), vp(0), 0, vp(0), 0, vp(0), vp(0)) == -1
    assert lib.skf_ltlt(10, vp(0), 10, vp(8), vp(8), 0, vp(256), 1 << 30, vp(0), vp(0)) == -2
    assert lib.skf_ltlt(10, vp(8), 9, vp(8), vp(8), 0, vp(256), 1 << 30, vp(0), vp(0)) == -3
    assert lib.skf_ltlt(10, vp(8), 10, vp(8), vp(8), 7, vp(256), 1 << 30, vp(0), vp(0)) == -6
    # workspace too small
    assert lib.skf_ltlt(10, vp(8), 10, vp(8), vp(8), 0, vp(256), 16, vp(0), vp(0)) == -104
    # skr2k: negative k, short leading dimension
    assert lib.skf_skr2k(4, -1, 1.0, vp(8), 4, vp(8), 4, 0.0, vp(8), 4, vp(0)) == -2
    assert lib.skf_skr2k(4, 2, 1.0, vp(8), 3, vp(8), 4, 0.0, vp(8), 4, vp(0)) == -5
    # solve: odd sizes are fine to validate; bad ldb
    assert lib.skf_solve(4, 1, vp(8), 4, vp(8), vp(8), vp(8), 3, vp(256), 1 << 20, vp(0), vp(0)) == -8
    # refine: negative tolerance
    it, be = ctypes.c_int(0), ctypes.c_double(0)
    assert lib.skf_solve_refine(4, 1, vp(8), 4, vp(8), 4, vp(8), vp(8), vp(8), 4, vp(8), 4, -1.0, 3,
                                ctypes.byref(it), ctypes.byref(be), vp(256), 1 << 20, vp(0)) == -13


def test_workspace_queries(lib):
    assert lib.skf_ltlt_workspace(16384, 0) >= 16384 * 16384 * 8
    assert lib.skf_ltlt_workspace(-1, 0) == 0
    assert lib.skf_solve_workspace(100, 16) > 0
    assert lib.skf_refine_workspace(100, 16) > lib.skf_solve_workspace(100, 16)


def test_argument_errors_of_the_pfaffian_paths(lib):
    vp = ctypes.c_void_p
    # skf_pfonly: same checks as skf_ltlt
    assert lib.skf_pfonly(-1, vp(0), 1, vp(0), vp(0), 0, vp(0), 0, vp(0), vp(0)) == -1
    assert lib.skf_pfonly(10, vp(8), 9, vp(8), vp(8), 0, vp(256), 1 << 30, vp(0), vp(0)) == -3
    assert lib.skf_pfonly(10, vp(8), 10, vp(8), vp(8), 0, vp(256), 16, vp(0), vp(0)) == -104
    # skf_pf_ratio: rank beyond the maximum, missing outputs, misaligned workspace
    args = [vp(8), 100, vp(8), vp(8), vp(8), 100, vp(8), 100]
    assert lib.skf_pf_ratio(100, 33, *args, vp(8), vp(8), vp(256), 1 << 30, vp(0), vp(0)) == -2
    assert lib.skf_pf_ratio(100, 2, *args, vp(0), vp(8), vp(256), 1 << 30, vp(0), vp(0)) == -11
    assert lib.skf_pf_ratio(100, 2, *args, vp(8), vp(8), vp(260), 1 << 30, vp(0), vp(0)) == -13
    assert lib.skf_pf_ratio_workspace(100, 33) == 0
    assert lib.skf_pf_ratio_workspace(100, 32) > 0
    # complex: short lda, null T, small workspace
    assert lib.skf_pfonly_c128(10, vp(8), 9, vp(8), vp(8), vp(256), 1 << 30, vp(0), vp(0)) == -3
    assert lib.skf_pfonly_c128(10, vp(8), 10, vp(8), vp(0), vp(256), 1 << 30, vp(0), vp(0)) == -5
    assert lib.skf_pfonly_c128(10, vp(8), 10, vp(8), vp(8), vp(256), 16, vp(0), vp(0)) == -104
    assert lib.skf_pfonly_c128_workspace(1000) >= 1000 * 1000 * 16
    assert lib.skf_logpf_c128_from_factors(4, vp(8), vp(8), vp(0), vp(8), vp(0)) == -4


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_solve_noalloc_rejects_beyond_scratch(lib):
    """n above the fixed scratch's limit is refused on the host, before any HIP call."""
    vp = ctypes.c_void_p
    from paper_2408_05238_amd import skf
    n = skf.SOLVE_NOALLOC_MAX_N + 2
    assert lib.skf_solve_noalloc(n, 1, vp(8), n, vp(8), vp(8), vp(8), n, vp(0), vp(0)) == skf.ESCRATCH
    assert b"4096" in lib.skf_last_error()
    assert lib.skf_solve_noalloc(-1, 1, vp(8), 4, vp(8), vp(8), vp(8), 4, vp(0), vp(0)) == -1
    assert lib.skf_solve_noalloc(4, 1, vp(8), 4, vp(8), vp(8), vp(8), 3, vp(0), vp(0)) == -8

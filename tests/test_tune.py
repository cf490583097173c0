"""Tuning table: loader, precedence, feasibility and the tuner's range
construction (host only; no GPU needed)."""
from __future__ import annotations

import json
import os

import pytest


@pytest.fixture()
def skf(monkeypatch):
    from paper_2408_05238_amd import skf as s
    if not os.path.exists(s.LIB_PATH):
        from paper_2408_05238_amd import build
        build.build()
    s.lib()
    monkeypatch.delenv("SKF_NB", raising=False)
    yield s
    s.load_tuning()    # back to the default table


def _write(tmp_path, entries):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"entries": entries}))
    return str(p)


def test_builtin_rules_without_table(skf):
    assert skf.load_tuning(path="off") == 0
    assert skf.tune_get("ltlt_nb", 16384) == 128      # 256 panel workgroups fit one per CU
    assert skf.tune_get("ltlt_nb", 32768) == 128      # 512 workgroups: two per CU at width 128
    assert skf.tune_get("pfonly_nb", 1000) == 128
    assert skf.tune_get("skr2k_band", 16384) == 8
    # wider orders take the narrower panels (more of their workgroups fit a CU;
    # here without a device: by LDS alone, 2 / 4 / 6 / 6 per CU at widths
    # 128 / 64 / 32 / 16 on 256 CUs, at most six per CU for any width)
    assert skf.tune_get("ltlt_nb", 40000) == 64
    assert skf.tune_get("ltlt_nb", 65537) == 64       # 1024 workgroups
    assert skf.tune_get("ltlt_nb", 65538) == 32
    assert skf.tune_get("ltlt_nb", 98305) == 32       # 1536 workgroups
    assert skf.tune_get("ltlt_nb", 98306) == 0        # no width fits
    assert skf.tune_get("pfonly_nb", 98305) == 32
    assert skf.tune_get("pfonly_nb", 30000) == 128    # the Pfaffian-only panel's LDS fits two per CU


def test_table_entries_and_precedence(skf, tmp_path):
    path = _write(tmp_path, [
        {"param": "ltlt_nb", "n_lo": 0, "n_hi": 4000, "value": 64},
        {"param": "ltlt_nb", "n_lo": 2000, "n_hi": 3000, "value": 128},   # later entry wins on its range
        {"param": "pfonly_nb", "n_lo": 0, "n_hi": 10 ** 9, "value": 64},
        {"param": "skr2k_band", "n_lo": 100, "n_hi": 10 ** 9, "value": 16},
    ])
    assert skf.load_tuning(path) == 4
    assert skf.tune_get("ltlt_nb", 1000) == 64
    assert skf.tune_get("ltlt_nb", 2500) == 128
    assert skf.tune_get("ltlt_nb", 3500) == 64
    assert skf.tune_get("ltlt_nb", 5000) == 128       # not covered: built-in rule
    assert skf.tune_get("pfonly_nb", 16384) == 64
    assert skf.tune_get("skr2k_band", 50) == 8
    assert skf.tune_get("skr2k_band", 500) == 16


def test_width_256_only_where_one_workgroup_per_cu_suffices(skf, tmp_path):
    # 130 KB of LDS per panel workgroup: one per CU, 256 workgroups of 64 rows
    skf.load_tuning(_write(tmp_path, [{"param": "ltlt_nb", "n_lo": 0, "n_hi": 10 ** 9, "value": 256},
                                      {"param": "pfonly_nb", "n_lo": 0, "n_hi": 10 ** 9, "value": 256}]))
    assert skf.tune_get("ltlt_nb", 16384) == 256
    assert skf.tune_get("ltlt_nb", 16385) == 256
    assert skf.tune_get("ltlt_nb", 16386) == 128      # 257 workgroups: the built-in rule
    assert skf.tune_get("pfonly_nb", 16385) == 256
    assert skf.tune_get("pfonly_nb", 20000) == 128


def test_infeasible_entry_is_ignored_and_env_overrides(skf, tmp_path, monkeypatch):
    skf.load_tuning(_write(tmp_path, [{"param": "ltlt_nb", "n_lo": 0, "n_hi": 10 ** 9, "value": 128}]))
    assert skf.tune_get("ltlt_nb", 40000) == 64       # 625 workgroups of width 128 cannot be resident
    monkeypatch.setenv("SKF_NB", "64")
    assert skf.tune_get("ltlt_nb", 1000) == 64
    assert skf.tune_get("pfonly_nb", 1000) == 64


def test_bad_entries_are_rejected(skf, tmp_path):
    lib = skf.lib()
    assert lib.skf_tune_set(7, 0, 10, 64) == -1
    assert lib.skf_tune_set(0, -1, 10, 64) == -2
    assert lib.skf_tune_set(0, 10, 9, 64) == -3
    assert lib.skf_tune_set(0, 0, 10, 512) == -4      # no panel of width 512
    assert lib.skf_tune_set(0, 0, 10, 256) == 0
    assert lib.skf_tune_set(2, 0, 10, 0) == -4
    assert lib.skf_tune_get(9, 100) == -1
    with pytest.raises(ValueError):
        skf.load_tuning(_write(tmp_path, [{"param": "ltlt_nb", "n_lo": 0, "n_hi": 10, "value": 96}]))


def test_ranges_cover_all_orders():
    from paper_2408_05238_amd.tune import N_MAX, _ranges
    r = _ranges([(1024, 64), (4096, 64), (16384, 128), (32768, 64)])
    assert r[0][0] == 0 and r[-1][1] == N_MAX
    assert [v for _, _, v in r] == [64, 128, 64]
    for (a, b, _), (c, d, _) in zip(r, r[1:]):
        assert c == b + 1
    assert r[0][1] == int((4096 * 16384) ** 0.5)


def test_committed_table_loads(skf):
    if not os.path.exists(skf.TUNING_PATH):
        pytest.skip("no tuning table committed")
    n = skf.load_tuning(skf.TUNING_PATH)
    assert n >= 3
    t = json.load(open(skf.TUNING_PATH))
    assert {e["param"] for e in t["entries"]} == set(skf.TUNE_PARAMS)

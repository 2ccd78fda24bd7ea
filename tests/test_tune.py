"""Autotuner cache handling on the CPU (no GPU timing here)."""
import json

import pytest

import paper_2307_06554_amd as pm
from paper_2307_06554_amd import tune


def test_candidates():
    assert tune.candidates(16) == [16]
    assert tune.candidates(32) == [32]
    assert tune.candidates(64) == [16, 32, 64]
    assert tune.candidates(512) == [16, 32, 64, 128]
    assert tune.candidates(4096) == [32, 64, 128]


def _cache(**kw):
    rec = {"version": tune.CACHE_VERSION, "arch": "gfx950", "csrc_hash": tune.csrc_hash(),
           "tiles": [{"n": 2048, "L": 4, "t": 128}],
           "karatsuba": [{"n": 4096, "products": 2048, "depth": 3}],
           "karatsuba64": [{"n": 65536, "products": 16, "depth": 2}],
           "params": {"plan_share_pct": 160, "plan_stream_pct": 150, "u64_karatsuba_runs": 2}}
    rec.update(kw)
    return json.dumps(rec)


def _reset():
    pm.polymul_tune_set(2048, 4, 0)
    pm.polymul_tune_set_karatsuba(4096, 2048, 4, pm.binding.KARATSUBA_BUILTIN)
    pm.polymul_tune_set_karatsuba(65536, 16, 8, pm.binding.KARATSUBA_BUILTIN)
    pm.polymul_tune_param_set("plan_share_pct", 140)
    pm.polymul_tune_param_set("plan_stream_pct", 125)
    pm.polymul_tune_param_set("u64_karatsuba_runs", 4)


def test_corrupt_stale_or_foreign_cache_is_ignored(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    p = tmp_path / "c.json"
    p.write_text("{not json")
    assert tune.apply(str(p)) is False
    p.write_text(_cache(arch="gfx942"))
    assert tune.apply(str(p)) is False
    p.write_text(_cache(csrc_hash="0123456789abcdef"))  # taken on other kernel sources
    assert tune.apply(str(p)) is False
    p.write_text(_cache(version=1))
    assert tune.apply(str(p)) is False
    assert pm.polymul_tune_get(2048, 4) == 64
    assert pm.polymul_tune_get_karatsuba(4096, 2048, 4) == 2
    assert pm.polymul_tune_param_get("plan_share_pct") == 140
    p.write_text(_cache(tiles=[{"n": 4096, "L": 4, "t": 48}]))
    try:
        assert tune.apply(str(p)) is False
        with pytest.raises(pm.PolymulError):
            tune.apply(str(p), strict=True)
    finally:
        _reset()


def test_cache_is_applied(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    p = tmp_path / "c.json"
    p.write_text(_cache())
    try:
        assert tune.apply(str(p)) is True
        assert pm.polymul_tune_get(2048, 4) == 128
        assert pm.polymul_tune_get_karatsuba(4096, 2048, 4) == 3
        assert pm.polymul_tune_get_karatsuba(65536, 16, 8) == 2
        assert pm.polymul_tune_param_get("plan_share_pct") == 160
        assert pm.polymul_tune_param_get("plan_stream_pct") == 150
        assert pm.polymul_tune_param_get("u64_karatsuba_runs") == 2
    finally:
        _reset()



def test_pick_keeps_the_builtin_choice_within_the_margin():
    assert tune.pick({32: 100.0, 64: 99.5, 128: 101.0}, 64) == 64
    assert tune.pick({32: 99.5, 64: 100.0}, 64) == 64        # 0.5% faster: noise
    assert tune.pick({32: 98.0, 64: 100.0}, 64) == 32        # 2% faster
    assert tune.pick({"0": 50.0, "3/4": 40.0, "3/2": 39.9}, "3/4") == "3/4"
    assert tune.pick({16: 80.0, 32: 100.0}, 48) == 16         # default not measured: the fastest

"""Autotuner cache handling on the CPU (no GPU timing here)."""
import json

import pytest

import paper_2307_06554_amd as pm
from paper_2307_06554_amd import tune


def test_candidates():
    assert tune.candidates(16) == [16]
    assert tune.candidates(64) == [32, 64]
    assert tune.candidates(4096) == [32, 64, 128]


def test_corrupt_or_foreign_cache_is_ignored(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    p = tmp_path / "c.json"
    p.write_text("{not json")
    assert tune.apply(str(p)) is False
    p.write_text(json.dumps({"version": 1, "arch": "gfx942", "entries": [{"n": 4096, "L": 4, "t": 128}]}))
    assert tune.apply(str(p)) is False
    assert pm.polymul_tune_get(4096, 4) == 64
    p.write_text(json.dumps({"version": 1, "arch": "gfx950", "entries": [{"n": 4096, "L": 4, "t": 48}]}))
    assert tune.apply(str(p)) is False
    with pytest.raises(pm.PolymulError):
        tune.apply(str(p), strict=True)


def test_cache_is_applied(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    p = tmp_path / "c.json"
    p.write_text(json.dumps({"version": 1, "arch": "gfx950", "entries": [{"n": 2048, "L": 4, "t": 128}]}))
    try:
        assert tune.apply(str(p)) is True
        assert pm.polymul_tune_get(2048, 4) == 128
    finally:
        pm.polymul_tune_set(2048, 4, 0)

"""bench.py's host-side logic on the CPU: the one-GPU rule, the oracle baseline's
word-for-word check of the timed output, and the gating of the committed
profile figures by the kernel-source hash.  No GPU is touched."""
import importlib.util
import json
import os
import subprocess
import sys
import types

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def _workload(seed=3, pairs=3, n=64):
    rng = np.random.Generator(np.random.PCG64(seed))
    qs = [1068236801, 1068212225]
    a = np.stack([rng.integers(0, q, size=(pairs, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(pairs, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    return types.SimpleNamespace(a=a, b=b, qs=qs)


def test_cpu_baseline_checks_the_timed_output_word_for_word():
    bench = _bench()
    w = _workload()
    good = oracle.negacyclic_rns(w.a, w.b, w.qs)
    base, parity = bench.cpu_baseline(w, 2.0, good)
    assert parity["bit_exact"] and parity["mismatches"] == 0
    assert parity["checked_products"] == parity["of_products"] == 6
    assert parity["checked_words"] == 6 * 64
    assert base["kind"] == "oracle" and base["value"] > 0 and base["cores"] >= 1
    bad = good.copy()
    bad[2, 1, 17] ^= 1
    _, parity = bench.cpu_baseline(w, 2.0, bad)
    assert parity["mismatches"] == 1 and not parity["bit_exact"]


def test_profile_figures_only_for_the_sources_they_were_taken_on(monkeypatch):
    bench = _bench()
    from paper_2307_06554_amd import tune
    with open(os.path.join(ROOT, "profiles", "traffic_mfma32_group_kernel_n4096_rns8.json")) as f:
        traffic = json.load(f)
    with open(os.path.join(ROOT, "profiles", "counters_mfma_lds_n4096_rns8.json")) as f:
        counters = json.load(f)
    monkeypatch.setattr(tune, "csrc_hash", lambda: traffic["csrc_hash"])
    assert bench.measured_traffic() == traffic["hbm_bytes_per_launch"]
    monkeypatch.setattr(tune, "csrc_hash", lambda: counters["csrc_hash"])
    assert bench.measured_mfma_busy() == counters["mfma_busy"]
    monkeypatch.setattr(tune, "csrc_hash", lambda: "0000000000000000")
    assert bench.measured_traffic() is None
    assert bench.measured_mfma_busy() is None


def test_preheat_route_choices():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--preheat-route", "ntt"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2 and "invalid choice" in res.stderr

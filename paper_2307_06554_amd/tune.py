"""Autotuner for the Toeplitz tile side of the LDS-resident 32-bit path.

The paper picks its matrix dimension by experiment (Sec. 2.6, matrix dimension
selection); here the experiment is automated: for each degree bound n and limb
count L, every allowed tile side t (n = t * r) is timed on the GPU on a batch
large enough to fill it, and the fastest is kept.  Results go to a JSON cache
keyed by the GPU architecture; `apply()` loads a cache into the library
(polymul_tune_set), so later launches and plans use the tuned tiles.

    python -m paper_2307_06554_amd.tune [--out PATH] [--ns 256,1024,4096]
"""
import argparse
import json
import os
import sys

from . import binding

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
CACHE_VERSION = 1


def candidates(n):
    if n <= 32:
        return [n]
    return [t for t in (32, 64, 128) if t <= n]


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def time_tile(n, L, t, products, reps=30, warm_s=0.25, trials=3):
    """Microseconds per batched launch of `products` products of degree bound n:
    best of `trials` runs of `reps` launches, each after `warm_s` seconds of
    untimed launches (the shader clock settles under sustained load)."""
    import numpy as np
    import torch
    q = {2: 65521, 3: 16777213, 4: 1068236801}[L]
    rng = np.random.Generator(np.random.PCG64(n + t))
    a = torch.from_numpy(rng.integers(0, q, size=(products, n), dtype=np.int64).astype(np.int32)).cuda()
    b = torch.from_numpy(rng.integers(0, q, size=(products, n), dtype=np.int64).astype(np.int32)).cuda()
    c = torch.empty_like(a)
    import time
    binding.polymul_tune_set(n, L, t)
    try:
        best = None
        for _ in range(trials):
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < warm_s:
                for _ in range(10):
                    binding.polymul_negacyclic(a, b, q, out=c)
                torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                binding.polymul_negacyclic(a, b, q, out=c)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1000.0 / reps
            best = us if best is None else min(best, us)
        return best
    finally:
        binding.polymul_tune_set(n, L, 0)


def tune(ns=(256, 512, 1024, 2048, 4096, 8192), Ls=(4,), work=2 ** 35, out=DEFAULT_CACHE, log=print):
    """Time every candidate; `work` sets the batch so products * n^2 ~ work
    (2^35: 2048 products at n = 4096, several rounds of workgroups per CU)."""
    entries = []
    for L in Ls:
        for n in ns:
            products = max(64, min(65536, work // (n * n)))
            best = None
            timings = {}
            for t in candidates(n):
                try:
                    us = time_tile(n, L, t, products)
                except binding.PolymulError:
                    continue
                timings[t] = us
                if best is None or us < timings[best]:
                    best = t
            log(f"n={n:6d} L={L} products={products:6d} " +
                " ".join(f"t={t}:{us:8.1f}us" for t, us in timings.items()) + f"  -> t={best}")
            entries.append({"n": n, "L": L, "t": best, "us": timings[best], "products": products,
                            "timings_us": {str(k): v for k, v in timings.items()}})
    rec = {"version": CACHE_VERSION, "arch": _arch(), "entries": entries}
    if out:
        with open(out + ".tmp", "w") as f:
            json.dump(rec, f, indent=1)
        os.replace(out + ".tmp", out)
    return rec


def apply(path=None, strict=False):
    """Load a tune cache into the library.  A missing, corrupt, stale or
    other-architecture cache leaves the built-in tiles (returns False)."""
    path = path or os.environ.get("POLYMUL_TUNE_CACHE", DEFAULT_CACHE)
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("version") != CACHE_VERSION:
            raise ValueError("cache version")
        if rec.get("arch") != _arch():
            raise ValueError("cache is for another GPU architecture")
        for e in rec["entries"]:
            binding.polymul_tune_set(int(e["n"]), int(e["L"]), int(e["t"]))
        return True
    except (OSError, ValueError, KeyError, TypeError, binding.PolymulError) as exc:
        if strict:
            raise
        print(f"polymul tune cache not used ({path}): {exc}", file=sys.stderr)
        return False


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--ns", default="256,512,1024,2048,4096,8192")
    ap.add_argument("--L", default="4")
    args = ap.parse_args()
    tune(tuple(int(x) for x in args.ns.split(",")), tuple(int(x) for x in args.L.split(",")), out=args.out)


if __name__ == "__main__":
    main()

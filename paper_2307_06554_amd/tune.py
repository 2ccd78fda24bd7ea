"""Autotuner: the parameters of the library that move time, found by experiment.

The paper picks its matrix dimension by experiment (Sec. 2.6, matrix dimension
selection) and names Karatsuba as a further improvement (Sec. 4); here the
experiments are automated and their winners loaded into the library:

  - the Toeplitz tile side t of the resident 32-bit path per degree bound n
    (16: the 16x16-tile kernel; 32, 64, 128: 32x32 tiles), polymul_tune_set;
  - the Karatsuba depth per degree bound and batch (the direct route included),
    for 32-bit RNS products and for 64-bit words, polymul_tune_set_karatsuba;
  - the K-run cap of the 64-bit Karatsuba route and the two scheduling knobs of
    grouped plans (split threshold, weight of streamed blocks),
    polymul_tune_param_set.

Every candidate is timed on the GPU on a batch large enough to fill it, best of
three runs after the shader clock has settled; a candidate replaces the built-in
choice only if it is more than MARGIN faster (closer timings are noise, and a
cache that flips between equals would move every figure taken with it).  Results
go to a JSON cache keyed
by the GPU architecture and by a hash of the kernel sources: a cache taken on
other sources or another GPU is ignored, and the built-in choices stay.

    python -m paper_2307_06554_amd.tune [--out PATH] [--quick]
"""
import argparse
import hashlib
import json
import os
import sys
import time

from . import binding

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")
CACHE_VERSION = 2
MARGIN = 0.01
Q30 = 1068236801
GOLDILOCKS = (1 << 64) - (1 << 32) + 1


def csrc_hash():
    """Hash of the library's kernel and host sources (what a measurement was taken on)."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def pick(timings, default, margin=MARGIN):
    """The fastest key of `timings`, or `default` unless that is beaten by more than `margin`."""
    best = min(timings, key=timings.get)
    if default in timings and timings[best] > timings[default] * (1.0 - margin):
        return default
    return best


def candidates(n):
    if n <= 32:
        return [n]
    small = [16] if 64 <= n <= 512 else []
    return small + [t for t in (32, 64, 128) if t <= n]


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def time_us(fn, reps=30, warm_s=0.25, trials=3):
    """Best of `trials` averages over `reps` calls, each after `warm_s` s of untimed calls."""
    import torch
    best = None
    for _ in range(trials):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < warm_s:
            for _ in range(10):
                fn()
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1000.0 / reps
        best = us if best is None else min(best, us)
    return best


def _rand(shape, q, seed, dtype_bits=32):
    import numpy as np
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    if dtype_bits == 32:
        return torch.from_numpy(rng.integers(0, q, size=shape, dtype=np.int64).astype(np.int32)).cuda()
    return torch.from_numpy(rng.integers(0, q, size=shape, dtype=np.uint64).view(np.int64)).cuda()


def tune_tiles(ns, Ls, work, log):
    entries = []
    for L in Ls:
        q = {2: 65521, 3: 16777213, 4: Q30}[L]
        for n in ns:
            products = max(64, min(65536, work // (n * n)))
            a, b = _rand((products, n), q, n), _rand((products, n), q, n + 1)
            c = a.clone()
            timings = {}
            for t in candidates(n):
                binding.polymul_tune_set(n, L, t)
                try:
                    timings[t] = time_us(lambda: binding.polymul_negacyclic(a, b, q, out=c))
                except binding.PolymulError as exc:
                    log(f"tile n={n} L={L} t={t}: {exc}")
                    continue
                finally:
                    binding.polymul_tune_set(n, L, 0)
            if not timings:
                continue
            best = pick(timings, binding.polymul_tune_get(n, L))
            log(f"tile n={n:6d} L={L} products={products:6d} " +
                " ".join(f"t={t}:{us:8.1f}us" for t, us in timings.items()) + f"  -> t={best}")
            entries.append({"n": n, "L": L, "t": best, "products": products,
                            "timings_us": {str(k): v for k, v in timings.items()}})
            binding.polymul_tune_set(n, L, best)  # later experiments run on the tuned tiles
    return entries


def tune_karatsuba(shapes, log):
    """32-bit RNS products: (n, channels, batch) shapes; depth 0 = the direct route."""
    import torch
    entries = []
    for n, L, batch in shapes:
        qs = [Q30] * L
        a, b = _rand((batch, L, n), Q30, n + 7), _rand((batch, L, n), Q30, n + 8)
        c = a.clone()
        timings = {0: time_us(lambda: binding.polymul_negacyclic_rns(a, b, qs, out=c))}
        for d in (1, 2, 3):
            if (n >> d) < 4:
                continue
            ws = torch.empty(max(16, binding.polymul_karatsuba_workspace_size(n, L, batch, d)), dtype=torch.uint8,
                             device="cuda")
            timings[d] = time_us(lambda: binding.polymul_negacyclic_rns_karatsuba(a, b, qs, d, workspace=ws, out=c))
            del ws
        binding.polymul_tune_set_karatsuba(n, batch * L, 4, binding.KARATSUBA_BUILTIN)
        best = pick(timings, binding.polymul_tune_get_karatsuba(n, batch * L, 4))
        log(f"karatsuba n={n:6d} products={batch * L:6d} " +
            " ".join(f"d={d}:{us:8.1f}us" for d, us in timings.items()) + f"  -> depth {best}")
        entries.append({"n": n, "products": batch * L, "depth": best,
                        "timings_us": {str(k): v for k, v in timings.items()}})
        binding.polymul_tune_set_karatsuba(n, batch * L, 4, best)
    return entries


def tune_karatsuba64(shapes, log):
    """64-bit words (Goldilocks): depth 0..3 and the K-run cap of the streamed sub-products."""
    import torch
    entries = []
    best_runs = 4
    for n, batch in shapes:
        a, b = _rand((batch, n), GOLDILOCKS, n + 9, 64), _rand((batch, n), GOLDILOCKS, n + 10, 64)
        c = a.clone()
        timings = {"0": time_us(lambda: binding.polymul_negacyclic_u64(a, b, GOLDILOCKS, out=c), reps=4,
                                trials=2)}
        for d in (1, 2, 3):
            ws = torch.empty(max(16, binding.polymul_karatsuba_u64_workspace_size(n, batch, d)), dtype=torch.uint8,
                             device="cuda")
            for runs in (1, 2, 4):
                binding.polymul_tune_param_set("u64_karatsuba_runs", runs)
                timings[f"{d}/{runs}"] = time_us(
                    lambda: binding.polymul_negacyclic_u64_karatsuba(a, b, GOLDILOCKS, d, workspace=ws, out=c),
                    reps=4, trials=2)
            del ws
        binding.polymul_tune_param_set("u64_karatsuba_runs", 4)
        binding.polymul_tune_set_karatsuba(n, batch, 8, binding.KARATSUBA_BUILTIN)
        d0 = binding.polymul_tune_get_karatsuba(n, batch, 8)
        key = pick(timings, "0" if d0 == 0 else f"{d0}/4")
        depth, runs = (0, 4) if key == "0" else (int(key.split("/")[0]), int(key.split("/")[1]))
        log(f"karatsuba64 n={n:6d} products={batch:4d} " +
            " ".join(f"{k}:{us:8.1f}us" for k, us in timings.items()) + f"  -> depth {depth}, runs {runs}")
        entries.append({"n": n, "products": batch, "depth": depth, "runs": runs, "timings_us": timings})
        binding.polymul_tune_set_karatsuba(n, batch, 8, depth)
        best_runs = runs
    return entries, best_runs


def tune_plan(log):
    """Grouped-plan knobs on the uneven batch (2048 x 256, 512 x 1024, 128 x 2048,
    64 x 4096, 16 x 8192 at 30-bit q)."""
    import torch
    groups = []
    for i, (count, n) in enumerate(((2048, 256), (512, 1024), (128, 2048), (64, 4096), (16, 8192))):
        a, b = _rand((count, n), Q30, 100 + i), _rand((count, n), Q30, 200 + i)
        groups.append((a, b, torch.empty_like(a), n, Q30))
    timings = {}
    for share in (50, 70, 100, 140, 200):
        for stream in (100, 125, 150, 200):
            binding.polymul_tune_param_set("plan_share_pct", share)
            binding.polymul_tune_param_set("plan_stream_pct", stream)
            plan = binding.Plan(groups)
            timings[f"{share}/{stream}"] = time_us(plan.execute, reps=50)
            plan.close()
    key = pick(timings, "140/125")
    share, stream = (int(x) for x in key.split("/"))
    binding.polymul_tune_param_set("plan_share_pct", share)
    binding.polymul_tune_param_set("plan_stream_pct", stream)
    log("plan " + " ".join(f"{k}:{us:6.1f}us" for k, us in timings.items()) + f"  -> share {share}%, stream {stream}%")
    return {"plan_share_pct": share, "plan_stream_pct": stream, "timings_us": timings}


def tune(out=DEFAULT_CACHE, quick=False, log=print):
    binding.load_library()
    ns = (256, 512, 1024, 2048, 4096, 8192) if not quick else (256, 1024, 4096)
    rec = {"version": CACHE_VERSION, "arch": _arch(), "csrc_hash": csrc_hash()}
    rec["tiles"] = tune_tiles(ns, (4, 2), 2 ** 35, log)
    kshapes = ((1024, 8, 256), (2048, 8, 256), (4096, 8, 256), (4096, 8, 32), (8192, 8, 64))
    rec["karatsuba"] = tune_karatsuba(kshapes if not quick else kshapes[2:3], log)
    rec["karatsuba64"], runs = tune_karatsuba64(((65536, 16),), log)
    rec["params"] = {"u64_karatsuba_runs": runs}
    plan = tune_plan(log)
    rec["params"]["plan_share_pct"] = plan["plan_share_pct"]
    rec["params"]["plan_stream_pct"] = plan["plan_stream_pct"]
    rec["plan_timings_us"] = plan["timings_us"]
    if out:
        with open(out + ".tmp", "w") as f:
            json.dump(rec, f, indent=1)
        os.replace(out + ".tmp", out)
    return rec


def apply(path=None, strict=False):
    """Load a tune cache into the library.  A missing, corrupt or stale cache (other
    version, GPU architecture or kernel sources) leaves the built-in choices and
    returns False."""
    path = path or os.environ.get("POLYMUL_TUNE_CACHE", DEFAULT_CACHE)
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("version") != CACHE_VERSION:
            raise ValueError("cache version")
        if rec.get("arch") != _arch():
            raise ValueError("cache is for another GPU architecture")
        if rec.get("csrc_hash") != csrc_hash():
            raise ValueError("cache was taken on other kernel sources")
        for e in rec["tiles"]:
            binding.polymul_tune_set(int(e["n"]), int(e["L"]), int(e["t"]))
        for e in rec.get("karatsuba", []):
            binding.polymul_tune_set_karatsuba(int(e["n"]), int(e["products"]), 4, int(e["depth"]))
        for e in rec.get("karatsuba64", []):
            binding.polymul_tune_set_karatsuba(int(e["n"]), int(e["products"]), 8, int(e["depth"]))
        for name, value in rec.get("params", {}).items():
            binding.polymul_tune_param_set(name, int(value))
        return True
    except (OSError, ValueError, KeyError, TypeError, binding.PolymulError) as exc:
        if strict:
            raise
        print(f"polymul tune cache not used ({path}): {exc}", file=sys.stderr)
        return False


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    tune(out=args.out, quick=args.quick)


if __name__ == "__main__":
    main()

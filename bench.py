#!/usr/bin/env python3
"""Throughput of the split-limb int8-MFMA negacyclic product on one MI355X.

One step = one pass of the whole path over one batch: the n = 4096 RNS workload
(256 ciphertext-like pairs x 8 residue channels with distinct 30-bit primes
q_i = 1 mod 2n, i.e. 2048 independent limb-products) through
polymul_negacyclic_rns, inputs already resident in HBM.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "negacyclic polymuls/sec at n=4096 30-bit q (int8-MFMA vs plain int); % int8 peak"
PEAK_INT8_TOPS = 5000.0      # MI355X dense int8 MFMA, published
PEAK_HBM_GBS = 8000.0
WORKLOAD_INDEX = 2


def csrc_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2307_06554_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, only if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_name}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("csrc_hash") != csrc_hash():
        return None
    return rec.get("bytes_per_launch")


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(w, budget_s):
    """The oracle, as it is, on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    q = w.qs[0]
    a, b = w.a[:, 0], w.b[:, 0]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on one product, then size the sample to about budget_s seconds
    t0 = time.perf_counter()
    oracle.negacyclic(a[:1], b[:1], q)
    one = time.perf_counter() - t0
    count = int(max(1, min(a.shape[0], budget_s / max(one, 1e-6) * min(cores, 8))))
    t0 = time.perf_counter()
    oracle.negacyclic(a[:count], b[:count], q)
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "polymuls/s", "cores": cores, "kind": "oracle",
            "sample": f"{count} products of channel 0 (n=4096, q={q}), {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=150,
                    help="untimed steps; the shader clock settles within about 100 launches")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the products are independent and this build has no "
              "multi-GPU path (see DESIGN.md for how it would shard). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2307_06554_amd as pm
    from paper_2307_06554_amd import inputs

    pm.load_library()
    dev = torch.device("cuda:0")
    w = inputs.make_workload(WORKLOAD_INDEX)
    B, L, n = w.a.shape
    products = B * L
    a = torch.from_numpy(w.a.view(np.int32)).to(dev)
    b = torch.from_numpy(w.b.view(np.int32)).to(dev)
    c = torch.empty_like(a)
    stream = torch.cuda.current_stream()

    ms = time_steps(lambda: pm.polymul_negacyclic_rns(a, b, w.qs, out=c), args.steps, args.warmup, stream)
    value = products / (ms / 1e3)

    # plain integer kernel on the same inputs, one channel at a time (same total work);
    # channel slices are copied once up front so the timed region holds only the kernel
    chans = [(a[:, l].contiguous(), b[:, l].contiguous(), q) for l, q in enumerate(w.qs)]
    cp = torch.empty((B, n), dtype=torch.int32, device=dev)

    def plain_run():
        for aa, bb, q in chans:
            pm.polymul_negacyclic_plain(aa, bb, q, out=cp)
    psteps = max(1, min(args.steps, 5))
    ms_plain = time_steps(plain_run, psteps, 1, stream)
    plain_value = products / (ms_plain / 1e3)

    Lm = 4  # int8 limbs per operand for a 30-bit modulus
    ops_per_product = 2 * Lm * Lm * n * n
    achieved_tops = ops_per_product * products / (ms / 1e3) / 1e12
    traffic = measured_traffic("mfma32_resident_kernel_L4")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "polymuls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "rns_channels": L, "pairs": B, "products_per_step": products,
                   "q_bits": 30, "limbs": Lm},
        "roofline": {"bound": "mfma", "achieved": achieved_tops, "peak": PEAK_INT8_TOPS, "unit": "TFLOP/s",
                     "frac": achieved_tops / PEAK_INT8_TOPS, "traffic": traffic},
        "plain_int": {"value": plain_value, "unit": "polymuls/s", "ms_per_step": ms_plain,
                      "mfma_speedup": value / plain_value},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

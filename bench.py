#!/usr/bin/env python3
"""Throughput of the split-limb int8-MFMA negacyclic product on one MI355X.

One step = one pass of the whole path over one batch: the n = 4096 RNS workload
(256 ciphertext-like pairs x 8 residue channels with distinct 30-bit primes
q_i = 1 mod 2n, i.e. 2048 independent limb-products) through
polymul_negacyclic_rns, inputs already resident in HBM.  Prints one JSON line
on stdout.  The same batch also goes through the Karatsuba route
(polymul_negacyclic_rns_karatsuba), the shared-operand route with one b per
channel (polymul_negacyclic_rns_shared) and the paper's small-modulus RNS with
CRT (polymul_negacyclic_rns_crt), all reported beside the headline, and the
plain integer kernel.  --all also times the other workloads (to stderr).
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "negacyclic polymuls/sec at n=4096 30-bit q (int8-MFMA vs plain int); % int8 peak"
PEAK_INT8_TOPS = 5000.0      # MI355X dense int8 MFMA, published
WORKLOAD_INDEX = 2
KERNEL = "mfma32_group_kernel<4,false>"


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    --pmc summary, only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_mfma32_group_kernel_n4096_rns8.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2307_06554_amd.tune import csrc_hash
    if rec.get("csrc_hash") != csrc_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_mfma_busy():
    """Share of the dominant kernel's cycles with its MFMA units busy, from the committed
    rocprofv3 counter summary, only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters_mfma_lds_n4096_rns8.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2307_06554_amd.tune import csrc_hash
    if rec.get("csrc_hash") != csrc_hash():
        return None
    return rec.get("mfma_busy")


def preheat(fn, seconds):
    """Run fn (untimed) for at least `seconds` of wall clock; returns (launches, seconds).
    The shader clock of a cold GPU takes a few hundred launches of this kernel to
    settle, more than a handful of warm-up steps cover."""
    import torch
    if seconds <= 0:
        return 0, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while True:
        for _ in range(8):
            fn()
        k += 8
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return k, dt


def time_steps(fn, steps, warmup):
    """Average milliseconds per step, events on the launch stream (torch's current)."""
    import torch
    stream = torch.cuda.current_stream()
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


def int8_gemm_reference(achieved_tops, seconds=0.5, reps=10):
    """The vendor library's int8 GEMM (hipBLASLt through torch._int_mm) on random
    int8 operands of 8192 x 8192 x 8192, timed like the headline: what the chip
    sustains on a plain dense int8 contraction, beside the published peak.  A
    reference measurement only; nothing of the polynomial path runs through it."""
    import torch
    M = K = N = 8192
    try:
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        x = torch.randint(-128, 128, (M, K), dtype=torch.int8, device="cuda", generator=g)
        y = torch.randint(-128, 128, (K, N), dtype=torch.int8, device="cuda", generator=g)
        run = lambda: torch._int_mm(x, y)
        preheat(run, seconds)
        ms = time_steps(run, reps, 2)
    except (RuntimeError, AttributeError) as exc:  # int8 GEMM not provided by this torch build
        return {"library": "torch._int_mm", "error": str(exc)[:200]}
    tops = 2 * M * K * N / (ms / 1e3) / 1e12
    return {"library": "hipBLASLt (torch._int_mm)", "shape": [M, K, N], "ms": ms, "tops": tops,
            "headline_vs_library": achieved_tops / tops}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, budget_s, c_gpu):
    """The oracle, as it is, on the host cores: best of up to three runs over a
    bounded sample of the same workload (all pairs when they fit the budget).  The
    sample's oracle results are also compared word for word with c_gpu, the output
    of the timed GPU launch; returns (baseline, parity)."""
    import numpy as np
    import oracle
    B, L, n = w.a.shape
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    oracle.negacyclic_rns(w.a[:1], w.b[:1], w.qs)  # one pair = L products, also the calibration
    per_pair = time.perf_counter() - t0
    pairs = int(max(1, min(B, budget_s / max(per_pair, 1e-6))))
    times = []
    mismatches = None
    while len(times) < 3:
        t0 = time.perf_counter()
        want = oracle.negacyclic_rns(w.a[:pairs], w.b[:pairs], w.qs)
        times.append(time.perf_counter() - t0)
        if mismatches is None:
            mismatches = int(np.count_nonzero(want != c_gpu[:pairs]))
        if sum(times) + times[-1] > budget_s:
            break
    dt = min(times)
    # one thread on one product (one channel of one pair), for the per-core rate
    prev = oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.negacyclic(w.a[:1, 0], w.b[:1, 0], w.qs[0])
    dt1 = time.perf_counter() - t1
    oracle.set_threads(prev)
    base = {"value": pairs * L / dt, "unit": "polymuls/s", "cores": cores, "kind": "oracle",
            "sample": f"{pairs} of {B} ciphertext pairs x {L} channels (n={n}, 30-bit q), best of "
                      f"{len(times)} runs: " + ", ".join(f"{t:.2f}" for t in times) + " s wall",
            "cpu_model": cpu_model(), "single_thread_value": 1 / dt1}
    parity = {"reference": "CPU oracle (schoolbook, 128-bit sums)", "checked_products": pairs * L,
              "of_products": B * L, "checked_words": pairs * L * n, "mismatches": mismatches,
              "bit_exact": mismatches == 0}
    return base, parity


def other_workloads(steps, warmup, pre_s=0.3):
    """The remaining workloads, each timed the same way (an untimed preheat of pre_s
    seconds first, as for the headline); printed to stderr."""
    import numpy as np
    import torch
    import paper_2307_06554_amd as pm
    from paper_2307_06554_amd import inputs
    dev = torch.device("cuda:0")
    out = {}
    for idx in (0, 1):
        w = inputs.make_workload(idx)
        a = torch.from_numpy(w.a.view(np.int32)).to(dev)
        b = torch.from_numpy(w.b.view(np.int32)).to(dev)
        c = torch.empty_like(a)
        run = lambda: pm.polymul_negacyclic(a, b, w.q, out=c)
        preheat(run, pre_s)
        ms = time_steps(run, steps, warmup)
        msp = time_steps(lambda: pm.polymul_negacyclic_plain(a, b, w.q, out=c), max(1, steps // 10), 2)
        out[w.name] = {"polymuls_per_s": a.shape[0] / ms * 1e3, "ms_per_step": ms,
                       "plain_int_polymuls_per_s": a.shape[0] / msp * 1e3}
    w = inputs.make_workload(3)
    groups = []
    for g in w.groups:
        ga = torch.from_numpy(g.a.view(np.int32)).to(dev)
        gb = torch.from_numpy(g.b.view(np.int32)).to(dev)
        groups.append((ga, gb, torch.empty_like(ga), g.n, g.q))
    plan = pm.Plan(groups)
    preheat(plan.execute, pre_s)
    ms = time_steps(plan.execute, steps, warmup)
    ops = sum(2 * 16 * g.n * g.n * g.count for g in w.groups)
    out[w.name] = {"polymuls_per_s": w.products() / ms * 1e3, "ms_per_step": ms, "int8_tops": ops / ms / 1e9,
                   "launch": "one persistent grouped kernel, hipGraph replay"}
    plan.close()
    w = inputs.make_workload(4)
    a = torch.from_numpy(w.a.view(np.int64)).to(dev)
    b = torch.from_numpy(w.b.view(np.int64)).to(dev)
    c = torch.empty_like(a)
    run = lambda: pm.polymul_negacyclic_u64(a, b, w.q, out=c)
    preheat(run, pre_s)
    ms = time_steps(run, max(2, steps // 20), 2)
    ops = 2 * 64 * w.n * w.n * a.shape[0]
    dk = pm.polymul_tune_get_karatsuba(w.n, a.shape[0], 8)
    ws = torch.empty(max(16, pm.polymul_karatsuba_u64_workspace_size(w.n, a.shape[0], dk)), dtype=torch.uint8,
                     device=dev)
    ck = torch.empty_like(a)
    msk = time_steps(lambda: pm.polymul_negacyclic_u64_karatsuba(a, b, w.q, dk, workspace=ws, out=ck),
                     max(2, steps // 20), 2)
    out[w.name] = {"polymuls_per_s": a.shape[0] / ms * 1e3, "ms_per_step": ms, "int8_tops": ops / ms / 1e9,
                   "karatsuba_depth": dk, "karatsuba_polymuls_per_s": a.shape[0] / msk * 1e3,
                   "karatsuba_ms_per_step": msk,
                   "karatsuba_bit_identical": bool(torch.equal(c, ck))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=150,
                    help="untimed steps; the shader clock settles within about 100 launches")
    ap.add_argument("--cpu-budget", type=float, default=24.0,
                    help="seconds of oracle work for cpu_baseline (and the parity check of the timed output)")
    ap.add_argument("--preheat-s", type=float, default=1.0,
                    help="untimed seconds of the headline launch before its warm-up steps (clock settling)")
    ap.add_argument("--preheat-route", choices=("direct", "crt", "karatsuba", "plain"), default="direct",
                    help="the route the untimed preheat runs on the headline batch (direct: the timed "
                         "launch itself; the others hold the GPU on that route, e.g. to read its power draw)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--all", action="store_true", help="also time the other workloads (stderr)")
    ap.add_argument("--karatsuba-depth", type=int, default=0,
                    help="levels of the Karatsuba route (0: the tuned depth; -1 skips the route)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the products are independent and this library has no "
              "multi-GPU path (each GPU would take its own share of the products). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2307_06554_amd as pm
    from paper_2307_06554_amd import inputs, tune

    pm.load_library()
    tuned = tune.apply()
    if args.calibrate_copy_mib:
        words = args.calibrate_copy_mib * (1 << 18)
        src = torch.ones(words, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dev = torch.device("cuda:0")
    w = inputs.make_workload(WORKLOAD_INDEX)
    B, L, n = w.a.shape
    products = B * L
    a = torch.from_numpy(w.a.view(np.int32)).to(dev)
    b = torch.from_numpy(w.b.view(np.int32)).to(dev)
    c = torch.empty_like(a)

    headline = lambda: pm.polymul_negacyclic_rns(a, b, w.qs, out=c)
    pre_fn = headline
    if args.preheat_route == "crt":
        c_pre = torch.empty_like(a)
        pre_fn = lambda: pm.polymul_negacyclic_rns_crt(a, b, w.qs, out=c_pre)
    elif args.preheat_route == "karatsuba":
        d_pre = pm.polymul_tune_get_karatsuba(n, products, 4) or 2
        ws_pre = torch.empty(max(16, pm.polymul_karatsuba_workspace_size(n, L, B, d_pre)), dtype=torch.uint8,
                             device=dev)
        c_pre = torch.empty_like(a)
        pre_fn = lambda: pm.polymul_negacyclic_rns_karatsuba(a, b, w.qs, d_pre, workspace=ws_pre, out=c_pre)
    elif args.preheat_route == "plain":
        a0, b0, c_pre = a[:, 0].contiguous(), b[:, 0].contiguous(), torch.empty((B, n), dtype=torch.int32,
                                                                                device=dev)
        pre_fn = lambda: pm.polymul_negacyclic_plain(a0, b0, w.qs[0], out=c_pre)
    pre_launches, pre_s = preheat(pre_fn, args.preheat_s)
    ms = time_steps(headline, args.steps, args.warmup)
    value = products / (ms / 1e3)
    c_timed = c.cpu().numpy().view(np.uint32).copy()  # output of the timed launches

    # the plain integer kernel on the same inputs, one channel at a time (same total work);
    # channel slices are copied once up front so the timed region holds only that kernel
    chans = [(a[:, l].contiguous(), b[:, l].contiguous(), q) for l, q in enumerate(w.qs)]
    cp = torch.empty((B, n), dtype=torch.int32, device=dev)

    def plain_run():
        for aa, bb, q in chans:
            pm.polymul_negacyclic_plain(aa, bb, q, out=cp)
    ms_plain = time_steps(plain_run, max(1, min(args.steps, 5)), 1)
    plain_value = products / (ms_plain / 1e3)

    kara = None
    if args.karatsuba_depth >= 0:
        d = args.karatsuba_depth or pm.polymul_tune_get_karatsuba(n, products, 4)
        ws = torch.empty(max(16, pm.polymul_karatsuba_workspace_size(n, L, B, d)), dtype=torch.uint8, device=dev)
        ck = torch.empty_like(a)
        ms_k = time_steps(lambda: pm.polymul_negacyclic_rns_karatsuba(a, b, w.qs, d, workspace=ws, out=ck),
                          args.steps, args.warmup)
        pm.polymul_negacyclic_rns(a, b, w.qs, out=c)
        torch.cuda.synchronize()
        sub_ops = 2 * 16 * (n >> d) ** 2 * 3 ** d * products
        kara = {"depth": d, "value": products / (ms_k / 1e3), "unit": "polymuls/s", "ms_per_step": ms_k,
                "speedup_vs_direct": ms / ms_k, "bit_identical_to_direct": bool(torch.equal(ck, c)),
                "kernels": ("split, matrix kernel on 3^d sub-products of degree n/2^d, combine" if d else
                            "direct route (the tuned depth is 0)"),
                "mfma_ops_per_step": sub_ops, "schoolbook_equivalent_tops": 2 * 16 * n * n * products / ms_k / 1e9}
        del ws, ck

    # one b per channel shared by all 256 pairs (same shapes and work, b staged once per chunk)
    bs = b[0].contiguous()
    cs = torch.empty_like(a)
    ms_s = time_steps(lambda: pm.polymul_negacyclic_rns_shared(a, bs, w.qs, out=cs), args.steps, args.warmup)
    shared = {"value": products / (ms_s / 1e3), "unit": "polymuls/s", "ms_per_step": ms_s,
              "speedup_vs_direct": ms / ms_s, "b": "pair 0's b for every pair, one per channel",
              "kernel": "mfma32_shared_kernel<4>"}
    del bs, cs

    # the paper's own coefficient method: 8-bit co-prime moduli and CRT (9 residue channels here)
    cc = torch.empty_like(a)
    ms_c = time_steps(lambda: pm.polymul_negacyclic_rns_crt(a, b, w.qs, out=cc), args.steps, args.warmup)
    chans = len(pm.polymul_crt_moduli(n, max(w.qs)))
    # LDS bytes read per lane and K-step of one channel: two A runs (five dwords each) and two
    # B runs (16 bytes each) feed the four MFMAs of a product's 2 x 2 tiles
    lds_bytes = products * chans * (n // 32) * 64 * (2 * 20 + 2 * 16)  # n/32 K-steps, 64 lanes
    crt = {"value": products / (ms_c / 1e3), "unit": "polymuls/s", "ms_per_step": ms_c,
           "vs_limbs": ms / ms_c, "moduli": pm.polymul_crt_moduli(n, max(w.qs)),
           "mfma_ops_per_step": 2 * chans * n * n * products,
           "lds_read_tb_per_s": lds_bytes / (ms_c / 1e3) / 1e12,
           "bound": "issue: per MFMA, half an A run to read and align and half a B run",
           "bit_identical_to_limbs": None,
           # at n = 4096 eight or nine channels run in two phases, two workgroups per CU
           "kernel": f"crt_phase_kernel<{chans}>" if chans in (8, 9) else f"crt_wave_kernel<{chans}>"}
    pm.polymul_negacyclic_rns(a, b, w.qs, out=c)
    torch.cuda.synchronize()
    crt["bit_identical_to_limbs"] = bool(torch.equal(cc, c))
    del cc

    limbs = 4  # int8 limbs per operand for a 30-bit modulus
    ops_per_product = 2 * limbs * limbs * n * n
    achieved_tops = ops_per_product * products / (ms / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "polymuls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "preheat": {"launches": pre_launches, "seconds": round(pre_s, 3), "route": args.preheat_route},
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "rns_channels": L, "pairs": B, "products_per_step": products,
                   "q_bits": 30, "limbs": limbs, "tile_t": pm.polymul_tune_get(n, limbs), "tune_cache": tuned},
        "roofline": {"bound": "mfma", "achieved": achieved_tops, "peak": PEAK_INT8_TOPS, "unit": "TOPS",
                     "frac": achieved_tops / PEAK_INT8_TOPS, "traffic": measured_traffic(), "mfma_busy": measured_mfma_busy(), "kernel": KERNEL},
        "karatsuba": kara,
        "shared_operand": shared,
        "rns_crt": crt,
        "plain_int": {"value": plain_value, "unit": "polymuls/s", "ms_per_step": ms_plain,
                      "mfma_speedup": value / plain_value,
                      "tmac_per_s": products * n * n / (ms_plain / 1e3) / 1e12,
                      "kernel": "plain_kernel (v_mad_u64_u32 per 32x32-bit term, lazy folds)"},
        "int8_gemm_reference": int8_gemm_reference(achieved_tops),
    }
    out["parity"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(w, args.cpu_budget, c_timed)
    if args.all:
        print(json.dumps({"other_workloads": other_workloads(max(20, args.steps // 4), 20)}), file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)
    if out["parity"] is not None and out["parity"]["mismatches"]:
        print(f"bench.py: the timed output differs from the oracle in {out['parity']['mismatches']} words",
              file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()

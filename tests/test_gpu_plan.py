"""GPU: grouped persistent plans (uneven degrees and moduli in one launch,
replayed from a HIP graph) and the tile table of the resident path."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu


def _groups_from_workload(w):
    out = []
    for g in w.groups:
        a, b = to_dev(g.a), to_dev(g.b)
        out.append((a, b, torch.zeros_like(a), g.n, g.q, g))
    return out


@pytest.mark.parametrize("flags", [0, pm.binding.POLYMUL_PLAN_NO_GRAPH])
def test_plan_workload3(flags):
    """The uneven workload (2048x256, 512x1024, 128x2048, 64x4096, 16x8192, one
    30-bit prime per group) in one plan; every replay checked, with eager work
    (zeroing the outputs, an unrelated product) between replays."""
    w = inputs.make_workload(3)
    gs = _groups_from_workload(w)
    want = [oracle.negacyclic(g.a, g.b, g.q) for (_, _, _, _, _, g) in gs]
    plan = pm.Plan([(a, b, c, n, q) for (a, b, c, n, q, _) in gs], flags)
    rng = np.random.Generator(np.random.PCG64(9))
    xa = to_dev(rng.integers(0, 3329, size=(4, 256), dtype=np.uint64).astype(np.uint32))
    for rep in range(3):
        for (_, _, c, _, _, _) in gs:
            c.zero_()
        pm.polymul_negacyclic(xa, xa, 3329)  # eager work between replays
        torch.cuda.synchronize()
        plan.execute()
        torch.cuda.synchronize()
        for (_, _, c, _, _, g), wv in zip(gs, want):
            got = to_host(c, np.uint32)
            assert np.array_equal(got, wv), f"replay {rep}, n={g.n}: " + mismatch_report(got, wv)
    plan.close()


def test_plan_mixed_degrees_and_word_sizes():
    rng = np.random.Generator(np.random.PCG64(17))
    specs = [(1, 17, 4, 5), (2, 3329, 4, 3), (8, 65537, 4, 7), (64, 1068236801, 4, 9), (256, (1 << 32) - 5, 4, 6),
             (4096, 1068236801, 4, 2), (8192, 3329, 4, 1), (16384, 1068236801, 4, 1),
             (64, inputs.GOLDILOCKS, 8, 3), (1024, (1 << 64) - 59, 8, 2), (16, 1 << 40, 8, 2)]
    groups, refs = [], []
    for n, q, eb, count in specs:
        dt = np.uint32 if eb == 4 else np.uint64
        a = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(dt)
        b = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(dt)
        da, db = to_dev(a), to_dev(b)
        groups.append((da, db, torch.zeros_like(da), n, q))
        refs.append((a, b, q, dt))
    plan = pm.Plan(groups)
    for rep in range(2):
        for g in groups:
            g[2].zero_()
        plan.execute()
        torch.cuda.synchronize()
        for (da, db, dc, n, q), (a, b, q2, dt) in zip(groups, refs):
            got = to_host(dc, dt)
            wv = oracle.negacyclic(a, b, q)
            assert np.array_equal(got, wv), f"replay {rep}, n={n}, q={q}: " + mismatch_report(got, wv)
    plan.close()


def test_plan_empty_groups():
    a = torch.zeros((0, 256), dtype=torch.int32, device="cuda")
    plan = pm.Plan([(a, a.clone(), a.clone(), 256, 17)])
    plan.execute()
    torch.cuda.synchronize()
    plan.close()
    plan = pm.Plan([])
    plan.execute()
    plan.close()


@pytest.mark.parametrize("n,t", [(256, 64), (256, 128), (1024, 64), (1024, 128), (2048, 32), (2048, 128),
                                 (4096, 32), (4096, 128), (8192, 32), (8192, 128), (128, 128)])
def test_tile_table_parity(n, t):
    q = 1068236801
    rng = np.random.Generator(np.random.PCG64(n * t))
    a = rng.integers(0, q, size=(5, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, size=(5, n), dtype=np.uint64).astype(np.uint32)
    try:
        pm.polymul_tune_set(n, 4, t)
        got = to_host(pm.polymul_negacyclic(to_dev(a), to_dev(b), q), np.uint32)
    finally:
        pm.polymul_tune_set(n, 4, 0)
    wv = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, wv), mismatch_report(got, wv)


def test_plan_split_k_runs():
    """A plan dominated by one large product: its K range is cut into runs on
    several workgroups whose residues the last run adds up; three replays."""
    rng = np.random.Generator(np.random.PCG64(23))
    specs = [(65536, 1068236801, 1), (2048, 3329, 3), (256, 17, 50), (8192, (1 << 32) - 5, 2)]
    groups, host = [], []
    for n, q, count in specs:
        a = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
        da, db = to_dev(a), to_dev(b)
        groups.append((da, db, torch.zeros_like(da), n, q))
        host.append((a, b, q))
    plan = pm.Plan(groups)
    big_a, big_b, big_q = host[0]
    jidx = rng.integers(0, 65536, size=96, dtype=np.uint64)
    jidx[:4] = [0, 1, 65534, 65535]
    pidx = np.zeros_like(jidx)
    want_big = oracle.negacyclic_sample(big_a, big_b, big_q, pidx, jidx)
    want_rest = [oracle.negacyclic(a, b, q) for (a, b, q) in host[1:]]
    for rep in range(3):
        for g in groups:
            g[2].zero_()
        plan.execute()
        torch.cuda.synchronize()
        got_big = to_host(groups[0][2], np.uint32)[0, jidx.astype(np.int64)]
        assert np.array_equal(got_big, want_big), f"replay {rep}: " + mismatch_report(got_big, want_big)
        for (da, db, dc, n, q), wv in zip(groups[1:], want_rest):
            got = to_host(dc, np.uint32)
            assert np.array_equal(got, wv), f"replay {rep}, n={n}: " + mismatch_report(got, wv)
    plan.close()


@pytest.mark.parametrize("flags", [0, pm.binding.POLYMUL_PLAN_NO_GRAPH])
def test_plan_back_to_back_replays(flags):
    """Replays queued back to back on one stream, two plans interleaved: each launch
    leaves its queue counters at zero for the next, with no reset in between."""
    rng = np.random.Generator(np.random.PCG64(31))
    specs = [[(16384, 1068236801, 1), (256, 3329, 40), (1024, 65537, 6)], [(4096, (1 << 32) - 5, 3), (64, 17, 9)]]
    plans, checks = [], []
    for spec in specs:
        groups, host = [], []
        for n, q, count in spec:
            a = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
            b = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
            da, db = to_dev(a), to_dev(b)
            groups.append((da, db, torch.zeros_like(da), n, q))
            host.append(oracle.negacyclic(a, b, q))
        plans.append(pm.Plan(groups, flags))
        checks.append((groups, host))
    for rep in range(4):
        for (groups, _), plan in zip(checks, plans):
            for g in groups:
                g[2].zero_()
            plan.execute()
    torch.cuda.synchronize()
    for groups, host in checks:
        for (_, _, dc, n, q), wv in zip(groups, host):
            got = to_host(dc, np.uint32)
            assert np.array_equal(got, wv), f"n={n}: " + mismatch_report(got, wv)
    for plan in plans:
        plan.close()


def test_plan_small_moduli_limb_counts():
    """Groups whose moduli need two or three int8 limbs run with that many (one
    grouped launch mixing 2-, 3- and 4-limb jobs, split items included)."""
    rng = np.random.Generator(np.random.PCG64(23))
    specs = [(256, 3329, 300), (1024, 3329, 40), (4096, 3329, 2), (2048, (1 << 24) - 3, 9),
             (4096, 12289, 1), (512, 1068236801, 17), (8192, 7681, 1)]
    groups, refs = [], []
    for n, q, count in specs:
        a = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
        da, db = to_dev(a), to_dev(b)
        groups.append((da, db, torch.zeros_like(da), n, q))
        refs.append((a, b, q))
    for share, stream in ((100, 125), (10, 400), (1000, 50)):
        pm.polymul_tune_param_set("plan_share_pct", share)
        pm.polymul_tune_param_set("plan_stream_pct", stream)
        try:
            plan = pm.Plan(groups)
        finally:
            pm.polymul_tune_param_set("plan_share_pct", 140)
            pm.polymul_tune_param_set("plan_stream_pct", 125)
        for rep in range(2):
            for g in groups:
                g[2].zero_()
            plan.execute()
            torch.cuda.synchronize()
            for (da, db, dc, n, q), (a, b, _) in zip(groups, refs):
                got = to_host(dc, np.uint32)
                wv = oracle.negacyclic(a, b, q)
                assert np.array_equal(got, wv), f"share {share}, replay {rep}, n={n}, q={q}: " + mismatch_report(got, wv)
        plan.close()


@pytest.mark.parametrize("t", [32, 64, 128])
def test_plan_k_window_runs(t):
    """K-split runs stage only the window of a and the B rows their K range reads
    (n = 8192 runs resident this way).  Every tile side, split depths from two runs
    to one K-step per run (share 10 %), two to four limbs; n = 128 on 128-wide tiles
    must not be split (its staging runs need n >= 256)."""
    rng = np.random.Generator(np.random.PCG64(41 + t))
    specs = [(8192, 1068236801, 2), (8192, (1 << 24) - 3, 1), (4096, 3329, 2), (2048, (1 << 24) - 3, 3),
             (1024, 1068236801, 3), (256, 12289, 5), (128, 17, 3)]
    groups, want = [], []
    for n, q, count in specs:
        a = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
        b = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(np.uint32)
        da, db = to_dev(a), to_dev(b)
        groups.append((da, db, torch.zeros_like(da), n, q))
        want.append(oracle.negacyclic(a, b, q))
    tiles = [(n, L) for n, _, _ in specs for L in (2, 3, 4) if t <= n]
    try:
        for n, L in tiles:
            pm.polymul_tune_set(n, L, t)
        for share in (10, 30, 60, 140, 1000):
            pm.polymul_tune_param_set("plan_share_pct", share)
            try:
                plan = pm.Plan(groups)
            finally:
                pm.polymul_tune_param_set("plan_share_pct", 140)
            for rep in range(2):
                for g in groups:
                    g[2].zero_()
                plan.execute()
                torch.cuda.synchronize()
                for (da, db, dc, n, q), wv in zip(groups, want):
                    got = to_host(dc, np.uint32)
                    assert np.array_equal(got, wv), f"t={t}, share {share}, replay {rep}, n={n}, q={q}: " + \
                        mismatch_report(got, wv)
            plan.close()
    finally:
        for n, L in tiles:
            pm.polymul_tune_set(n, L, 0)


@pytest.mark.parametrize("seed", range(12))
def test_plan_random_compositions(seed):
    """Seeded random plans: 3-6 groups of random degree (4 .. 16384), modulus (2 .. 64
    bits) and count, built at a random split share (K-split runs, windowed runs and
    streamed blocks mixed), two replays each checked word for word against the oracle."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    moduli32 = [17, 3329, 12289, 65537, 7681, (1 << 24) - 3, 1068236801, 536903681, (1 << 32) - 5]
    moduli64 = [inputs.GOLDILOCKS, (1 << 64) - 59, (1 << 40) + 15]
    groups, refs = [], []
    for _ in range(int(rng.integers(3, 7))):
        n = int(2 ** rng.integers(2, 15))
        wide = rng.random() < 0.2
        pool = moduli64 if wide else moduli32
        q = pool[int(rng.integers(len(pool)))]  # by index: a choice over the list would round 2^64 - 59 to float
        count = int(rng.integers(1, max(2, min(40, (1 << 16) // n))))
        dt = np.uint64 if wide else np.uint32
        a = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(dt)
        b = rng.integers(0, q, size=(count, n), dtype=np.uint64).astype(dt)
        da, db = to_dev(a), to_dev(b)
        groups.append((da, db, torch.zeros_like(da), n, q))
        refs.append((oracle.negacyclic(a, b, q), dt))
    share = int(rng.choice([10, 30, 70, 140, 400]))
    pm.polymul_tune_param_set("plan_share_pct", share)
    try:
        plan = pm.Plan(groups)
    finally:
        pm.polymul_tune_param_set("plan_share_pct", 140)
    for rep in range(2):
        for g in groups:
            g[2].zero_()
        plan.execute()
        torch.cuda.synchronize()
        for (da, db, dc, n, q), (wv, dt) in zip(groups, refs):
            got = to_host(dc, dt)
            assert np.array_equal(got, wv), f"seed {seed}, share {share}, replay {rep}, n={n}, q={q}: " + \
                mismatch_report(got, wv)
    plan.close()

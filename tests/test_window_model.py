"""K-window staging of K-split plan runs on the CPU: every LDS read of a run's K
loop stays inside its planes, every byte a matrix instruction uses was staged
with the right ext index or B row, no staging run is taken twice, and the runs'
sums add up to the oracle's product."""
import numpy as np
import pytest

import oracle
from window_model import geometry, host_window, reads, run_window, splittable, stage

CASES = [(256, 128, 2), (512, 128, 4), (1024, 128, 8), (1024, 128, 32), (2048, 128, 16), (4096, 64, 2),
         (4096, 64, 4), (4096, 128, 128), (8192, 32, 2), (8192, 32, 4), (8192, 64, 4), (8192, 128, 8),
         (8192, 128, 256)]


def _runs(n, t, k):
    g = geometry(n, t)
    a_plane, b_rows, steps = host_window(g, k)
    for grp in range(g["U"] // 4):
        for part in range(k):
            st_lo, st_hi = part * steps // k, (part + 1) * steps // k
            E, v_lo, ranges = run_window(g, a_plane, b_rows, grp, st_lo, st_hi)
            yield g, a_plane, b_rows, grp, st_lo, st_hi, E, v_lo, ranges


@pytest.mark.parametrize("n,t,k", CASES)
def test_window_reads_stay_inside_and_find_their_bytes(n, t, k):
    assert splittable(n, t)
    for g, a_plane, b_rows, grp, st_lo, st_hi, E, v_lo, ranges in _runs(n, t, k):
        runs = [cr for lo, cnt in ranges for cr in range(lo, lo + cnt)]
        assert len(runs) == len(set(runs)) and all(0 <= cr < 2 * (n >> 8) for cr in runs)
        apos, brow = stage(g, a_plane, b_rows, E, v_lo, ranges)
        sample = range(st_lo, st_hi) if st_hi - st_lo <= 8 else sorted({st_lo, st_lo + 1, (st_lo + st_hi) // 2,
                                                                           st_hi - 2, st_hi - 1})
        for st in sample:
            d = st >> g["log2spd"]
            for z, u, base, S, row, boff in reads(g, E, v_lo, grp, st):
                assert 0 <= base and base + 20 <= a_plane  # five dwords read per A run
                for i in range(16):
                    assert apos.get(S + i) == E - (S + i)  # position p holds ext[E - p]
                assert 0 <= row < b_rows and boff + 16 <= g["rowstride"]
                assert brow[row] == (u - d if u - d < g["r"] else None)


@pytest.mark.parametrize("n,t,k", [(256, 128, 2), (512, 128, 4), (512, 128, 16), (1024, 128, 2),
                                   (1024, 128, 32)])
def test_window_runs_add_up_to_the_product(n, t, k):
    q = 1000003
    rng = np.random.Generator(np.random.PCG64(n + k))
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)
    g = geometry(n, t)
    r = g["r"]

    def ext(e):
        return int(a[e]) if e >= 0 else -int(a[n + e])

    def bval(v, w):
        if v is None:
            return 0
        return int(b[v * t + w]) if v >= 0 else -int(b[(v + r) * t + w])

    got = [0] * n
    for g, a_plane, b_rows, grp, st_lo, st_hi, E, v_lo, ranges in _runs(n, t, k):
        apos, brow = stage(g, a_plane, b_rows, E, v_lo, ranges)
        for st in range(st_lo, st_hi):
            w0 = (st & (g["spd"] - 1)) << 5
            lanes = reads(g, E, v_lo, grp, st)
            for lane in range(0, len(lanes), 64):  # one wave: its 32 rows z and 32 columns u
                wave = lanes[lane:lane + 64]
                for zl in range(32):
                    z, _, _, S_lo, _, _ = wave[zl]
                    _, _, _, S_hi, _, _ = wave[32 + zl]
                    arow = [ext(apos[S_lo + i]) for i in range(16)] + [ext(apos[S_hi + i]) for i in range(16)]
                    for ul in range(32):
                        _, u, _, _, row, _ = wave[ul]
                        if z >= t or u >= r:
                            continue
                        bcol = [bval(brow[row], w0 + kk) for kk in range(32)]
                        got[u * t + z] += sum(x * y for x, y in zip(arow, bcol))
    want = oracle.negacyclic(a.astype(np.uint32)[None], b.astype(np.uint32)[None], q)[0]
    assert np.array_equal(np.array([x % q for x in got], dtype=np.uint32), want)

"""Model of the K-window staging of K-split resident runs (grouped plans), for the
CPU tests: the same index arithmetic as the kernel, written out with Python
integers.

A run of K-steps [st_lo, st_hi) of one product on the Toeplitz recast (Sec. 2.2,
Eq. (3); block split n = t r of Sec. 2.5) touches d in [d_lo, d_hi): ext indices
d_lo t - t + 1 .. d_hi t - 1 and B rows v = u - d of the group's u tiles.  The
run stages the ext range with E = d_hi t - 1 at reversed position 0 and the rows
from v_lo = u_lo - d_hi + 1, taking the runs of 64 word groups (a's n/4, then
b's n/4) that hold a byte of either; the host sizes the planes for the widest
run.  The model returns what the kernel would stage and read, so that the tests
can check bounds, coverage and the sums against the oracle.
"""


def geometry(n, t):
    """Tile geometry of the resident path for t >= 32 (rowlen = t)."""
    r = n // t
    spd = t // 32
    tz, tu = t // 32, (r + 31) // 32
    rowstride = t if (t // 16) & 1 else t + 16
    return dict(n=n, t=t, r=r, spd=spd, log2spd=spd.bit_length() - 1, tz=tz, tu=tu, U=tz * tu,
                rowstride=rowstride)


def splittable(n, t):
    g = geometry(n, t)
    return n >= 256 and t >= 32 and g["U"] >= 4


def host_window(g, k):
    """Plane sizes for kparts = k (the widest run's d range)."""
    steps = g["r"] << g["log2spd"]
    dmax = 0
    for part in range(k):
        lo, hi = part * steps // k, (part + 1) * steps // k
        dmax = max(dmax, ((hi - 1) >> g["log2spd"]) + 1 - (lo >> g["log2spd"]))
    a_plane = (dmax * g["t"] + g["t"] + 4 + 15) & ~15
    b_rows = 32 * (4 // g["tz"]) + dmax - 1
    return a_plane, b_rows, steps


def run_window(g, a_plane, b_rows, grp, st_lo, st_hi):
    """E, v_lo and the staged run ranges [(lo, count)] of one run of group grp."""
    n, t, r = g["n"], g["t"], g["r"]
    ut_lo = ((grp * 4) % g["U"]) // g["tz"]
    d_lo, d_hi = st_lo >> g["log2spd"], ((st_hi - 1) >> g["log2spd"]) + 1
    E = d_hi * t - 1
    v_lo = 32 * ut_lo - d_hi + 1
    q4, a_runs = n // 4, n >> 8
    e4, A4 = (E + 1) >> 2, a_plane >> 2
    ranges, end = [], 0
    for lo, hi, base in ((max(0, e4 - A4), min(q4, e4), 0),
                         (max(0, e4 + q4 - A4), min(q4, e4 + q4), 0),
                         (max(0, v_lo) * (t // 4), min(r, v_lo + b_rows) * (t // 4), a_runs),
                         (max(0, v_lo + r) * (t // 4), min(r, v_lo + r + b_rows) * (t // 4), a_runs)):
        rlo, rhi = base + (lo >> 6), base + ((hi + 63) >> 6)
        if lo >= hi:
            rlo = rhi = end
        rlo = max(rlo, end)
        rhi = max(rhi, rlo)
        ranges.append((rlo, rhi - rlo))
        end = rhi
    return E, v_lo, ranges


def stage(g, a_plane, b_rows, E, v_lo, ranges):
    """Staged A bytes {position: ext index} and B rows {row: v}, as the kernel writes them."""
    n, t, r = g["n"], g["t"], g["r"]
    q4, a_runs = n // 4, n >> 8
    e4, A4 = (E + 1) >> 2, a_plane >> 2
    apos, brow = {}, {}
    for lo, cnt in ranges:
        for cr in range(lo, lo + cnt):
            for lane in range(64):
                if cr < a_runs:
                    j = cr * 64 + lane
                    dw = (e4 - 1 - j) % (1 << 32)  # unsigned: "below zero" wraps and is skipped
                    for kk in range(4):
                        if dw < A4:
                            apos[dw * 4 + kk] = 4 * j + 3 - kk
                        if (dw + q4) % (1 << 32) < A4:
                            apos[((dw + q4) % (1 << 32)) * 4 + kk] = 4 * j + 3 - kk - n
                else:
                    e = (cr - a_runs) * 64 + lane
                    vs = e // (t // 4)
                    for row, v in ((vs - v_lo, vs), (vs - r - v_lo, vs - r)):
                        if 0 <= row < b_rows:
                            brow[row] = v
    for row in range(max(0, r - v_lo), b_rows):  # rows v >= r: zero
        brow[row] = None
    return apos, brow


def reads(g, E, v_lo, grp, st):
    """Per wave and lane of group grp at K-step st: (first A dword byte, A bytes used,
    B row, B byte offset in the row)."""
    t = g["t"]
    d, w0 = st >> g["log2spd"], (st & (g["spd"] - 1)) << 5
    out = []
    for wave in range(4):
        tile = (grp * 4 + wave) & (g["U"] - 1)
        z0, u0 = 32 * (tile % g["tz"]), 32 * (tile // g["tz"])
        for lane in range(64):
            zl, hi = lane & 31, lane >> 5
            S = E - (z0 + zl) + 16 * hi - d * t + w0
            out.append((z0 + zl, u0 + zl, (S >> 2) * 4, S, u0 + zl - d - v_lo, w0 + 16 * hi))
    return out

"""The small-modulus residue path on the CPU: its moduli rule, its exactness
bound and its reconstruction, checked against the oracle."""
import math

import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from crt_model import moduli, product


@pytest.mark.parametrize("n", [1, 4, 256, 1024, 4096, 65536])
@pytest.mark.parametrize("q", [2, 3329, 12289, 1068236801, 536903681, (1 << 32) - 5])
def test_moduli_rule(n, q):
    ms = moduli(n, q)
    assert ms and len(ms) <= 11
    assert all(2 <= m <= 256 for m in ms) and ms == sorted(ms, reverse=True)
    assert all(math.gcd(x, y) == 1 for i, x in enumerate(ms) for y in ms[i + 1:])
    B = n * (q // 2) ** 2
    assert math.prod(ms) > 2 * B * (1 + 2 ** -16)
    assert math.prod(ms[:-1]) <= 2 * B + ((2 * B) >> 16) + 1  # no modulus more than needed
    assert pm.polymul_crt_moduli(n, q) == ms  # the library's ExtractModuli agrees


def test_moduli_known_values():
    # the largest co-prime 8-bit moduli, as the paper's base rules ask (Sec. 2.6)
    assert moduli(4096, 1068236801) == [256, 255, 253, 251, 247, 241, 239, 233, 229]
    assert moduli(256, 3329) == [256, 255, 253, 251]


@pytest.mark.parametrize("q", [17, 3329, 1068236801, (1 << 32) - 5])
@pytest.mark.parametrize("n", [1, 2, 8, 32])
def test_model_matches_oracle(n, q):
    rng = np.random.Generator(np.random.PCG64(n * 7 + q % 101))
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)
    got, _, worst = product(a, b, q)
    dt = np.uint32
    want = oracle.negacyclic(a.astype(dt)[None], b.astype(dt)[None], q)[0]
    assert [int(x) for x in got] == [int(x) for x in want]
    assert worst < 0.5 - 2 ** -17


@pytest.mark.parametrize("q", [3329, 1068236801, (1 << 32) - 5])
def test_extreme_sums(q):
    # every coefficient floor(q/2): X_{n-1} = n floor(q/2)^2 = B, the largest sum there is
    n = 32
    h = q // 2
    a = np.full(n, h, dtype=np.uint64)
    got, ms, worst = product(a, a, q)
    want = oracle.negacyclic(a.astype(np.uint32)[None], a.astype(np.uint32)[None], q)[0]
    assert [int(x) for x in got] == [int(x) for x in want]
    assert abs(worst - n * h * h / math.prod(ms)) < 1e-12
    assert worst < 0.5 - 2 ** -17


def test_padding_keeps_results():
    rng = np.random.Generator(np.random.PCG64(3))
    q, n = 12289, 16
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)
    base, ms0, _ = product(a, b, q)
    padded, ms1, _ = product(a, b, q, pad=11)
    assert len(ms1) == 11 and ms1[:len(ms0)] == ms0
    assert list(base) == list(padded)


def test_planted_mistake_is_caught():
    # dropping the rounding count kappa (plain sum of s_c M/m_c mod q) breaks the result
    rng = np.random.Generator(np.random.PCG64(9))
    q, n = 3329, 8
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)
    ms = moduli(n, q)
    M = math.prod(ms)
    from crt_model import centred, negacyclic_int
    X = negacyclic_int(centred(a, q), centred(b, q))
    wrong = [sum(((x % m) * pow(M // m % m, -1, m) % m) * (M // m) for m in ms) % q for x in X]
    want = oracle.negacyclic(a.astype(np.uint32)[None], b.astype(np.uint32)[None], q)[0]
    assert [int(x) for x in wrong] != [int(x) for x in want]


def _f32_kappa_sum(s, ms):
    """The kernels' fp32 evaluation of sum_c s_c / m_c + 0.5: terms fl(s_c * fl(1/m_c)),
    added in channel order, then + 0.5."""
    f = np.float32(0.0)
    for sc, m in zip(s, ms):
        f = np.float32(f + np.float32(np.float32(sc) * np.float32(np.float32(1.0) / np.float32(m))))
    return np.float32(f + np.float32(0.5))


@pytest.mark.parametrize("n,q", [(4096, 1068236801), (4096, (1 << 32) - 5), (1, (1 << 32) - 5), (256, 3329)])
def test_kappa_fp32_sum_within_its_bound(n, q):
    """The rounding count kappa = round(sum_c s_c / m_c) is taken from an fp32 sum.
    Over sums X at and next to the extremes +-B (the largest centred negacyclic
    sums, B = n floor(q/2)^2), X = 0 and random X, and over the residue vector
    with every s_c = m_c - 1 (every term and running sum at its largest), the fp32
    value stays within the stated bound (2C + C(C+1)/2 + C + 1) 2^-24 of the exact
    fraction, that bound stays below the 2^-17 margin the moduli rule leaves, and
    kappa comes out exact."""
    from fractions import Fraction
    ms = moduli(n, q)
    C = len(ms)
    M = math.prod(ms)
    u = Fraction(1, 1 << 24)
    bound = (2 * C + C * (C + 1) // 2 + C + 1) * u
    assert bound < Fraction(1, 1 << 17)
    B = n * (q // 2) ** 2
    rng = np.random.Generator(np.random.PCG64(C))
    xs = [B, -B, B - 1, -B + 1, 0, 1, -1] + [int(x) for x in rng.integers(-B, B, size=200, dtype=np.int64)] \
        if B < (1 << 62) else [B, -B, 0, 1, -1]
    worst = Fraction(0)
    for X in xs:
        s = [(X % m) * pow(M // m % m, -1, m) % m for m in ms]
        exact = sum(Fraction(sc, m) for sc, m in zip(s, ms))  # = X / M + kappa
        kappa = exact - Fraction(X, M)
        assert kappa.denominator == 1
        # the true fraction sits at least 2^-17 from the rounding boundary
        assert abs(Fraction(X, M)) <= Fraction(1, 2) - Fraction(1, 1 << 17)
        f = _f32_kappa_sum(s, ms)
        err = abs(Fraction(float(f)) - (exact + Fraction(1, 2)))
        worst = max(worst, err)
        assert err <= bound, (X, float(err), float(bound))
        assert math.floor(float(f)) == kappa
    # every term at its largest: m_c - 1 (a residue vector, whatever X it stands for)
    s = [m - 1 for m in ms]
    exact = sum(Fraction(sc, m) for sc, m in zip(s, ms)) + Fraction(1, 2)
    err = abs(Fraction(float(_f32_kappa_sum(s, ms))) - exact)
    assert err <= bound

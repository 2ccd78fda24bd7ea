"""CPU model of the split-limb recast: exactness and accumulator bounds."""
import random

import numpy as np
import pytest

import oracle
from limb_model import digits, model_product, limb_count
from paper_2307_06554_amd import inputs


@pytest.mark.parametrize("q", [3329, 65537, 1068236801, (1 << 32) - 5, inputs.GOLDILOCKS, (1 << 64) - 59])
def test_digit_window_round_trip(q):
    L = limb_count(q)
    S = sum(256 ** i for i in range(L))
    xs = sorted({0, 1, q - 1, q // 2, min(127 * S, q - 1), min(127 * S + 1, q - 1)} |
                {(0x80 * (256 ** i)) % q for i in range(L)} | {int("80" * L, 16) % q})
    d = digits(xs, q, L)
    assert d.min() >= -128 and d.max() <= 127
    for col, x in enumerate(xs):
        v = sum(int(d[i, col]) * 256 ** i for i in range(L))
        assert v % q == x % q


@pytest.mark.parametrize("n,q", [(1, 17), (8, 3329), (64, 3329), (256, 1068236801), (1024, (1 << 32) - 5),
                                 (2048, 1068236801)])
def test_model_matches_oracle(n, q):
    rng = random.Random(n)
    a = [rng.randrange(q) for _ in range(n)]
    b = [rng.randrange(q) for _ in range(n)]
    c, worst = model_product(a, b, q)
    want = oracle.negacyclic(np.array([a], dtype=np.uint64).astype(np.uint32),
                             np.array([b], dtype=np.uint64).astype(np.uint32), q)[0]
    assert c == [int(v) for v in want]
    assert worst < 2 ** 31


def test_worst_case_digits_bound():
    """Digits pinned near -128 (representative -0x7F808080 = digits [-128,-128,-128,-127]):
    every digit product is about +2^14 and the largest class holds L = 4 pairs, so
    |T_s| <= 4 * n * 2^14 -- below 2^31 up to n = 8192 (the resident kernel's limit),
    not at n = 32768."""
    q = (1 << 32) - 5
    x = q - 0x7F808080
    n = 64
    c, worst = model_product([x] * n, [x] * n, q, L=4)
    want = oracle.negacyclic(np.full((1, n), x, dtype=np.uint32), np.full((1, n), x, dtype=np.uint32), q)[0]
    assert c == [int(v) for v in want]
    assert 3 * n * 2 ** 14 < worst <= 4 * n * 2 ** 14
    assert 4 * 8192 * 2 ** 14 < 2 ** 31 <= 4 * 32768 * 2 ** 14


def test_kchunk_split_bound_goldilocks():
    """With L = 8 a shift class holds 8 pairs: 8 * K * 2^14 < 2^31 needs K <= 16383;
    chunking K keeps every int32 partial in range and the result exact."""
    q = inputs.GOLDILOCKS
    rng = random.Random(3)
    n = 64
    a = [rng.randrange(q) for _ in range(n)]
    b = [rng.randrange(q) for _ in range(n)]
    c_full, worst_full = model_product(a, b, q, L=8)
    c_split, worst_split = model_product(a, b, q, L=8, kchunk=16)
    want = oracle.negacyclic(np.array([a], dtype=np.uint64), np.array([b], dtype=np.uint64), q)[0]
    assert c_full == c_split == [int(v) for v in want]
    assert worst_split <= worst_full
    assert 8 * 16383 * 2 ** 14 < 2 ** 31 <= 8 * 16384 * 2 ** 14
    assert 4 * 32767 * 2 ** 14 < 2 ** 31 <= 4 * 32768 * 2 ** 14

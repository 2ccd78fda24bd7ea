"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import os
import random
import re

import numpy as np
import pytest

import oracle
import pins
from paper_2307_06554_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
Q30 = 1068236801          # a 30-bit prime, q = 1 (mod 8192)
Q32 = (1 << 32) - 5       # largest 32-bit prime
Q_EVEN = (1 << 31) + 6    # q need not be prime (Sec. 2.1)
GOLD_Q = inputs.GOLDILOCKS


def impl(a, b, q):
    return oracle.negacyclic(a, b, q)


# ------------------------------------------------------------- Example 1
def _parse_example1():
    rows, coeffs = [], {}
    with open(os.path.join(GOLD, "example1_n3.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rhs = (s.strip() for s in line.split("="))
            if key.startswith("matrix_row"):
                rows.append(rhs.split())
            else:
                coeffs[key] = re.findall(r"([+-])a(\d)\*b(\d)", rhs)
    return rows, coeffs


@pytest.mark.parametrize("q", [2, 3329, Q30, Q32, Q_EVEN, GOLD_Q])
def test_example1_printed_formulas(q):
    """Example 1 (Sec. 2.2, Eq. (2)): n = 3 coefficients match the printed formulas."""
    rows, coeffs = _parse_example1()
    assert len(coeffs) == 3 and len(rows) == 3
    rng = random.Random(q)
    for _ in range(20):
        a = [rng.randrange(q) for _ in range(3)]
        b = [rng.randrange(q) for _ in range(3)]
        c = impl(np.array([a], dtype=object), np.array([b], dtype=object), q)[0]
        for j in range(3):
            terms = coeffs[f"c{j}"]
            want = sum((1 if s == "+" else -1) * a[int(i)] * b[int(k)] for s, i, k in terms) % q
            assert int(c[j]) == want
        # the printed matrix, row vector a times it
        M = [[(-1 if e.startswith("-") else 1) * b[int(e.lstrip("-")[1])] for e in row] for row in rows]
        assert [int(v) for v in c] == [v % q for v in pins.vec_mat(a, M)]


# ------------------------------------------------- closed forms, invariants
@pytest.mark.parametrize("q", [3329, Q30, Q32, Q_EVEN, GOLD_Q, (1 << 64) - 59])
@pytest.mark.parametrize("n", [2, 4, 64, 1024])
def test_x_to_the_n_is_minus_one(n, q):
    pins.check_minus_one(impl, n, q)


@pytest.mark.parametrize("q", [3329, Q30, Q32, GOLD_Q])
@pytest.mark.parametrize("n", [8, 256, 2048])
def test_monomial_is_signed_rotation(n, q):
    rng = random.Random(n * 7 + q % 1000)
    pins.check_rotation(impl, n, q, rng, sorted({0, 1, n // 2, n - 1, rng.randrange(n)}))


@pytest.mark.parametrize("q", [2, 3329, Q30, Q32, Q_EVEN, GOLD_Q])
@pytest.mark.parametrize("n", [1, 4, 128])
def test_ring_axioms(n, q):
    pins.check_ring_axioms(impl, n, q, random.Random(n + q % 997))


# ---------------------------------------------------- independent algorithms
@pytest.mark.parametrize("q", [2, 3329, Q30, Q32, Q_EVEN, GOLD_Q, (1 << 64) - 59, (1 << 63) + 2])
@pytest.mark.parametrize("n", [1, 3, 16, 256])
def test_kronecker_substitution(n, q):
    pins.check_kronecker(impl, n, q, random.Random(3 * n + q % 991))


@pytest.mark.parametrize("n,q", [(256, 7681), (1024, Q30), (4096, Q30), (2048, 3 * (1 << 30) + 1),
                                 (4096, GOLD_Q), (8, GOLD_Q)])
def test_ntt_product(n, q):
    assert inputs.is_prime(q) and (q - 1) % (2 * n) == 0
    pins.check_ntt(impl, n, q, random.Random(n ^ (q & 0xFFFF)), batch=1)


@pytest.mark.parametrize("n,q", [(1, 5), (1, 7), (2, 2), (2, 3), (2, 5), (4, 2), (4, 3)])
def test_bruteforce_tiny(n, q):
    pins.check_bruteforce(impl, n, q)


@pytest.mark.parametrize("n,q", [(2, 3329), (8, Q30), (64, Q32), (32, GOLD_Q)])
def test_eq3_matrix_and_fig1_split(n, q):
    pins.check_eq3_and_fig1(impl, n, q, random.Random(n))


def test_fig1_block_identities():
    """Derived from Eq. (3): in the half split, M_A = M_D and M_C = -M_B."""
    rng = random.Random(5)
    n, h = 16, 8
    M = pins.eq3_matrix([rng.randrange(100) for _ in range(n)], n)
    MA = [row[:h] for row in M[:h]]
    MB = [row[h:] for row in M[:h]]
    MC = [row[:h] for row in M[h:]]
    MD = [row[h:] for row in M[h:]]
    assert MA == MD
    assert MC == [[-v for v in row] for row in MB]


# ------------------------------------------------------------ input handling
def test_noncanonical_inputs_are_read_mod_q():
    rng = np.random.Generator(np.random.PCG64(9))
    q, n = 3329, 64
    a = rng.integers(0, 1 << 32, size=(3, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, size=(3, n), dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(impl(a, b, q), impl(a % q, b % q, q))
    a64 = rng.integers(0, np.iinfo(np.uint64).max, size=(2, n), dtype=np.uint64, endpoint=True)
    b64 = rng.integers(0, np.iinfo(np.uint64).max, size=(2, n), dtype=np.uint64, endpoint=True)
    assert np.array_equal(impl(a64, b64, GOLD_Q), impl(a64 % np.uint64(GOLD_Q), b64 % np.uint64(GOLD_Q), GOLD_Q))


def test_output_is_canonical_and_dtype():
    w = inputs.make_workload(1, scale=2 / 4096)
    c = impl(w.a, w.b, w.q)
    assert c.dtype == np.uint32 and c.shape == w.a.shape and int(c.max()) < w.q


def test_rns_is_channelwise():
    """Sec. 2.4: each residue channel is an independent product with its own modulus."""
    w = inputs.make_workload(2, scale=2 / 256)
    a, b = w.a[:, :, :256].copy(), w.b[:, :, :256].copy()
    c = oracle.negacyclic_rns(a, b, w.qs)
    for l, q in enumerate(w.qs):
        assert np.array_equal(c[:, l], impl(a[:, l] % q, b[:, l] % q, q))
    # channel 0 on a truncated ring is pinned independently
    q = w.qs[0]
    c2 = oracle.negacyclic_rns(a[:, :1, :64].copy(), b[:, :1, :64].copy(), [q])
    for r in range(a.shape[0]):
        assert [int(v) for v in c2[r, 0]] == pins.kronecker_product(
            [int(v) for v in a[r, 0, :64]], [int(v) for v in b[r, 0, :64]], q)


def test_sample_matches_full():
    w = inputs.make_workload(1, scale=3 / 4096)
    full = impl(w.a, w.b, w.q)
    pidx = np.array([0, 1, 2, 2, 0], dtype=np.uint64)
    jidx = np.array([0, 1023, 5, 512, 77], dtype=np.uint64)
    assert np.array_equal(oracle.negacyclic_sample(w.a, w.b, w.q, pidx, jidx), full[pidx.astype(int), jidx.astype(int)])
    a = w.a.astype(np.uint64)
    b = w.b.astype(np.uint64)
    full64 = impl(a, b, GOLD_Q)
    assert np.array_equal(oracle.negacyclic_sample(a, b, GOLD_Q, pidx, jidx), full64[pidx.astype(int), jidx.astype(int)])


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.negacyclic(np.zeros((1, 4), np.uint32), np.zeros((1, 4), np.uint32), 1)
    with pytest.raises(ValueError):
        oracle.negacyclic(np.zeros((1, 4), np.uint32), np.zeros((1, 5), np.uint32), 17)


# ------------------------------------------------------- the pins have teeth
def _python_definition(mistake=None):
    """Pure-Python version of the definition with an optional planted mistake,
    to show that the pins above catch each kind of slip."""
    def f(a, b, q):
        a, b = np.asarray(a), np.asarray(b)
        out = np.zeros(a.shape, dtype=a.dtype)
        n = a.shape[-1]
        for r in range(a.shape[0]):
            A = [int(v) % q for v in a[r]]
            B = [int(v) % q for v in b[r]]
            for j in range(n):
                s = 0
                for i in range(n):
                    if i <= j:
                        if mistake == "drop_term" and i == j and j == n - 1 and n > 2:
                            continue
                        s += A[i] * B[j - i]
                    else:
                        k = n + j - i
                        if mistake == "wrong_index":
                            k = (k + 1) % n
                        if mistake == "transposed":
                            s += A[i] * B[k]  # becomes correlation below
                            continue
                        s += (A[i] * B[k]) if mistake == "sign" else -(A[i] * B[k])
                if mistake == "transposed":
                    s = sum((A[i] * B[(i - j) % n]) * (1 if i >= j else -1) for i in range(n))
                if mistake == "no_final_mod":
                    out[r, j] = s % (1 << 32) if s >= 0 else (s + q * n * q) % (1 << 32)
                else:
                    out[r, j] = s % q
        return out
    return f


def test_correct_python_definition_passes_all_pins():
    assert pins.run_all(_python_definition()) == []


@pytest.mark.parametrize("mistake", ["drop_term", "sign", "wrong_index", "transposed", "no_final_mod"])
def test_planted_mistakes_are_caught(mistake):
    failures = pins.run_all(_python_definition(mistake))
    assert failures, f"planted mistake '{mistake}' passed every pin"


# --------------------------------------------------- cyclic ring x^n - 1
def cyc(a, b, q):
    return oracle.cyclic(a, b, q)


@pytest.mark.parametrize("q", [2, 3329, Q30, Q32])
@pytest.mark.parametrize("n", [1, 3, 8, 64])
def test_cyclic_kronecker_and_long_division(n, q):
    """Kronecker substitution for the Z[x] product, remainder by x^n - 1."""
    rng = random.Random(n * 31 + q % 1009)
    a = [rng.randrange(q) for _ in range(n)]
    b = [rng.randrange(q) for _ in range(n)]
    k = (n * (q - 1) ** 2).bit_length() + 1
    P = sum(v << (k * i) for i, v in enumerate(a)) * sum(v << (k * i) for i, v in enumerate(b))
    prod = [(P >> (k * d)) & ((1 << k) - 1) for d in range(2 * n - 1)]
    want = [v % q for v in pins.poly_rem_monic(prod, [-1] + [0] * (n - 1) + [1])]
    got = cyc(np.array([a], dtype=np.uint64).astype(np.uint32), np.array([b], dtype=np.uint64).astype(np.uint32), q)[0]
    assert [int(v) for v in got] == want


def test_cyclic_monomial_is_plain_rotation():
    rng = np.random.Generator(np.random.PCG64(5))
    n, q = 64, Q30
    a = rng.integers(0, q, size=(1, n), dtype=np.uint64).astype(np.uint32)
    for k in (0, 1, 17, n - 1):
        b = np.zeros((1, n), dtype=np.uint32)
        b[0, k] = 1
        assert np.array_equal(cyc(a, b, q)[0], np.roll(a[0], k))
    # x^(n-1) * x = x^n = 1
    a = np.zeros((1, n), dtype=np.uint32)
    a[0, n - 1] = 1
    b = np.zeros((1, n), dtype=np.uint32)
    b[0, 1] = 1
    want = np.zeros(n, dtype=np.uint32)
    want[0] = 1
    assert np.array_equal(cyc(a, b, q)[0], want)


def test_cyclic_evaluation_at_roots_of_unity():
    """For q = 1 mod n, c(w^i) = a(w^i) b(w^i) at every n-th root of unity w^i."""
    n, q = 64, 7681  # 7681 = 1 + 120 * 64
    rng = random.Random(11)
    g = 17
    w = pow(g, (q - 1) // n, q)
    while pow(w, n // 2, q) == 1:
        g += 1
        w = pow(g, (q - 1) // n, q)
    a = [rng.randrange(q) for _ in range(n)]
    b = [rng.randrange(q) for _ in range(n)]
    c = [int(v) for v in cyc(np.array([a], dtype=np.uint32), np.array([b], dtype=np.uint32), q)[0]]
    for i in range(n):
        x = pow(w, i, q)
        assert pins.poly_eval(c, x, q) == pins.poly_eval(a, x, q) * pins.poly_eval(b, x, q) % q


def test_cyclic_bruteforce_tiny():
    import itertools
    for n, q in ((2, 3), (4, 2), (3, 3)):
        vecs = list(itertools.product(range(q), repeat=n))
        A = np.array([v for v in vecs for _ in vecs], dtype=np.uint32)
        B = np.array([w for _ in vecs for w in vecs], dtype=np.uint32)
        C = cyc(A, B, q)
        mod = [-1] + [0] * (n - 1) + [1]
        for r in range(A.shape[0]):
            want = [v % q for v in pins.poly_rem_monic(pins.zpoly_mul(list(A[r].astype(int)), list(B[r].astype(int))), mod)]
            assert [int(v) for v in C[r]] == want


@pytest.mark.parametrize("q", [GOLD_Q, (1 << 64) - 59, (1 << 40) + 15])
def test_cyclic_u64_kronecker(q):
    rng = random.Random(q % 997)
    for n in (1, 4, 32):
        a = [rng.randrange(q) for _ in range(n)]
        b = [rng.randrange(q) for _ in range(n)]
        k = (n * (q - 1) ** 2).bit_length() + 1
        P = sum(v << (k * i) for i, v in enumerate(a)) * sum(v << (k * i) for i, v in enumerate(b))
        prod = [(P >> (k * d)) & ((1 << k) - 1) for d in range(2 * n - 1)]
        want = [v % q for v in pins.poly_rem_monic(prod, [-1] + [0] * (n - 1) + [1])]
        got = oracle.cyclic(np.array([a], dtype=np.uint64), np.array([b], dtype=np.uint64), q)[0]
        assert [int(v) for v in got] == want

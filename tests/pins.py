"""Independent checks that pin the CPU oracle (and, through it, the GPU path).

None of these re-types the oracle's formula: each is either a different
algorithm (Kronecker substitution with Python big integers, a psi-twisted
number-theoretic transform, generic polynomial long division), a closed form
(x^n = -1, x^k a = signed rotation), an algebraic invariant of the ring, or a
construction printed in the paper (Example 1, the Eq. (3) matrix, the Fig. 1
divide-and-conquer split).  Each `check_*` takes an implementation
`impl(a, b, q) -> c` over arrays [batch, n] so that planted mistakes can be
shown to fail at least one of them.
"""
import random

import numpy as np


# ----------------------------------------------------------------- helpers
def as_int_lists(x):
    x = np.asarray(x)
    return [[int(v) for v in row] for row in x.reshape(-1, x.shape[-1])]


def zpoly_mul(a, b):
    """Product in Z[x] by the definition of polynomial multiplication (lists of ints)."""
    out = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai:
            for k, bk in enumerate(b):
                out[i + k] += ai * bk
    return out


def poly_rem_monic(p, d):
    """Remainder of p(x) divided by a monic d(x) over Z, by long division.
    Coefficient lists are lowest degree first."""
    p = list(p)
    m = len(d) - 1
    assert d[-1] == 1
    for top in range(len(p) - 1, m - 1, -1):
        coef = p[top]
        if coef:
            for i in range(m + 1):
                p[top - m + i] -= coef * d[i]
    return p[:m] + [0] * max(0, m - len(p))


def negacyclic_modulus(n):
    return [1] + [0] * (n - 1) + [1]  # x^n + 1


def kronecker_product(a, b, q):
    """c = a*b mod (x^n+1, q) via Kronecker substitution: pack each polynomial
    into one big integer at a slot width wide enough that no coefficient of
    the Z[x] product can carry, multiply once, unpack, then reduce by long
    division by x^n + 1 and mod q."""
    n = len(a)
    bound = n * (q - 1) ** 2
    k = bound.bit_length() + 1
    A = sum(int(v) << (k * i) for i, v in enumerate(a))
    B = sum(int(v) << (k * i) for i, v in enumerate(b))
    P = A * B
    mask = (1 << k) - 1
    prod = [(P >> (k * d)) & mask for d in range(2 * n - 1)]
    rem = poly_rem_monic(prod, negacyclic_modulus(n))
    return [v % q for v in rem]


def find_psi(q, n, rng):
    """A primitive 2n-th root of unity mod prime q (psi^n = -1)."""
    assert (q - 1) % (2 * n) == 0
    while True:
        h = rng.randrange(2, q - 1)
        psi = pow(h, (q - 1) // (2 * n), q)
        if pow(psi, n, q) == q - 1:
            return psi


def _fft(vals, w, q):
    n = len(vals)
    if n == 1:
        return list(vals)
    even = _fft(vals[0::2], w * w % q, q)
    odd = _fft(vals[1::2], w * w % q, q)
    out = [0] * n
    t = 1
    for i in range(n // 2):
        u, v = even[i], odd[i] * t % q
        out[i] = (u + v) % q
        out[i + n // 2] = (u - v) % q
        t = t * w % q
    return out


def ntt_product(a, b, q, psi):
    """psi-twisted NTT: evaluate at the n odd powers psi^(2i+1) (roots of x^n+1),
    multiply pointwise, interpolate back (n a power of 2, q prime, 2n | q-1)."""
    n = len(a)
    w = psi * psi % q
    ta = [int(v) * pow(psi, i, q) % q for i, v in enumerate(a)]
    tb = [int(v) * pow(psi, i, q) % q for i, v in enumerate(b)]
    fa, fb = _fft(ta, w, q), _fft(tb, w, q)
    fc = [x * y % q for x, y in zip(fa, fb)]
    winv = pow(w, q - 2, q)
    ninv = pow(n, q - 2, q)
    tc = _fft(fc, winv, q)
    psiinv = pow(psi, q - 2, q)
    return [v * ninv % q * pow(psiinv, i, q) % q for i, v in enumerate(tc)]


def poly_eval(c, x, q):
    acc = 0
    for v in reversed(c):
        acc = (acc * x + int(v)) % q
    return acc


def eq3_matrix(b, n):
    """The Eq. (3) matrix: row 0 is (b_0, ..., b_{n-1}); each following row is the
    previous one shifted right by one place with the entry that wraps round into
    column 0 negated."""
    rows = [list(int(v) for v in b)]
    for _ in range(1, n):
        prev = rows[-1]
        rows.append([-prev[-1]] + prev[:-1])
    return rows


def vec_mat(v, M):
    n = len(M[0])
    return [sum(int(v[i]) * M[i][j] for i in range(len(v))) for j in range(n)]


# ------------------------------------------------------------------ checks
def _dtype(q):
    return np.uint64 if q >= (1 << 32) else np.uint32


def _rand(rng, shape, q):
    return np.array([[rng.randrange(q) for _ in range(shape[1])] for _ in range(shape[0])], dtype=object).astype(_dtype(q))


def check_minus_one(impl, n, q):
    """x^(n-1) * x = x^n = -1."""
    a = np.zeros((1, n), dtype=_dtype(q))
    b = np.zeros((1, n), dtype=_dtype(q))
    a[0, n - 1] = 1
    b[0, 1] = 1
    c = impl(a, b, q)
    want = np.zeros(n, dtype=object)
    want[0] = q - 1
    assert [int(v) for v in c[0]] == [int(v) for v in want], "x^n != -1"


def check_rotation(impl, n, q, rng, ks):
    """x^k * a(x) is the signed (negacyclic) rotation of a by k places."""
    a = _rand(rng, (len(ks), n), q)
    b = np.zeros((len(ks), n), dtype=_dtype(q))
    for r, k in enumerate(ks):
        b[r, k] = 1
    c = impl(a, b, q)
    for r, k in enumerate(ks):
        al = [int(v) for v in a[r]]
        want = [al[j - k] if j >= k else (q - al[n + j - k]) % q for j in range(n)]
        assert [int(v) for v in c[r]] == want, f"rotation by x^{k} wrong"


def check_ring_axioms(impl, n, q, rng, batch=3):
    a, b, d = (_rand(rng, (batch, n), q) for _ in range(3))
    ab, ba = impl(a, b, q), impl(b, a, q)
    assert np.array_equal(ab, ba), "not commutative"
    one = np.zeros((batch, n), dtype=_dtype(q))
    one[:, 0] = 1
    assert np.array_equal(impl(a, one, q), a), "1 is not the identity"
    zero = np.zeros((batch, n), dtype=_dtype(q))
    assert not impl(a, zero, q).any(), "a*0 != 0"
    bd = np.array([[(int(x) + int(y)) % q for x, y in zip(r1, r2)] for r1, r2 in zip(b, d)], dtype=object).astype(_dtype(q))
    lhs = impl(a, bd, q)
    ad = impl(a, d, q)
    rhs = np.array([[(int(x) + int(y)) % q for x, y in zip(r1, r2)] for r1, r2 in zip(ab, ad)], dtype=object).astype(_dtype(q))
    assert np.array_equal(lhs, rhs), "not distributive"
    neg_a = np.array([[(q - int(x)) % q for x in r] for r in a], dtype=object).astype(_dtype(q))
    neg_ab = np.array([[(q - int(x)) % q for x in r] for r in ab], dtype=object).astype(_dtype(q))
    assert np.array_equal(impl(neg_a, b, q), neg_ab), "(-a)b != -(ab)"


def check_kronecker(impl, n, q, rng, batch=2):
    a, b = _rand(rng, (batch, n), q), _rand(rng, (batch, n), q)
    c = impl(a, b, q)
    for r in range(batch):
        want = kronecker_product([int(v) for v in a[r]], [int(v) for v in b[r]], q)
        assert [int(v) for v in c[r]] == want, "differs from Kronecker substitution"


def check_ntt(impl, n, q, rng, batch=2):
    psi = find_psi(q, n, rng)
    a, b = _rand(rng, (batch, n), q), _rand(rng, (batch, n), q)
    c = impl(a, b, q)
    for r in range(batch):
        want = ntt_product([int(v) for v in a[r]], [int(v) for v in b[r]], q, psi)
        assert [int(v) for v in c[r]] == want, "differs from the NTT product"


def check_bruteforce(impl, n, q):
    """Every pair (a, b) in Z_q^n x Z_q^n against Z[x] product + long division."""
    import itertools
    vecs = list(itertools.product(range(q), repeat=n))
    A = np.array([v for v in vecs for _ in vecs], dtype=_dtype(q)).reshape(-1, n)
    B = np.array([w for _ in vecs for w in vecs], dtype=_dtype(q)).reshape(-1, n)
    C = impl(A, B, q)
    mod = negacyclic_modulus(n)
    for r in range(A.shape[0]):
        want = [v % q for v in poly_rem_monic(zpoly_mul(list(A[r].astype(int)), list(B[r].astype(int))), mod)]
        assert [int(v) for v in C[r]] == want, f"brute force mismatch at a={A[r]}, b={B[r]}"


def check_eq3_and_fig1(impl, n, q, rng):
    """Eq. (3): c = a x M(b); Fig. 1: the half-size split reproduces it."""
    a, b = _rand(rng, (1, n), q), _rand(rng, (1, n), q)
    c = [int(v) for v in impl(a, b, q)[0]]
    M = eq3_matrix([int(v) for v in b[0]], n)
    assert [v % q for v in vec_mat([int(v) for v in a[0]], M)] == c, "differs from the Eq. (3) matrix product"
    h = n // 2
    V1, V2 = [int(v) for v in a[0, :h]], [int(v) for v in a[0, h:]]
    MA = [row[:h] for row in M[:h]]
    MB = [row[h:] for row in M[:h]]
    MC = [row[:h] for row in M[h:]]
    MD = [row[h:] for row in M[h:]]
    r1 = [x + y for x, y in zip(vec_mat(V1, MA), vec_mat(V2, MC))]
    r2 = [x + y for x, y in zip(vec_mat(V1, MB), vec_mat(V2, MD))]
    assert [v % q for v in r1 + r2] == c, "Fig. 1 split differs"


ALL_CHECK_NAMES = ("minus_one", "rotation", "ring_axioms", "kronecker", "ntt", "bruteforce", "eq3_fig1")


def run_all(impl, rng=None):
    """Run every check at small sizes; returns the names of the failing checks."""
    rng = rng or random.Random(12345)
    failures = []
    q_ntt = 7681  # prime, 7681 = 1 + 15*512
    cases = [
        ("minus_one", lambda: [check_minus_one(impl, n, q) for n in (2, 8, 16) for q in (17, 3329)]),
        ("rotation", lambda: check_rotation(impl, 16, 3329, rng, [0, 1, 5, 15])),
        ("ring_axioms", lambda: check_ring_axioms(impl, 8, 97, rng)),
        ("kronecker", lambda: [check_kronecker(impl, n, 3329, rng) for n in (4, 16)]),
        ("ntt", lambda: check_ntt(impl, 16, q_ntt, rng)),
        ("bruteforce", lambda: check_bruteforce(impl, 2, 3)),
        ("eq3_fig1", lambda: check_eq3_and_fig1(impl, 8, 3329, rng)),
    ]
    for name, fn in cases:
        try:
            fn()
        except AssertionError:
            failures.append(name)
    return failures
